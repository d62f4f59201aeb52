// Batches of graphs (placeholder until the persistent batched solver lands).
#include "device_common.hpp"

struct nvd_batch {
  int G;
};

extern "C" {
nvd_status nvd_batch_create(int32_t G, nvd_graph* const* graphs, void* stream, nvd_batch** out) {
  (void)G; (void)graphs; (void)stream;
  if (out) *out = nullptr;
  nvd::set_error("nvd_batch_create: not available in this build");
  return NVD_E_UNSUPPORTED;
}
nvd_status nvd_batch_destroy(nvd_batch* b) {
  delete b;
  return NVD_OK;
}
nvd_status nvd_batch_distances(nvd_batch* b, const int32_t* k_per_graph, const double* P,
                               const double* Q, const nvd_opts* opts, double* d_out,
                               double* X_out, nvd_pair_info* info, void* stream) {
  (void)b; (void)k_per_graph; (void)P; (void)Q; (void)opts; (void)d_out; (void)X_out; (void)info; (void)stream;
  nvd::set_error("nvd_batch_distances: not available in this build");
  return NVD_E_UNSUPPORTED;
}
}
