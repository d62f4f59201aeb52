// Internal state of a batch handle (nvd_batch), shared by the persistent
// solver (batch.hip) and the sweep solver (batch_sweep.hip).
#pragma once

#include <string>
#include <vector>

#include "nvd_internal.hpp"

namespace nvd {
struct BGraph;
}

struct nvd_batch {
  int G = 0;
  std::vector<int> n, nnz, weighted;
  std::vector<long> rp_off, nnz_off, node_off;
  std::vector<int> long_off, n_long;
  long tot_n = 0, tot_rp = 0, tot_nnz = 0, tot_long = 0;
  bool any_weighted = false;
  // device graph data
  int* rp = nullptr;
  int* ci = nullptr;
  double* w64 = nullptr;
  float* w32 = nullptr;
  double* invd64 = nullptr;
  float* invd32 = nullptr;
  int* long_rows = nullptr;
  // workspace (grown on demand)
  int cap_T = 0;
  double *b64 = nullptr, *x64 = nullptr, *r64 = nullptr;
  void *cv = nullptr, *rv = nullptr, *pv = nullptr, *qv = nullptr;
  int cap_vsize = 0;   // element size of cv..qv
  nvd::BGraph* gd = nullptr;
  int* plan_buf = nullptr;
  int plan_cap = 0;
  unsigned* ctr = nullptr;
  unsigned* pool_next = nullptr;
  int* err = nullptr;
  int* h_err = nullptr;
  double* part = nullptr;
  nvd_pair_info* info = nullptr;
  int info_cap = 0;
  int64_t bytes = 0;
  // captured launch (reset + persistent kernel), replayed while the call's
  // arguments are unchanged
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<long> key;
  bool capture_failed = false;
  int64_t replays = 0;
  int64_t captures = 0;
  int64_t eager = 0;
  // CG iterations per graph measured on the previous call (work plan weights)
  std::vector<double> it_est;
  // optional per-graph timing of the last call (NVD_BATCH_TRACE=1)
  unsigned long long* trace = nullptr;
  std::vector<int> last_team_size;
  // sweep solver: chunk table (built on first use) and its workspace
  std::vector<int> h_long_rows;        // long rows of all graphs (local ids, at long_off)
  int n_chunks = 0;
  int* ch_buf = nullptr;               // [3][n_chunks]: graph, first row, end row (-1: one long row)
  std::vector<int> ch_first, ch_nshort, ch_nlong;   // per graph
  std::vector<int> ch_xcd;             // XCD of each graph in the current table
  int xfirst[8] = {}, xcount[8] = {};  // chunk range of each XCD
  void* sg_dev = nullptr;              // per-graph descriptors of the sweep kernels
  double* spart = nullptr;             // per-chunk partial sums
  size_t spart_cap = 0;
  char* sstate = nullptr;              // per (graph, column) solver state
  size_t sstate_cap = 0;
  int* h_poll = nullptr;               // pinned host words for polling
  int64_t sweeps = 0;
  // sweep solver: a chunk of inner iterations (apply, update, direction
  // kernels) captured in a hipGraph, replayed while its arguments match
  hipGraph_t sw_graph = nullptr;
  hipGraphExec_t sw_exec = nullptr;
  std::vector<unsigned char> sw_key;
  bool sw_capture_failed = false;
};

static void batch_drop_graph(nvd_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->gexec = nullptr;
  b->graph = nullptr;
  b->key.clear();
}

static void batch_drop_sweep_graph(nvd_batch* b) {
  if (b->sw_exec) (void)hipGraphExecDestroy(b->sw_exec);
  if (b->sw_graph) (void)hipGraphDestroy(b->sw_graph);
  b->sw_exec = nullptr;
  b->sw_graph = nullptr;
  b->sw_key.clear();
}

static inline void batch_free(nvd_batch* b) {
  batch_drop_graph(b);
  batch_drop_sweep_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  void* ptrs[] = {b->rp, b->ci, b->w64, b->w32, b->invd64, b->invd32,
                  b->long_rows, b->b64, b->x64, b->r64, b->cv, b->rv, b->pv, b->qv, b->gd,
                  b->plan_buf, b->ctr, b->pool_next, b->err, b->part, b->info, b->trace,
                  b->ch_buf, b->sg_dev, b->spart, b->sstate};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (b->h_err) (void)hipHostFree(b->h_err);
  if (b->h_poll) (void)hipHostFree(b->h_poll);
}

template <typename T>
static nvd_status balloc(nvd_batch* b, T** p, size_t count) {
  if (count == 0) count = 1;
  NVD_HIP(hipMalloc((void**)p, count * sizeof(T)));
  b->bytes += (int64_t)(count * sizeof(T));
  return NVD_OK;
}


namespace nvd {
// Sweep solver: all graphs of the batch as one block-diagonal operator,
// swept by the whole GPU kernel by kernel (batch_sweep.hip).
nvd_status run_sweep(nvd_batch* b, const std::vector<int>& ks, int T, const nvd_opts& o,
                     const double* P, const double* Q, double* d_out, double* X,
                     nvd_pair_info* info_host, hipStream_t s);
}  // namespace nvd
