// Optional launch timing: when enabled, the solver brackets each launch of
// the kernels it classifies (SpMM, CG update, CG direction; FP64 / FP32)
// with HIP events on the launch stream and records the algorithmic bytes
// of that launch.  nvd_prof_read sums elapsed time per class.
#include <vector>

#include "device_common.hpp"
#include "prof.hpp"

namespace nvd {

namespace {
struct Rec {
  hipEvent_t a = nullptr, b = nullptr;
  int kind = 0;
  double bytes = 0.0;
  bool idle = false;
};
std::vector<Rec> g_recs;
size_t g_used = 0;
bool g_on = false;
int g_last = -1;
}  // namespace

bool prof_enabled() { return g_on; }

int prof_begin(hipStream_t s, int kind, double bytes) {
  if (!g_on) return -1;
  if (g_used == g_recs.size()) {
    Rec r;
    if (hipEventCreate(&r.a) != hipSuccess || hipEventCreate(&r.b) != hipSuccess) return -1;
    g_recs.push_back(r);
  }
  Rec& r = g_recs[g_used];
  r.kind = kind;
  r.bytes = bytes;
  r.idle = false;
  if (hipEventRecord(r.a, s) != hipSuccess) return -1;
  g_last = (int)g_used;
  return (int)g_used++;
}

int prof_last_id() { return g_on ? g_last : -1; }

void prof_mark_idle(int id) {
  if (id >= 0 && (size_t)id < g_used) g_recs[id].idle = true;
}

void prof_end(hipStream_t s, int id) {
  if (id < 0) return;
  (void)hipEventRecord(g_recs[id].b, s);
}

}  // namespace nvd

extern "C" {

nvd_status nvd_prof_enable(int32_t on) {
  nvd::g_on = on != 0;
  nvd::g_used = 0;
  return NVD_OK;
}

nvd_status nvd_prof_read(double* ms, int64_t* launches, double* bytes) {
  using namespace nvd;
  if (!ms || !launches || !bytes) {
    set_error("nvd_prof_read: NULL argument");
    return NVD_E_ARG;
  }
  for (int k = 0; k < NVD_PROF_KINDS; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
    bytes[k] = 0.0;
  }
  for (size_t i = 0; i < g_used; ++i) {
    Rec& r = g_recs[i];
    if (r.idle) continue;
    NVD_HIP(hipEventSynchronize(r.b));
    float t = 0.0f;
    NVD_HIP(hipEventElapsedTime(&t, r.a, r.b));
    ms[r.kind] += t;
    launches[r.kind] += 1;
    bytes[r.kind] += r.bytes;
  }
  g_used = 0;
  return NVD_OK;
}

}  // extern "C"
