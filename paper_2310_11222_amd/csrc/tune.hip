// Autotuner for the tile: the number of right-hand-side columns per solve
// pass (T) and the neighbour lanes per row of the Laplacian apply (NL).
//
// Wider tiles read the CSR fewer times and gather longer rows of X per
// neighbour (fewer, fuller memory transactions); narrower tiles keep the
// solver's vectors small enough to stay in the last-level cache, which the
// vector passes of every iteration (update, direction) feel as much as the
// apply.  Which wins depends on the graph, so the candidates are timed on the
// graph itself: for each T the apply alone picks NL, then one whole CG
// iteration (apply, update, direction) with that NL is timed, and the T
// minimising the time for all k columns, ceil(k / T) * t_iter(T), is cached in
// the graph handle per (precision, k bucket).
#include <algorithm>
#include <cstdlib>

#include "device_common.hpp"

namespace nvd {

static int log2i(int v) {
  int l = 0;
  while ((1 << (l + 1)) <= v) ++l;
  return l;
}

static bool tuning_disabled() {
  const char* e = std::getenv("NVD_TUNE");
  return e && e[0] == '0';
}

// Heuristic used when tuning is off: the largest power of two <= min(k, 32).
static int heuristic_tile(int k) {
  int T = 1;
  while (T * 2 <= k && T * 2 <= 32) T *= 2;
  return T;
}

static nvd_status time_spmm(DevGraph* g, int prec, int T, int nl, hipStream_t s, float* ms) {
  Workspace* ws = g->ws;
  SpmmCall sc{};
  sc.g = g;
  sc.prec = prec;
  sc.T = T;
  sc.nl = nl;
  sc.x = prec == 0 ? (const void*)ws->p64 : (const void*)ws->p32;
  sc.ldx = T;
  sc.y = prec == 0 ? (void*)ws->q64 : (void*)ws->q32;
  sc.ldy = T;
  sc.epi = EPI_PLAIN;
  hipEvent_t a, b;
  NVD_HIP(hipEventCreate(&a));
  NVD_HIP(hipEventCreate(&b));
  nvd_status st = launch_spmm(sc, ws->red, s);   // warm-up
  const int reps = 3;
  if (st == NVD_OK) st = hipEventRecord(a, s) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
  for (int i = 0; i < reps && st == NVD_OK; ++i) st = launch_spmm(sc, ws->red, s);
  if (st == NVD_OK) st = hipEventRecord(b, s) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
  if (st == NVD_OK) st = hipEventSynchronize(b) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
  float t = 0.0f;
  if (st == NVD_OK) st = hipEventElapsedTime(&t, a, b) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *ms = t / reps;
  if (st != NVD_OK) set_error("autotuner: timing failed");
  return st;
}

int tuned_nl(const DevGraph* g, int precision, int T) {
  const int p = precision == NVD_MIXED ? 1 : 0;
  const int nl = g->tuned_nl[p][log2i(T)];
  return nl > 0 ? nl : default_nl(T);
}

int untimed_tile(const DevGraph* g, int k, int precision) {
  if (k <= 8 || g->n < 4096) return heuristic_tile(k);
  const int p = precision == NVD_MIXED ? 1 : 0;
  const int t = g->tuned_tile[p][std::min(log2i(k), 7)];
  return t > 0 ? t : heuristic_tile(k);
}

int choose_tile(DevGraph* g, int k, int precision, hipStream_t s) {
  if (k <= 8 || g->n < 4096 || tuning_disabled()) return heuristic_tile(k);
  const int p = precision == NVD_MIXED ? 1 : 0;
  const int kb = std::min(log2i(k), 7);
  if (g->tuned_tile[p][kb] > 0) return g->tuned_tile[p][kb];
  // the SpMM of the inner solver dominates: FP32 for MIXED, FP64 otherwise
  const int prec = p;
  int tmax = 1;
  while (tmax * 2 <= k && tmax * 2 <= kMaxTile) tmax *= 2;
  if (ensure_workspace(g, tmax, prec == 1) != NVD_OK) return heuristic_tile(k);
  double best = 1e30;
  int bestT = heuristic_tile(k);
  for (int T = 8; T <= tmax; T *= 2) {
    float best_apply = 1e30f;
    int nlT = default_nl(T);
    for (int nl = 1; nl <= spmm_max_nl(prec, T); nl *= 2) {
      float ms = 0.0f;
      if (time_spmm(g, prec, T, nl, s, &ms) != NVD_OK) return heuristic_tile(k);
      if (ms < best_apply) {
        best_apply = ms;
        nlT = nl;
      }
    }
    g->tuned_nl[p][log2i(T)] = nlT;
    float it_ms = 0.0f;
    if (time_cg_iteration(g, prec, T, nlT, s, &it_ms) != NVD_OK) return heuristic_tile(k);
    const double total = (double)((k + T - 1) / T) * it_ms;
    if (total < best) {
      best = total;
      bestT = T;
    }
  }
  g->tuned_tile[p][kb] = bestT;
  return bestT;
}

}  // namespace nvd

extern "C" nvd_status nvd_tune_query(nvd_graph* h, int32_t k, int32_t precision, int32_t* tile,
                                     int32_t* nl, void* stream) {
  using namespace nvd;
  if (!h || !tile || !nl || k < 1 || (precision != NVD_FP64 && precision != NVD_MIXED)) {
    set_error("nvd_tune_query: bad argument");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  *tile = choose_tile(g, k, precision, reinterpret_cast<hipStream_t>(stream));
  *nl = tuned_nl(g, precision, *tile);
  return NVD_OK;
}
