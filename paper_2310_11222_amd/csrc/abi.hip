// The extern "C" entry points declared in include/nvd.h: argument checks,
// tiling of the k pairs, and the edge-weight adjoint kernel.
#include <algorithm>
#include <climits>
#include <cmath>
#include <vector>

#include "device_common.hpp"

namespace nvd {

nvd_status graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* w, hipStream_t s, DevGraph** out);
nvd_status graph_destroy(DevGraph* g);

// Edge-weight adjoint: one thread per (row, column) pair of a tile is too
// fine for short rows, so a group of T lanes takes one row and walks its
// neighbours; each CSR entry's value is the sum over the tile's columns,
// reduced across the T lanes by shuffles.
template <int T>
__global__ __launch_bounds__(kBS) void k_grad_w(int n, const int* rp, const int* ci,
                                                const int* in_pos, const double* X, long ldx,
                                                const double* gs, double* gw, int accumulate) {
  constexpr int RW = 64 / T;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int c = lane % T;
  const int g = lane / T;
  const double gc = gs[c];
  const long rows_per_step = (long)gridDim.x * (kBS / 64) * RW;
  for (long row = (long)blockIdx.x * (kBS / 64) * RW + (t >> 6) * RW + g; row < n;
       row += rows_per_step) {
    const double xi = X[row * ldx + c];
    const int lo = rp[row], hi = rp[row + 1];
    for (int e = lo; e < hi; ++e) {
      const double df = xi - X[(long)ci[e] * ldx + c];
      double v = -0.5 * gc * df * df;
#pragma unroll
      for (int off = 1; off < T; off <<= 1) v += __shfl_xor(v, off, 64);
      if (c == 0) {
        const long pos = in_pos ? in_pos[e] : e;
        gw[pos] = accumulate ? gw[pos] + v : v;
      }
    }
  }
}

// Adjoint with respect to the node vectors: d(sum_j g_j d_j^2)/dP = 2 X
// diag(g) and d/dQ its negative (x_j = L^+ delta_j is the saved solution;
// L^+ is symmetric, so no second solve is needed).  Either output may be null.
__global__ __launch_bounds__(kBS) void k_grad_vec(int n, int k, const double* __restrict__ X,
                                                  long ldx, const double* __restrict__ gs,
                                                  double* __restrict__ GP, long ldp,
                                                  double* __restrict__ GQ, long ldq) {
  const long tot = (long)n * k;
  for (long e = (long)blockIdx.x * kBS + threadIdx.x; e < tot; e += (long)gridDim.x * kBS) {
    const long i = e / k;
    const int c = (int)(e % k);
    const double v = 2.0 * gs[c] * X[i * ldx + c];
    if (GP) GP[i * ldp + c] = v;
    if (GQ) GQ[i * ldq + c] = -v;
  }
}

// Upstream gradient on d turned into the scale on d^2: dd/d(d^2) = 1/(2d),
// defined as 0 where d = 0 (d is not differentiable there; the zero vector
// is the minimum-norm subgradient).
__global__ void k_grad_scale_d(int k, const double* __restrict__ g, const double* __restrict__ d,
                               double* __restrict__ gs) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double dj = d[j];
  gs[j] = dj > 0.0 ? g[j] / (2.0 * dj) : 0.0;
}

// New edge weights from a device array in the input CSR order, checked
// before anything is replaced: every value finite and > 0 and equal to its
// mirror entry's.  flag bit 1: bad value, bit 2: asymmetric.
__global__ void k_check_weights(int n, const int* rp, const int* ci, const int* in_pos,
                                const double* w_in, int* flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int e = rp[i]; e < rp[i + 1]; ++e) {
    const double v = w_in[in_pos ? in_pos[e] : e];
    if (!(v > 0.0) || !isfinite(v)) atomicOr(flag, 1);
    const int j = ci[e];
    int lo = rp[j], hi = rp[j + 1];
    while (lo < hi) {                  // mirror entry (j, i)
      const int mid = (lo + hi) >> 1;
      if (ci[mid] < i)
        lo = mid + 1;
      else
        hi = mid;
    }
    if (lo >= rp[j + 1] || ci[lo] != i || w_in[in_pos ? in_pos[lo] : lo] != v) atomicOr(flag, 2);
  }
}

// Commit checked weights: every internal entry takes its input value.
__global__ void k_set_weights(int nnz, const int* in_pos, const double* w_in, double* w64,
                              float* w32) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnz) return;
  const double v = w_in[in_pos ? in_pos[e] : e];
  w64[e] = v;
  w32[e] = (float)v;
}

__global__ void k_degree_refresh(int n, const int* rp, const double* w64, double* deg64,
                                 float* deg32, double* invd64, float* invd32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = rp[i]; e < rp[i + 1]; ++e) d += w64[e];
  deg64[i] = d;
  deg32[i] = (float)d;
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  invd64[i] = inv;
  invd32[i] = (float)inv;
}

// Solver options: precision, tolerances, limits and tile.
nvd_status check_solve_opts(const nvd_opts* o) {
  if (o->precision != NVD_FP64 && o->precision != NVD_MIXED) {
    set_error("nvd_opts.precision must be NVD_FP64 or NVD_MIXED");
    return NVD_E_ARG;
  }
  if (!(o->rtol > 0.0) || !(o->rtol < 1.0) || !(o->inner_rtol > 0.0) || !(o->inner_rtol < 1.0)) {
    set_error("nvd_opts: rtol and inner_rtol must lie in (0, 1)");
    return NVD_E_ARG;
  }
  if ((o->flags & NVD_PRECOND_ACHOL) && (o->flags & (NVD_PRECOND_TREE | NVD_PRECOND_AUTO))) {
    set_error("nvd_opts: NVD_PRECOND_ACHOL excludes NVD_PRECOND_TREE and NVD_PRECOND_AUTO");
    return NVD_E_ARG;
  }
  if (o->max_iter < 1 || o->max_refine < 1) {
    set_error("nvd_opts: max_iter and max_refine must be >= 1");
    return NVD_E_ARG;
  }
  const int t = o->tile_k;
  if (t != 0 && t != 1 && t != 2 && t != 4 && t != 8 && t != 16 && t != 32 && t != 64) {
    set_error("nvd_opts.tile_k must be 0 or a power of two up to 64");
    return NVD_E_ARG;
  }
  return NVD_OK;
}

}  // namespace nvd

using namespace nvd;

struct nvd_batch;   // defined in batch.hip

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

extern "C" {

int32_t nvd_abi_version(void) { return NVD_ABI_VERSION; }

const char* nvd_status_string(int32_t s) {
  switch (s) {
    case NVD_OK: return "ok";
    case NVD_E_ARG: return "invalid argument";
    case NVD_E_GRAPH: return "invalid graph";
    case NVD_E_VALUE: return "non-finite value in input";
    case NVD_E_NOCONV: return "did not converge";
    case NVD_E_BREAKDOWN: return "solver breakdown";
    case NVD_E_DEVICE: return "device error";
    case NVD_E_NOMEM: return "out of device memory";
    case NVD_E_UNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* nvd_last_error(void) { return get_error(); }

nvd_status nvd_opts_default(nvd_opts* o) {
  if (!o) {
    set_error("nvd_opts_default: NULL");
    return NVD_E_ARG;
  }
  o->precision = NVD_FP64;
  o->rtol = 1e-10;
  o->inner_rtol = 1e-5;
  o->max_iter = 20000;
  o->max_refine = 30;
  o->tile_k = 0;
  o->flags = 0;
  return NVD_OK;
}

nvd_status nvd_graph_create_ex(int64_t n, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col_idx, const double* weights, uint32_t flags,
                               void* stream, nvd_graph** out) {
  set_error("");
  if (!out) {
    set_error("nvd_graph_create: out is NULL");
    return NVD_E_ARG;
  }
  *out = nullptr;
  if (flags & ~(uint32_t)NVD_PTR_DEVICE) {
    set_error("nvd_graph_create_ex: unknown flag");
    return NVD_E_ARG;
  }
  DevGraph* g = nullptr;
  if (flags & NVD_PTR_DEVICE) {
    // device arrays: staged to the host, where validation and set-up run
    if (n < 1 || nnz < 0 || n >= INT32_MAX || nnz >= INT32_MAX || !row_ptr || (nnz > 0 && !col_idx)) {
      set_error("nvd_graph_create_ex: need 1 <= n < 2^31, 0 <= nnz < 2^31 and non-NULL arrays");
      return NVD_E_ARG;
    }
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> ci(std::max<int64_t>(nnz, 1));
    std::vector<double> w(weights ? std::max<int64_t>(nnz, 1) : 0);
    hipStream_t s = as_stream(stream);
    NVD_HIP(hipStreamSynchronize(s));
    NVD_HIP(hipMemcpy(rp.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
    if (nnz > 0) NVD_HIP(hipMemcpy(ci.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    if (weights && nnz > 0)
      NVD_HIP(hipMemcpy(w.data(), weights, sizeof(double) * nnz, hipMemcpyDeviceToHost));
    NVD_TRY(graph_create(n, nnz, rp.data(), ci.data(), weights ? w.data() : nullptr, s, &g));
  } else {
    NVD_TRY(graph_create(n, nnz, row_ptr, col_idx, weights, as_stream(stream), &g));
  }
  *out = new nvd_graph{g};
  return NVD_OK;
}

nvd_status nvd_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, const double* weights, void* stream,
                            nvd_graph** out) {
  return nvd_graph_create_ex(n, nnz, row_ptr, col_idx, weights, NVD_PTR_HOST, stream, out);
}

nvd_status nvd_graph_destroy(nvd_graph* g) {
  if (!g) return NVD_OK;
  graph_destroy(g->g);
  delete g;
  return NVD_OK;
}

nvd_status nvd_graph_stats(const nvd_graph* h, nvd_stats* s) {
  if (!h || !s) {
    set_error("nvd_graph_stats: NULL argument");
    return NVD_E_ARG;
  }
  const DevGraph* g = h->g;
  s->n = g->n;
  s->nnz = g->nnz;
  s->n_comp = g->n_comp;
  s->n_isolated = g->n_isolated;
  s->max_deg = g->max_deg;
  s->n_long_rows = g->n_long_rows;
  s->device_bytes = g->bytes;
  s->weighted = g->weighted ? 1 : 0;
  s->self_loops_dropped = g->self_loops;
  s->achol_rounds = g->achol ? g->achol->rounds : 0;
  s->achol_factor_nnz = g->achol ? g->achol->nnz : 0;
  s->achol_remainder = g->achol ? g->achol->remainder : 0;
  return NVD_OK;
}

nvd_status nvd_graph_query(const nvd_graph* h, int32_t* labels, double* degree) {
  if (!h) {
    set_error("nvd_graph_query: NULL graph");
    return NVD_E_ARG;
  }
  const DevGraph* g = h->g;
  if (labels) std::copy(g->h_comp.begin(), g->h_comp.end(), labels);
  if (degree) NVD_HIP(hipMemcpy(degree, g->deg64, sizeof(double) * g->n, hipMemcpyDeviceToHost));
  return NVD_OK;
}

nvd_status nvd_laplacian_apply(nvd_graph* h, int32_t dtype, int32_t k, const void* X,
                               int64_t ldx, void* Y, int64_t ldy, void* stream) {
  set_error("");
  if (!h || !X || !Y || k < 1 || ldx < k || ldy < k) {
    set_error("nvd_laplacian_apply: bad argument (NULL pointer, k < 1 or ld < k)");
    return NVD_E_ARG;
  }
  if (dtype != NVD_DT_F64 && dtype != NVD_DT_F32) {
    set_error("nvd_laplacian_apply: dtype must be NVD_DT_F64 or NVD_DT_F32");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  NVD_TRY(ensure_workspace(g, 1, false));
  const size_t es = dtype == NVD_DT_F64 ? 8 : 4;
  for (int c0 = 0; c0 < k;) {
    int T = 64;
    while (T > k - c0) T >>= 1;
    SpmmCall sc{};
    sc.g = g;
    sc.prec = dtype == NVD_DT_F64 ? 0 : 1;
    sc.T = T;
    sc.x = static_cast<const char*>(X) + c0 * es;
    sc.ldx = ldx;
    sc.y = static_cast<char*>(Y) + c0 * es;
    sc.ldy = ldy;
    sc.epi = EPI_PLAIN;
    NVD_TRY(launch_apply(sc, g->ws->red, as_stream(stream)));
    c0 += T;
  }
  return NVD_OK;
}

nvd_status nvd_project(nvd_graph* h, int32_t k, const double* P, const double* Q, int64_t ld,
                       double* Dbar, int64_t ldd, double* norms, void* stream) {
  set_error("");
  if (!h || !P || !Q || !Dbar || k < 1 || ld < k || ldd < k) {
    set_error("nvd_project: bad argument (NULL pointer, k < 1 or ld < k)");
    return NVD_E_ARG;
  }
  for (int c0 = 0; c0 < k;) {
    int T = 64;
    while (T > k - c0) T >>= 1;
    NVD_TRY(project_tile(h->g, T, P + c0, Q + c0, ld, Dbar + c0, ldd, norms ? norms + c0 : nullptr,
                         as_stream(stream)));
    c0 += T;
  }
  return NVD_OK;
}


nvd_status nvd_distances(nvd_graph* h, int32_t k, const double* P, const double* Q, int64_t ld,
                         const nvd_opts* opts, double* d_out, double* X, int64_t ldx,
                         nvd_pair_info* info, void* stream) {
  set_error("");
  if (!h || !P || !Q || !d_out || k < 1 || ld < k || (X && ldx < k)) {
    set_error("nvd_distances: bad argument (NULL pointer, k < 1 or ld < k)");
    return NVD_E_ARG;
  }
  nvd_opts o;
  nvd_opts_default(&o);
  if (opts) o = *opts;
  NVD_TRY(check_solve_opts(&o));
  if ((o.flags & NVD_WARM_START) && !X) {
    set_error("nvd_distances: NVD_WARM_START needs X_inout");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  hipStream_t s = as_stream(stream);
  SolveParams sp{};
  sp.precision = o.precision;
  sp.rtol = o.rtol;
  sp.inner_rtol = o.inner_rtol;
  sp.max_iter = o.max_iter;
  sp.max_refine = o.max_refine;
  sp.warm = (o.flags & NVD_WARM_START) != 0;
  sp.achol = (o.flags & NVD_PRECOND_ACHOL) != 0;
  sp.tree = sp.achol || use_tree(g, o.flags);
  sp.out_dsq = (o.flags & NVD_OUT_DSQ) != 0;
  int tile = o.tile_k;
  if (tile == 0) tile = choose_tile(g, k, o.precision, s);
  std::vector<nvd_pair_info> hinfo(k);
  nvd_status agg = NVD_OK;
  nvd_status st = NVD_OK;
  for (int c0 = 0; c0 < k && st == NVD_OK;) {
    int T = tile;
    while (T > k - c0) T >>= 1;
    sp.nl = tuned_nl(g, o.precision, T);
    st = ensure_workspace(g, T, o.precision == NVD_MIXED);
    const int nb = st == NVD_OK ? small_blocks(g, T, sp) : 0;
    bool done = false;
    if (st == NVD_OK && nb > 0) {
      st = solve_small(g, T, nb, P + c0, Q + c0, ld, sp, d_out + c0, X ? X + c0 : nullptr, ldx,
                       g->ws->info, s);
      done = st != NVD_E_UNSUPPORTED;   // a launch too large for the device: multi-kernel path
      if (!done) {
        st = NVD_OK;
        set_error("");
      }
    }
    if (st == NVD_OK && !done)
      st = solve_tile(g, T, P + c0, Q + c0, ld, sp, d_out + c0, X ? X + c0 : nullptr, ldx,
                      g->ws->info, s);
    if (st == NVD_OK) {
      hipError_t e = hipMemcpyAsync(hinfo.data() + c0, g->ws->info, sizeof(nvd_pair_info) * T,
                                    hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        set_error(std::string("nvd_distances: ") + hipGetErrorString(e));
        st = NVD_E_DEVICE;
      }
    }
    c0 += T;
  }
  if (st != NVD_OK) return st;
  for (int j = 0; j < k; ++j) {
    if (hinfo[j].status == NVD_E_DEVICE) {
      if (info) std::copy(hinfo.begin(), hinfo.end(), info);
      set_error("nvd_distances: a grid barrier of the single-launch solve gave up");
      return NVD_E_DEVICE;
    }
    if (hinfo[j].status == NVD_E_BREAKDOWN) agg = NVD_E_BREAKDOWN;
    else if (hinfo[j].status == NVD_E_NOCONV && agg == NVD_OK) agg = NVD_E_NOCONV;
  }
  if (info) std::copy(hinfo.begin(), hinfo.end(), info);
  if (agg != NVD_OK) set_error("nvd_distances: some pairs did not converge (see info)");
  return agg;
}

nvd_status nvd_graph_set_weights(nvd_graph* h, const double* w, void* stream) {
  set_error("");
  if (!h || !w) {
    set_error("nvd_graph_set_weights: NULL argument");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  hipStream_t s = as_stream(stream);
  // 1. check the new values; the graph is left untouched if they are rejected
  int* flag = nullptr;
  NVD_HIP(hipMalloc((void**)&flag, sizeof(int)));
  int hflag = 0;
  hipError_t e = hipMemcpyAsync(flag, &hflag, sizeof(int), hipMemcpyHostToDevice, s);
  const int grid = (g->n + 255) / 256;
  if (e == hipSuccess) {
    k_check_weights<<<grid, 256, 0, s>>>(g->n, g->rp, g->ci, g->in_pos, w, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(flag);
  if (e != hipSuccess) {
    set_error(std::string("nvd_graph_set_weights: ") + hipGetErrorString(e));
    return NVD_E_DEVICE;
  }
  if (hflag) {
    set_error(std::string("nvd_graph_set_weights: ") +
              ((hflag & 1) ? "a weight is not a finite positive number" : "") +
              ((hflag & 3) == 3 ? "; " : "") +
              ((hflag & 2) ? "weights of an entry and its mirror differ" : ""));
    return NVD_E_GRAPH;
  }
  // 2. commit: weights, degrees and their inverses
  if (!g->w64) {
    NVD_HIP(hipMalloc((void**)&g->w64, sizeof(double) * std::max(g->nnz, 1)));
    NVD_HIP(hipMalloc((void**)&g->w32, sizeof(float) * std::max(g->nnz, 1)));
    g->bytes += (int64_t)12 * std::max(g->nnz, 1);
  }
  if (g->nnz > 0)
    k_set_weights<<<(g->nnz + 255) / 256, 256, 0, s>>>(g->nnz, g->in_pos, w, g->w64, g->w32);
  k_degree_refresh<<<grid, 256, 0, s>>>(g->n, g->rp, g->w64, g->deg64, g->deg32, g->invd64,
                                        g->invd32);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_error(std::string("nvd_graph_set_weights: ") + hipGetErrorString(e));
    return NVD_E_DEVICE;
  }
  g->weighted = true;
  // the spanning forest (tree preconditioner) holds 1/w of its edges and is
  // built from the host copy of the weights: refresh the copy, drop the forest
  free_tree(g->tree);
  g->tree = nullptr;
  if (g->achol) g->bytes -= g->achol->bytes;
  free_achol(g->achol);
  g->achol = nullptr;
  // the slices of the one-column apply hold copies of the weights
  free_slices(g);
  g->h_w.resize(std::max(g->nnz, 1));
  if (hipMemcpy(g->h_w.data(), g->w64, sizeof(double) * g->nnz, hipMemcpyDeviceToHost) != hipSuccess) {
    set_error("nvd_graph_set_weights: copying the weights back failed");
    return NVD_E_DEVICE;
  }
  g->h_w.resize(g->nnz);
  return NVD_OK;
}

nvd_status nvd_grad_vectors(nvd_graph* h, int32_t k, const double* X, int64_t ldx,
                            const double* gscale, double* GP, int64_t ldp, double* GQ,
                            int64_t ldq, void* stream) {
  set_error("");
  if (!h || !X || !gscale || (!GP && !GQ) || k < 1 || ldx < k || (GP && ldp < k) ||
      (GQ && ldq < k)) {
    set_error("nvd_grad_vectors: bad argument (NULL pointer, k < 1 or ld < k)");
    return NVD_E_ARG;
  }
  const int n = h->g->n;
  const long grid = std::min<long>(std::max<long>(((long)n * k + kBS - 1) / kBS, 1), 4096);
  k_grad_vec<<<grid, kBS, 0, as_stream(stream)>>>(n, k, X, ldx, gscale, GP, ldp, GQ, ldq);
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

nvd_status nvd_grad_scale_from_d(int32_t k, const double* g_d, const double* d, double* gscale,
                                 void* stream) {
  set_error("");
  if (!g_d || !d || !gscale || k < 1) {
    set_error("nvd_grad_scale_from_d: bad argument (NULL pointer or k < 1)");
    return NVD_E_ARG;
  }
  k_grad_scale_d<<<(k + 255) / 256, 256, 0, as_stream(stream)>>>(k, g_d, d, gscale);
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

nvd_status nvd_grad_weights(nvd_graph* h, int32_t k, const double* X, int64_t ldx,
                            const double* gscale, double* grad_w, void* stream) {
  set_error("");
  if (!h || !X || !gscale || !grad_w || k < 1 || ldx < k) {
    set_error("nvd_grad_weights: bad argument");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  hipStream_t s = as_stream(stream);
  if (g->in_pos) NVD_HIP(hipMemsetAsync(grad_w, 0, sizeof(double) * g->nnz_in, s));
  for (int c0 = 0; c0 < k;) {
    int T = 64;
    while (T > k - c0) T >>= 1;
    const int rows_per_block = (kBS / 64) * (64 / T);
    long grid = (g->n + rows_per_block - 1) / rows_per_block;
    grid = std::min<long>(std::max<long>(grid, 1), 8192);
    const int acc = c0 > 0 ? 1 : 0;
    switch (T) {
#define NVD_G(TT) \
  case TT: k_grad_w<TT><<<grid, kBS, 0, s>>>(g->n, g->rp, g->ci, g->in_pos, X + c0, ldx, gscale + c0, grad_w, acc); break;
      NVD_G(1) NVD_G(2) NVD_G(4) NVD_G(8) NVD_G(16) NVD_G(32) NVD_G(64)
#undef NVD_G
      default: break;
    }
    NVD_HIP(hipGetLastError());
    c0 += T;
  }
  return NVD_OK;
}

}  // extern "C"
