// One launch per tile for small connected graphs: the whole Jacobi-PCG solve
// of nvd_distances (projection, CG iterations, FP64 restarts or the mixed
// refinement with its stagnation guard, the quadratic form and the per-pair
// info) in a single 1024-thread block, with block barriers where the
// multi-kernel path has kernel boundaries and host polls.
//
// On a graph of a few thousand nodes every kernel of the multi-kernel path
// is a few microseconds of work behind a launch, and the host reads the
// convergence state between chunks of iterations: a 1e3-node solve of ~25
// iterations costs ~0.7 ms, almost all of it launch gaps and polls.  Here
// the block keeps every per-column scalar in LDS; block reductions run in a
// fixed order, so results repeat bit for bit.  One block sees its own global
// writes after a barrier, so the vectors stay in the graph's workspace.
//
// The arithmetic is that of the multi-kernel path (same recurrences, same
// stopping rules, same edge-difference form of L x), so the results agree
// up to the order of floating-point sums.
#include <cstdlib>

#include "device_common.hpp"
#include "refine_guard.hpp"

namespace nvd {

constexpr int kSmallBS = 1024;
// Work bound for the single-block path: (nnz + n) * T gathered/streamed
// elements per iteration, and n * T elements per vector.
constexpr long kSmallWork = 1L << 17;
constexpr long kSmallVec = 1L << 16;

struct SmallArgs {
  int n;
  const int* rp;
  const int* ci;
  const double* w64;   // null for unit weights
  const float* w32;
  const double* invd64;
  const float* invd32;
  const double* P;
  const double* Q;
  long ld;
  double *b64, *x64, *r64, *p64, *q64;
  float *x32, *r32, *p32, *q32;
  double rtol2, irtol2, stall_ratio2;
  int max_iter, max_refine, mixed, out_dsq;
  double* d_out;
  double* X;
  long ldx;
  nvd_pair_info* info;
};

struct SmallState {
  double rho[kMaxTile], alpha[kMaxTile], beta[kMaxTile], bnorm2[kMaxTile], obnorm2[kMaxTile];
  double itol2[kMaxTile], orr[kMaxTile], mean[kMaxTile];
  double dots[5][kMaxTile];
  int active[kMaxTile], oactive[kMaxTile], iters[kMaxTile], it_cur[kMaxTile], status[kMaxTile];
  int refine[kMaxTile], stall[kMaxTile], fb[kMaxTile], fbdone[kMaxTile];
  int count;
};

// Column sums of ND per-thread values: thread t holds column t % T (the
// block size is a multiple of T).  out[d * kMaxTile + c], fixed order.
template <int ND, int T>
__device__ __forceinline__ void small_reduce(const double (&acc)[ND], double* sh, double* out) {
  const int t = threadIdx.x;
#pragma unroll
  for (int d = 0; d < ND; ++d) sh[d * kSmallBS + t] = acc[d];
  __syncthreads();
  for (int half = kSmallBS / 2; half >= T; half >>= 1) {
    if (t < half) {
#pragma unroll
      for (int d = 0; d < ND; ++d) sh[d * kSmallBS + t] += sh[d * kSmallBS + t + half];
    }
    __syncthreads();
  }
  if (t < T) {
#pragma unroll
    for (int d = 0; d < ND; ++d) out[d * kMaxTile + t] = sh[d * kSmallBS + t];
  }
  __syncthreads();
}

// Number of columns whose flag is set (thread 0 counts; all threads read).
__device__ __forceinline__ int small_count(SmallState& S, const int* flag, int T) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int k = 0;
    for (int c = 0; c < T; ++c) k += flag[c];
    S.count = k;
  }
  __syncthreads();
  return S.count;
}

// y = L x (edge differences), per-thread partial of x^T y for its column.
template <typename V, int T, bool UNIT>
__device__ __forceinline__ double small_apply(const SmallArgs& a, const V* __restrict__ w,
                                              const V* __restrict__ x, V* __restrict__ y) {
  double acc = 0.0;
  const long nT = (long)a.n * T;
  for (long e = threadIdx.x; e < nT; e += kSmallBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    const V xi = x[e];
    V sum = (V)0;
    const int lo = a.rp[i], hi = a.rp[i + 1];
    int j = lo;
    for (; j + 3 < hi; j += 4) {
      int cj[4];
      V wj[4], xj[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        cj[u] = a.ci[j + u];
        wj[u] = UNIT ? (V)1 : w[j + u];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) xj[u] = x[(long)cj[u] * T + c];
#pragma unroll
      for (int u = 0; u < 4; ++u) sum += wj[u] * (xi - xj[u]);
    }
    for (; j < hi; ++j) sum += (UNIT ? (V)1 : w[j]) * (xi - x[(long)a.ci[j] * T + c]);
    y[e] = sum;
    acc += (double)xi * (double)sum;
  }
  return acc;
}

// r = b - L x in FP64 and its dots: b^T x, x^T r, r^T r, sum r, sum x
// (S.dots[0..4]).
template <int T, bool UNIT>
__device__ void small_resid(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const long nT = (long)a.n * T;
  for (long e = threadIdx.x; e < nT; e += kSmallBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    const double xi = a.x64[e];
    double sum = 0.0;
    for (int j = a.rp[i]; j < a.rp[i + 1]; ++j)
      sum += (UNIT ? 1.0 : a.w64[j]) * (xi - a.x64[(long)a.ci[j] * T + c]);
    const double bb = a.b64[e];
    const double rr = bb - sum;
    a.r64[e] = rr;
    acc[0] += bb * xi;
    acc[1] += xi * rr;
    acc[2] += rr * rr;
    acc[3] += rr;
    acc[4] += xi;
  }
  small_reduce<5, T>(acc, sh, red);
  if (threadIdx.x < T) {
#pragma unroll
    for (int d = 0; d < 5; ++d) S.dots[d][threadIdx.x] = red[d * kMaxTile + threadIdx.x];
  }
  __syncthreads();
}

// x -= its column mean (one component).
template <int T>
__device__ void small_center_x(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  double acc[1] = {0.0};
  const long nT = (long)a.n * T;
  for (long e = threadIdx.x; e < nT; e += kSmallBS) acc[0] += a.x64[e];
  small_reduce<1, T>(acc, sh, red);
  if (threadIdx.x < T) S.mean[threadIdx.x] = red[threadIdx.x] / (double)a.n;
  __syncthreads();
  for (long e = threadIdx.x; e < nT; e += kSmallBS) a.x64[e] -= S.mean[e % T];
  __syncthreads();
}

// CG iterations (preconditioner D) until no column is active: as cg_loop
// with k_spmm (EPI_CG), k_update and k_direction.
template <typename V, int T, bool UNIT>
__device__ void small_cg(const SmallArgs& a, const V* w, const V* invd, V* x, V* r, V* p, V* q,
                         double rtol2, SmallState& S, double* sh, double* red) {
  const int t = threadIdx.x;
  const int c = t % T;
  const long nT = (long)a.n * T;
  for (int it = 0; it < a.max_iter; ++it) {
    if (small_count(S, S.active, T) == 0) break;
    {
      double acc[1] = {small_apply<V, T, UNIT>(a, w, p, q)};
      small_reduce<1, T>(acc, sh, red);
      if (t < T) {
        double al = 0.0;
        if (S.active[t]) {
          const double sg = red[t];
          if (!(sg > 0.0) || !isfinite(sg)) {
            S.status[t] = kStBreak;
            S.active[t] = 0;
            S.oactive[t] = 0;
          } else {
            al = S.rho[t] / sg;
          }
        }
        S.alpha[t] = al;
      }
      __syncthreads();
    }
    {
      const V al = (V)S.alpha[c];
      double acc[2] = {0.0, 0.0};
      for (long e = t; e < nT; e += kSmallBS) {
        x[e] += al * p[e];
        const V rv = r[e] - al * q[e];
        r[e] = rv;
        const double rd = (double)rv;
        acc[0] += rd * rd * (double)invd[e / T];
        acc[1] += rd * rd;
      }
      small_reduce<2, T>(acc, sh, red);
      if (t < T) {
        double be = 0.0;
        if (S.active[t]) {
          const double rz = red[t], rr = red[kMaxTile + t];
          S.iters[t] += 1;
          S.it_cur[t] += 1;
          const double tol2 = S.itol2[t] > 0.0 ? S.itol2[t] : rtol2;
          if (rr <= tol2 * S.bnorm2[t]) {
            S.active[t] = 0;
          } else if (S.it_cur[t] >= a.max_iter) {
            S.active[t] = 0;
            S.status[t] = kStNoconv;
            S.oactive[t] = 0;
          } else if (!(rz > 0.0) || !isfinite(rz)) {
            S.active[t] = 0;
            S.status[t] = kStBreak;
            S.oactive[t] = 0;
          } else {
            be = rz / S.rho[t];
            S.rho[t] = rz;
          }
        }
        S.beta[t] = be;
      }
      __syncthreads();
    }
    {
      const V be = (V)S.beta[c];
      const int act = S.active[c];
      for (long e = t; e < nT; e += kSmallBS)
        if (act) p[e] = r[e] * invd[e / T] + be * p[e];
      __syncthreads();
    }
  }
}

// FP64 CG from the restart state, then the true residual with up to two
// restarts from it; ends with x mean-zero and the residual of the final x.
template <int T, bool UNIT>
__device__ void small_fp64(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  const int t = threadIdx.x;
  const long nT = (long)a.n * T;
  for (int restarts = 0;; ++restarts) {
    small_cg<double, T, UNIT>(a, a.w64, a.invd64, a.x64, a.r64, a.p64, a.q64, a.rtol2, S, sh, red);
    small_center_x<T>(a, S, sh, red);
    small_resid<T, UNIT>(a, S, sh, red);
    if (t < T)
      S.oactive[t] = S.status[t] == kStOk && S.obnorm2[t] > 0.0 && S.dots[2][t] > a.rtol2 * S.obnorm2[t];
    if (small_count(S, S.oactive, T) == 0 || restarts >= 2) break;
    // restart from the true residual: p = D^-1 r, rho = r^T D^-1 r
    double acc[1] = {0.0};
    for (long e = t; e < nT; e += kSmallBS) {
      const double z = a.r64[e] * a.invd64[e / T];
      a.p64[e] = z;
      acc[0] += a.r64[e] * z;
    }
    small_reduce<1, T>(acc, sh, red);
    if (t < T) {
      S.rho[t] = red[t];
      S.active[t] = S.oactive[t] && red[t] > 0.0;
      S.bnorm2[t] = S.obnorm2[t];
      S.itol2[t] = 0.0;
      S.it_cur[t] = 0;
    }
    __syncthreads();
  }
}

template <int T, bool UNIT>
__global__ __launch_bounds__(kSmallBS) void k_small_solve(SmallArgs a) {
  __shared__ double sh[5 * kSmallBS];
  __shared__ double red[5 * kMaxTile];
  __shared__ SmallState S;
  const int t = threadIdx.x;
  const int c = t % T;
  const int n = a.n;
  const long nT = (long)n * T;
  // (a2) delta_bar = (P - Q) minus its mean (one component)
  {
    double acc[1] = {0.0};
    for (long e = t; e < nT; e += kSmallBS) {
      const long i = e / T;
      acc[0] += a.P[i * a.ld + c] - a.Q[i * a.ld + c];
    }
    small_reduce<1, T>(acc, sh, red);
    if (t < T) S.mean[t] = red[t] / (double)n;
    __syncthreads();
  }
  {
    const double m = S.mean[c];
    double acc[2] = {0.0, 0.0};
    for (long e = t; e < nT; e += kSmallBS) {
      const long i = e / T;
      const double v = a.P[i * a.ld + c] - a.Q[i * a.ld + c] - m;
      a.b64[e] = v;
      a.x64[e] = 0.0;
      acc[0] += v * v;
      if (!a.mixed) {
        const double z = v * a.invd64[i];
        a.r64[e] = v;
        a.p64[e] = z;
        acc[1] += v * z;
      }
    }
    small_reduce<2, T>(acc, sh, red);
    if (t < T) {
      const double bb = red[t];
      S.obnorm2[t] = bb;
      S.bnorm2[t] = bb;
      S.orr[t] = bb;
      S.rho[t] = red[kMaxTile + t];
      S.oactive[t] = bb > 0.0;
      S.active[t] = !a.mixed && bb > 0.0;
      S.iters[t] = S.it_cur[t] = S.refine[t] = 0;
      S.status[t] = kStOk;
      S.itol2[t] = 0.0;
      S.stall[t] = S.fb[t] = S.fbdone[t] = 0;
    }
    __syncthreads();
  }
  bool fp64_finish = !a.mixed;
  if (!a.mixed) {
    small_fp64<T, UNIT>(a, S, sh, red);
  } else {
    bool first = true;
    for (int step = 0; step <= a.max_refine; ++step) {
      const double* src = a.b64;
      if (!first) {
        // (a7) FP64 outer residual and the outer check on its projection
        small_resid<T, UNIT>(a, S, sh, red);
        if (t < T) {
          S.mean[t] = S.dots[3][t] / (double)n;
          if (S.oactive[t]) {
            const double rr = S.dots[2][t] - (double)n * S.mean[t] * S.mean[t];
            if (rr <= a.rtol2 * S.obnorm2[t]) {
              S.oactive[t] = 0;
            } else if (S.refine[t] >= a.max_refine) {
              S.oactive[t] = 0;
              S.status[t] = kStNoconv;
            }
          }
        }
        if (small_count(S, S.oactive, T) == 0) break;
        src = a.r64;
      }
      // inner set-up from src (minus its mean after the first step)
      {
        const double m = first ? 0.0 : S.mean[c];
        double acc[3] = {0.0, 0.0, 0.0};
        for (long e = t; e < nT; e += kSmallBS) {
          const double v = src[e] - m;
          const float f = (float)v;
          const float z = f * a.invd32[e / T];
          a.r32[e] = f;
          a.x32[e] = 0.0f;
          a.p32[e] = z;
          acc[0] += v * v;
          acc[1] += (double)f * (double)z;
          acc[2] += (double)f * (double)f;
        }
        small_reduce<3, T>(acc, sh, red);
        if (t < T) {
          const double rr = red[t];
          const double rr_old = S.orr[t];
          S.orr[t] = rr;
          int act = 0;
          if (S.oactive[t] && !first)
            S.stall[t] = refine_stall_count(rr_old, rr, S.stall[t], a.stall_ratio2);
          if (S.oactive[t]) {
            if (!first && rr <= a.rtol2 * S.obnorm2[t]) {
              S.oactive[t] = 0;
            } else if (refine_hand_to_fp64(S.stall[t])) {
              S.oactive[t] = 0;
              S.fb[t] = 1;
            } else if (S.refine[t] >= a.max_refine) {
              S.oactive[t] = 0;
              S.status[t] = kStNoconv;
            } else if (red[2 * kMaxTile + t] > 0.0) {
              act = 1;
              S.refine[t] += 1;
            } else {
              S.oactive[t] = 0;
            }
          }
          S.active[t] = act;
          S.bnorm2[t] = red[2 * kMaxTile + t];
          S.rho[t] = red[kMaxTile + t];
          S.it_cur[t] = 0;
          const double need2 = rr > 0.0 ? 0.09 * a.rtol2 * S.obnorm2[t] / rr : 0.0;
          S.itol2[t] = need2 > a.irtol2 ? (need2 < 0.25 ? need2 : 0.25) : a.irtol2;
        }
        if (small_count(S, S.oactive, T) == 0) break;
      }
      first = false;
      small_cg<float, T, UNIT>(a, a.w32, a.invd32, a.x32, a.r32, a.p32, a.q32, a.irtol2, S, sh, red);
      // x += c on the pairs whose inner solve ended well; a pair whose FP32
      // solve ran out of iterations goes to the FP64 solver instead
      {
        const int ok = S.status[c] == kStOk;
        for (long e = t; e < nT; e += kSmallBS)
          if (ok) a.x64[e] += (double)a.x32[e];
        __syncthreads();
        if (t < T && S.status[t] == kStNoconv && S.it_cur[t] >= a.max_iter) {
          S.status[t] = kStOk;
          S.fb[t] = 1;
        }
        __syncthreads();
      }
    }
    if (small_count(S, S.fb, T) > 0) {
      // the FP64 solver finishes the pairs that stalled, from their current x
      small_resid<T, UNIT>(a, S, sh, red);
      if (t < T) {
        S.oactive[t] = S.fb[t];
        if (S.fb[t]) S.fbdone[t] = 1;
        S.fb[t] = 0;
      }
      __syncthreads();
      double acc[1] = {0.0};
      for (long e = t; e < nT; e += kSmallBS) {
        const double z = a.r64[e] * a.invd64[e / T];
        a.p64[e] = z;
        acc[0] += a.r64[e] * z;
      }
      small_reduce<1, T>(acc, sh, red);
      if (t < T) {
        S.rho[t] = red[t];
        S.active[t] = S.oactive[t] && red[t] > 0.0;
        S.bnorm2[t] = S.obnorm2[t];
        S.itol2[t] = 0.0;
        S.it_cur[t] = 0;
      }
      __syncthreads();
      small_fp64<T, UNIT>(a, S, sh, red);
      fp64_finish = true;
    } else {
      small_center_x<T>(a, S, sh, red);
      small_resid<T, UNIT>(a, S, sh, red);
    }
  }
  // (a8) quadratic form, distances, per-pair info; x out
  if (a.X) {
    for (long e = t; e < nT; e += kSmallBS) a.X[(e / T) * a.ldx + (e % T)] = a.x64[e];
  }
  if (t < T) {
    const double bx = S.dots[0][t], xr = S.dots[1][t], rr = S.dots[2][t];
    const double bb = S.obnorm2[t];
    double dsq = bx + xr;
    double rel = 0.0;
    if (bb > 0.0)
      rel = sqrt(rr / bb);
    else
      dsq = 0.0;
    int st = S.status[t];
    if (fp64_finish && st == kStOk && S.oactive[t]) st = kStNoconv;
    const double d0 = dsq > 0.0 ? dsq : 0.0;
    a.d_out[t] = a.out_dsq ? d0 : sqrt(d0);
    nvd_pair_info pi;
    pi.status = st;
    pi.iters = S.iters[t];
    pi.refine_steps = S.refine[t];
    pi.flags = S.fbdone[t] ? NVD_INFO_FP64_FALLBACK : 0;
    pi.rel_res = rel;
    pi.dsq_plain = bb > 0.0 ? bx : 0.0;
    pi.dsq = dsq;
    a.info[t] = pi;
  }
}

bool small_eligible(const DevGraph* g, int T, const SolveParams& sp) {
  if (g->n_comp != 1 || sp.tree || sp.achol || sp.warm) return false;
  const long work = ((long)g->nnz + g->n) * T;
  if (work > kSmallWork || (long)g->n * T > kSmallVec) return false;
  const char* e = std::getenv("NVD_SMALL");
  return !(e && e[0] == '0');
}

nvd_status solve_small(DevGraph* g, int T, const double* P, const double* Q, int64_t ld,
                       const SolveParams& sp, double* d_out, double* X, int64_t ldx,
                       nvd_pair_info* info_dev, hipStream_t s) {
  const bool mixed = sp.precision == NVD_MIXED;
  NVD_TRY(ensure_workspace(g, T, mixed));
  Workspace* ws = g->ws;
  SmallArgs a{};
  a.n = g->n;
  a.rp = g->rp;
  a.ci = g->ci;
  a.w64 = g->w64;
  a.w32 = g->w32;
  a.invd64 = g->invd64;
  a.invd32 = g->invd32;
  a.P = P;
  a.Q = Q;
  a.ld = ld;
  a.b64 = ws->b64;
  a.x64 = ws->x64;
  a.r64 = ws->r64;
  a.p64 = ws->p64;
  a.q64 = ws->q64;
  a.x32 = ws->x32;
  a.r32 = ws->r32;
  a.p32 = ws->p32;
  a.q32 = ws->q32;
  a.rtol2 = sp.rtol * sp.rtol;
  a.irtol2 = sp.inner_rtol * sp.inner_rtol;
  a.stall_ratio2 = kStallRatio2;
  if (const char* e = std::getenv("NVD_REFINE_STALL_RATIO2")) {
    const double v = std::strtod(e, nullptr);
    if (v >= 0.0 && v <= 1.0) a.stall_ratio2 = v;
  }
  a.max_iter = sp.max_iter;
  a.max_refine = sp.max_refine;
  a.mixed = mixed ? 1 : 0;
  a.out_dsq = sp.out_dsq ? 1 : 0;
  a.d_out = d_out;
  a.X = X;
  a.ldx = ldx;
  a.info = info_dev;
  const bool unit = !g->weighted;
#define NVD_SMALL_T(TT)                                                      \
  case TT:                                                                   \
    if (unit)                                                                \
      k_small_solve<TT, true><<<1, kSmallBS, 0, s>>>(a);                     \
    else                                                                     \
      k_small_solve<TT, false><<<1, kSmallBS, 0, s>>>(a);                    \
    break;
  switch (T) {
    NVD_SMALL_T(1) NVD_SMALL_T(2) NVD_SMALL_T(4) NVD_SMALL_T(8) NVD_SMALL_T(16) NVD_SMALL_T(32)
    NVD_SMALL_T(64)
    default:
      set_error("small solve: tile must be a power of two up to 64");
      return NVD_E_ARG;
  }
#undef NVD_SMALL_T
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

}  // namespace nvd
