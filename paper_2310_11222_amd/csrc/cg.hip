// Jacobi-preconditioned conjugate gradients for L x = delta_bar on one graph,
// a tile of T independent right-hand sides at a time (the paper's section 3.2
// replaces L^+ by such a Laplacian solve), and the FP64 quadratic form.
//
// Per CG iteration (per column c, preconditioner M = D):
//   q = L p                 sigma = p^T q        alpha = rho / sigma   (SpMM, EPI_CG)
//   r -= alpha q; z = r / deg;  rho' = r^T z; ||r||^2; beta = rho'/rho (k_update)
//   x += alpha p; p = z + beta p                                       (k_direction)
// x is updated where p is read anyway: 8 vector passes per iteration
// instead of 9.
// Every reduction finishes on the device (last block of the grid), so the
// host only polls one word per chunk of iterations.
//
// Precision modes:
//   FP64  : all of the above in FP64; at the end x is made mean-zero per
//           component and the true residual r = delta_bar - L x is taken in
//           FP64 (restarting CG from it if it is above rtol).
//   MIXED : outer iterative refinement in FP64 -- r = delta_bar - L x (FP64
//           operator), per-component mean removal, ||r|| -- around an inner
//           FP32 CG solve of L c = r to inner_rtol; x += c in FP64.
// Both return d^2 = delta_bar^T x + x^T r from the final FP64 residual.
#include <algorithm>
#include <cstddef>
#include <cstdlib>
#include <cmath>
#include <vector>

#include "device_common.hpp"
#include "prof.hpp"
#include "refine_guard.hpp"

namespace nvd {

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
struct ProjSrc {
  const double* a;   // first operand (row-major, lda)
  long lda;
  const double* b;   // optional second operand subtracted (ldb), may be null
  long ldb;
};

// Column sums of (a - b) over all rows; the grid's last block stores
// mean[c] = sum / n (single-component graphs).
template <int T>
__global__ __launch_bounds__(kBS) void k_colsum(int n, ProjSrc src, ColState* cs, GridRed red) {
  __shared__ double sh[kBS];
  __shared__ double vals[kMaxTile];
  const int t = threadIdx.x;
  const int c = t % T;
  constexpr int RPB = kBS / T;
  double acc[1][1] = {{0.0}};
  for (long i = (long)blockIdx.x * RPB + t / T; i < n; i += (long)gridDim.x * RPB) {
    double v = src.a[i * src.lda + c];
    if (src.b) v -= src.b[i * src.ldb + c];
    acc[0][0] += v;
  }
  block_reduce_cols<kBS, 1, 1>(acc, T, sh);
  if (t < T) vals[t] = sh[t];
  __syncthreads();
  if (!grid_reduce<kBS>(vals, T, red)) return;
  if (t < T) cs->mean[t] = vals[t] / (double)n;
}

// Per-component means of (a - b): one block per component.
template <int T>
__global__ __launch_bounds__(kBS) void k_comp_mean(int ncomp, const int* perm, const int* off,
                                                   ProjSrc src, double* cmean) {
  __shared__ double sh[kBS];
  const int t = threadIdx.x;
  const int c = t % T;
  constexpr int RPB = kBS / T;
  for (int k = blockIdx.x; k < ncomp; k += gridDim.x) {
    const int lo = off[k], hi = off[k + 1];
    double acc[1][1] = {{0.0}};
    for (int p = lo + t / T; p < hi; p += RPB) {
      const long i = perm[p];
      double v = src.a[i * src.lda + c];
      if (src.b) v -= src.b[i * src.ldb + c];
      acc[0][0] += v;
    }
    block_reduce_cols<kBS, 1, 1>(acc, T, sh);
    if (t < T) cmean[(long)k * kMaxTile + t] = sh[t] / (double)(hi - lo);
    __syncthreads();
  }
}

// Where a projection takes its means from.
struct MeanSrc {
  const double* colmean;   // [T] (single component) or null
  const double* cmean;     // [ncomp][kMaxTile] or null
  const int* comp;
  const double* dots_sum;  // mean = dots_sum[c] / n (sum from a residual pass) or null
  int n;
};

__device__ __forceinline__ double mean_of(const MeanSrc& m, long i, int c) {
  if (m.cmean) return m.cmean[(long)m.comp[i] * kMaxTile + c];
  if (m.colmean) return m.colmean[c];
  if (m.dots_sum) return m.dots_sum[c] / (double)m.n;
  return 0.0;
}

// delta_bar = (P - Q) - mean; b = delta_bar; x = 0; for the FP64 solver also
// r = delta_bar, p = D^-1 r, q = 0 and rho = r^T D^-1 r.  Padding beyond n*T
// is zeroed.
template <int T>
__global__ __launch_bounds__(kBS) void k_proj_init(int n, long cap, ProjSrc src, MeanSrc m,
                                                   const double* invd, double* b64, double* x64,
                                                   double* r64, double* p64, double* q64,
                                                   int fp64cg, ColState* cs, GridRed red) {
  __shared__ double sh[2 * kBS];
  __shared__ double vals[2 * kMaxTile];
  const int t = threadIdx.x;
  double acc[2][1] = {{0.0}, {0.0}};
  for (long e = (long)blockIdx.x * kBS + t; e < cap; e += (long)gridDim.x * kBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    double v = 0.0;
    if (i < n) {
      v = src.a[i * src.lda + c] - (src.b ? src.b[i * src.ldb + c] : 0.0) - mean_of(m, i, c);
      acc[0][0] += v * v;
      acc[1][0] += v * v * invd[i];
    }
    b64[e] = v;
    x64[e] = 0.0;
    if (fp64cg) {
      r64[e] = v;
      p64[e] = i < n ? v * invd[i] : 0.0;   // p0 = z0 = D^-1 r0
      q64[e] = 0.0;
    }
  }
  block_reduce_cols<kBS, 2, 1>(acc, T, sh);
  if (t < T) {
    vals[t] = sh[t];
    vals[T + t] = sh[kBS + t];
  }
  __syncthreads();
  if (!grid_reduce<kBS>(vals, 2 * T, red)) return;
  if (t < T) {
    const double bb = vals[t];
    cs->obnorm2[t] = bb;
    cs->bnorm2[t] = bb;
    cs->orr[t] = bb;
    cs->rho[t] = vals[T + t];
    cs->alpha[t] = 0.0;
    cs->beta[t] = 0.0;
    const int act = bb > 0.0;
    cs->oactive[t] = act;
    cs->active[t] = fp64cg ? act : 0;
    cs->iters[t] = 0;
    cs->it_cur[t] = 0;
    cs->refine[t] = 0;
    cs->status[t] = kStOk;
    cs->itol2[t] = 0.0;
    cs->stall[t] = 0;
    cs->fb[t] = 0;
    cs->fbdone[t] = 0;
  }
  if (t == 0) cs->xseq = cs->xdone = 0;   // a CG run starts: no x update pending
  recount_active(cs, T);
}

// Loads and stores of the vector passes of an iteration (update,
// direction): non-temporal (NVD_STREAM_NT=1, the default), since each
// vector is touched once per pass and the tile's vectors together exceed
// the last-level cache on large graphs.  Measured on the 1e7-node
// configuration model at T = 16 (FP32): the direction kernel went from 5.6
// to 6.7 TB/s and the update from 5.5 to 5.8 TB/s, 79.1 -> 75.8 ms per
// 16 distances (mixed) and 106.3 -> 101.7 ms (FP64).
#ifndef NVD_STREAM_NT
#define NVD_STREAM_NT 1
#endif
template <typename V, typename VT>
__device__ __forceinline__ VT sld(const VT* p) {
#if NVD_STREAM_NT
  using E = typename VecOf<V, Vec16<V>::N>::type;
  const E e = __builtin_nontemporal_load(reinterpret_cast<const E*>(p));
  VT out;
  __builtin_memcpy(&out, &e, sizeof(VT));
  return out;
#else
  return *p;
#endif
}
template <typename V, typename VT>
__device__ __forceinline__ void sst(const VT& v, VT* p) {
#if NVD_STREAM_NT
  using E = typename VecOf<V, Vec16<V>::N>::type;
  E e;
  __builtin_memcpy(&e, &v, sizeof(VT));
  __builtin_nontemporal_store(e, reinterpret_cast<E*>(p));
#else
  *p = v;
#endif
}

// 1/deg for the N elements of vector i (row-major n x T, N elements per
// 16-byte vector).  When T >= N all N elements share one row: one load.
// Otherwise the N rows are loaded with clamped indices (no branch per load)
// and zeroed past n.
template <typename V, int T>
__device__ __forceinline__ void invd_of(const V* __restrict__ invd, int n, long i, V (&iv)[Vec16<V>::N]) {
  constexpr int N = Vec16<V>::N;
  if constexpr (T >= N) {
    const long row = (i * N) / T;
    const V v = invd[row < n ? row : n - 1];
#pragma unroll
    for (int k = 0; k < N; ++k) iv[k] = row < n ? v : (V)0;
  } else {
#pragma unroll
    for (int k = 0; k < N; ++k) {
      const long row = (i * N + k) / T;
      const V v = invd[row < n ? row : n - 1];
      iv[k] = row < n ? v : (V)0;
    }
  }
}

// r -= alpha q; rho' = r^T D^-1 r; ||r||^2.  The grid's last block forms
// beta, retires converged columns and advances xseq (x += alpha p of this
// iteration is left to the direction kernel, which reads p anyway).  TREE
// (spanning-tree preconditioner): ||r||^2 and retirement only; rho' = r^T z
// and beta follow once z = L_T^+ r is known (k_rz).
template <typename V, int T, bool TREE = false>
__global__ __launch_bounds__(kBS) void k_update(int n, long cap, V* __restrict__ r,
                                                const V* __restrict__ q,
                                                const V* __restrict__ invd, double rtol2,
                                                int max_iter, ColState* cs, GridRed red) {
  using VT = typename Vec16<V>::type;
  constexpr int N = Vec16<V>::N;
  __shared__ double sh[2 * kBS * N];
  __shared__ double vals[2 * kMaxTile];
  if (cs->n_active == 0) {
    // no iteration ran: the direction kernel that follows has no x to update
    if (blockIdx.x == 0 && threadIdx.x == 0) cs->xdone = cs->xseq;
    return;
  }
  const int t = threadIdx.x;
  V al[N];
#pragma unroll
  for (int v = 0; v < N; ++v) al[v] = (V)cs->alpha[(t * N + v) % T];
  double acc[2][N];
#pragma unroll
  for (int v = 0; v < N; ++v) acc[0][v] = acc[1][v] = 0.0;
  const long nv = cap / N;
  for (long i = (long)blockIdx.x * kBS + t; i < nv; i += (long)gridDim.x * kBS) {
    VT rv = sld<V>(reinterpret_cast<const VT*>(r) + i);
    const VT qv = sld<V>(reinterpret_cast<const VT*>(q) + i);
    V* rs = reinterpret_cast<V*>(&rv);
    const V* qs = reinterpret_cast<const V*>(&qv);
    V iv[N];
    if constexpr (!TREE) invd_of<V, T>(invd, n, i, iv);
#pragma unroll
    for (int v = 0; v < N; ++v) {
      rs[v] -= al[v] * qs[v];
      const double rd = (double)rs[v];
      if constexpr (!TREE) acc[0][v] += rd * rd * (double)iv[v];
      acc[1][v] += rd * rd;
    }
    sst<V>(rv, reinterpret_cast<VT*>(r) + i);
  }
  block_reduce_cols<kBS, 2, N>(acc, T, sh);
  if (t < T) {
    vals[t] = sh[t];
    vals[T + t] = sh[kBS * N + t];
  }
  __syncthreads();
  if (!grid_reduce<kBS>(vals, 2 * T, red)) return;
  if (t < T) {
    double be = 0.0;
    if (cs->active[t]) {
      const double rz = vals[t];
      const double rr = vals[T + t];
      cs->iters[t] += 1;
      cs->it_cur[t] += 1;
      const double tol2 = cs->itol2[t] > 0.0 ? cs->itol2[t] : rtol2;
      if (rr <= tol2 * cs->bnorm2[t]) {
        cs->active[t] = 0;
      } else if (cs->it_cur[t] >= max_iter) {
        cs->active[t] = 0;
        cs->status[t] = kStNoconv;
        cs->oactive[t] = 0;
      } else if (TREE) {
        // beta from r^T z in k_rz
      } else if (!(rz > 0.0) || !isfinite(rz)) {
        cs->active[t] = 0;
        cs->status[t] = kStBreak;
        cs->oactive[t] = 0;
      } else {
        be = rz / cs->rho[t];
        cs->rho[t] = rz;
      }
      vals[t] = cs->active[t] ? rr / (tol2 * cs->bnorm2[t]) : 0.0;
    } else {
      vals[t] = 0.0;
    }
    cs->beta[t] = be;
  }
  __syncthreads();
  if (t == 0) {
    double wmax = 0.0;
    for (int c = 0; c < T; ++c) wmax = vals[c] > wmax ? vals[c] : wmax;
    cs->worst = wmax;
    cs->xseq += 1;
  }
  recount_active(cs, T);
}

// x += alpha p (the iteration whose update kernel ran, columns that retired
// in it included; alpha is 0 on columns inactive at the apply), then
// p = D^-1 r + beta p while any column is active.
template <typename V, int T>
__global__ __launch_bounds__(kBS) void k_direction(int n, long cap, V* __restrict__ x,
                                                   V* __restrict__ p, const V* __restrict__ r,
                                                   const V* __restrict__ invd,
                                                   const ColState* cs) {
  using VT = typename Vec16<V>::type;
  constexpr int N = Vec16<V>::N;
  const bool xup = cs->xseq != cs->xdone;
  const bool pup = cs->n_active != 0;
  if (!xup && !pup) return;
  const int t = threadIdx.x;
  V al[N], be[N];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    al[v] = (V)cs->alpha[(t * N + v) % T];
    be[v] = (V)cs->beta[(t * N + v) % T];
  }
  const long nv = cap / N;
  for (long i = (long)blockIdx.x * kBS + t; i < nv; i += (long)gridDim.x * kBS) {
    VT pv = sld<V>(reinterpret_cast<const VT*>(p) + i);
    const V* ps = reinterpret_cast<const V*>(&pv);
    if (xup) {
      VT xv = sld<V>(reinterpret_cast<const VT*>(x) + i);
      V* xs = reinterpret_cast<V*>(&xv);
#pragma unroll
      for (int v = 0; v < N; ++v) xs[v] += al[v] * ps[v];
      sst<V>(xv, reinterpret_cast<VT*>(x) + i);
    }
    if (pup) {
      const VT rv = sld<V>(reinterpret_cast<const VT*>(r) + i);
      V* pw = reinterpret_cast<V*>(&pv);
      const V* rs = reinterpret_cast<const V*>(&rv);
      V iv[N];
      invd_of<V, T>(invd, n, i, iv);
#pragma unroll
      for (int v = 0; v < N; ++v) pw[v] = rs[v] * iv[v] + be[v] * pw[v];
      sst<V>(pv, reinterpret_cast<VT*>(p) + i);
    }
  }
}

// Spanning-tree preconditioner: rho = r^T z with z = L_T^+ r.
//   MODE 0 (start of a CG run): rho = r^T z (columns with r^T z <= 0, i.e.
//           r = 0, are retired);
//   MODE 1 (each iteration): beta = rho' / rho, rho = rho'.  r^T z >= 0
//           holds exactly, but once r is at rounding level the computed
//           value can fall to zero or below (more so with a preconditioner
//           as close to L^+ as a tree is on tree-like graphs): such a column
//           is retired as stalled, and the true-residual check that follows
//           every CG run decides whether it converged.  Only a value that
//           is not finite is a breakdown.
template <typename V, int T, int MODE>
__global__ __launch_bounds__(kBS) void k_rz(long cap, const V* __restrict__ r, const V* __restrict__ z,
                                            ColState* cs, GridRed red) {
  using VT = typename Vec16<V>::type;
  constexpr int N = Vec16<V>::N;
  __shared__ double sh[kBS * N];
  __shared__ double vals[kMaxTile];
  if (MODE == 1 && cs->n_active == 0) return;
  const int t = threadIdx.x;
  double acc[1][N];
#pragma unroll
  for (int v = 0; v < N; ++v) acc[0][v] = 0.0;
  const long nv = cap / N;
  for (long i = (long)blockIdx.x * kBS + t; i < nv; i += (long)gridDim.x * kBS) {
    const VT rv = reinterpret_cast<const VT*>(r)[i];
    const VT zv = reinterpret_cast<const VT*>(z)[i];
    const V* rs = reinterpret_cast<const V*>(&rv);
    const V* zs = reinterpret_cast<const V*>(&zv);
#pragma unroll
    for (int v = 0; v < N; ++v) acc[0][v] += (double)rs[v] * (double)zs[v];
  }
  block_reduce_cols<kBS, 1, N>(acc, T, sh);
  if (t < T) vals[t] = sh[t];
  __syncthreads();
  if (!grid_reduce<kBS>(vals, T, red)) return;
  if (t < T) {
    const double rz = vals[t];
    if constexpr (MODE == 0) {
      cs->rho[t] = rz;
      if (cs->active[t] && !(rz > 0.0)) cs->active[t] = 0;
    } else {
      double be = 0.0;
      if (cs->active[t]) {
        if (!isfinite(rz)) {
          cs->active[t] = 0;
          cs->status[t] = kStBreak;
          cs->oactive[t] = 0;
        } else if (!(rz > 0.0)) {
          cs->active[t] = 0;
        } else {
          be = rz / cs->rho[t];
          cs->rho[t] = rz;
        }
      }
      cs->beta[t] = be;
    }
  }
  recount_active(cs, T);
}

// x += alpha p as in k_direction, then p = z + beta p (z = L_T^+ r)
template <typename V, int T>
__global__ __launch_bounds__(kBS) void k_direction_z(long cap, V* __restrict__ x, V* __restrict__ p,
                                                     const V* __restrict__ z, const ColState* cs) {
  using VT = typename Vec16<V>::type;
  constexpr int N = Vec16<V>::N;
  const bool xup = cs->xseq != cs->xdone;
  const bool pup = cs->n_active != 0;
  if (!xup && !pup) return;
  const int t = threadIdx.x;
  V al[N], be[N];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    al[v] = (V)cs->alpha[(t * N + v) % T];
    be[v] = (V)cs->beta[(t * N + v) % T];
  }
  const long nv = cap / N;
  for (long i = (long)blockIdx.x * kBS + t; i < nv; i += (long)gridDim.x * kBS) {
    VT pv = reinterpret_cast<const VT*>(p)[i];
    const V* ps = reinterpret_cast<const V*>(&pv);
    if (xup) {
      VT xv = reinterpret_cast<const VT*>(x)[i];
      V* xs = reinterpret_cast<V*>(&xv);
#pragma unroll
      for (int v = 0; v < N; ++v) xs[v] += al[v] * ps[v];
      reinterpret_cast<VT*>(x)[i] = xv;
    }
    if (pup) {
      const VT zv = reinterpret_cast<const VT*>(z)[i];
      V* pw = reinterpret_cast<V*>(&pv);
      const V* zs = reinterpret_cast<const V*>(&zv);
#pragma unroll
      for (int v = 0; v < N; ++v) pw[v] = zs[v] + be[v] * pw[v];
      reinterpret_cast<VT*>(p)[i] = pv;
    }
  }
}

// Inner (FP32) solve set-up from an FP64 vector src (the outer residual or
// delta_bar): rbar = src - mean (FP64), r32 = rbar, p32 = D^-1 r32, x32 = 0,
// and q32 = 0 on the padding past n*T (the apply writes every row below n
// before q is read).  Four consecutive elements per thread, moved as 16-byte
// vectors; the grid stride is a multiple of T, so a thread's four columns
// stay the same throughout.
// The last block checks outer convergence on ||rbar|| (FP64) and starts the
// inner CG on the pairs that are still open.
__global__ __launch_bounds__(kBS) void k_inner_init_any(int T, int n, long cap, const double* src,
                                                        MeanSrc m, const float* invd32, float* x32,
                                                        float* r32, float* p32, float* q32,
                                                        double rtol2, double irtol2, int max_refine,
                                                        int first, double stall_ratio2, ColState* cs,
                                                        GridRed red) {
  constexpr int NE = 4;
  __shared__ double sh[3 * kBS * NE];
  __shared__ double vals[3 * kMaxTile];
  const int t = threadIdx.x;
  double acc[3][NE];
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int j = 0; j < NE; ++j) acc[d][j] = 0.0;
  const long nT = (long)n * T;
  const long nq = cap / NE;                 // cap is a multiple of 16
  for (long qd = (long)blockIdx.x * kBS + t; qd < nq; qd += (long)gridDim.x * kBS) {
    const double2 s01 = reinterpret_cast<const double2*>(src)[2 * qd];
    const double2 s23 = reinterpret_cast<const double2*>(src)[2 * qd + 1];
    const double sv[NE] = {s01.x, s01.y, s23.x, s23.y};
    float f[NE], z[NE];
#pragma unroll
    for (int j = 0; j < NE; ++j) {
      const long e = qd * NE + j;
      f[j] = 0.0f;
      z[j] = 0.0f;
      if (e < nT) {
        const long i = e / T;
        const double v = sv[j] - mean_of(m, i, (int)(e % T));
        f[j] = (float)v;
        z[j] = f[j] * invd32[i];             // p0 = z0 = D^-1 r0
        acc[0][j] += v * v;
        const double fd = (double)f[j];
        acc[1][j] += fd * (double)z[j];
        acc[2][j] += fd * fd;
      }
    }
    reinterpret_cast<float4*>(r32)[qd] = make_float4(f[0], f[1], f[2], f[3]);
    reinterpret_cast<float4*>(x32)[qd] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    reinterpret_cast<float4*>(p32)[qd] = make_float4(z[0], z[1], z[2], z[3]);
    if (qd * NE + NE > nT) reinterpret_cast<float4*>(q32)[qd] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  }
  block_reduce_cols<kBS, 3, NE>(acc, T, sh);
  if (t < T) {
    vals[t] = sh[t];
    vals[T + t] = sh[kBS * NE + t];
    vals[2 * T + t] = sh[2 * kBS * NE + t];
  }
  __syncthreads();
  if (!grid_reduce<kBS>(vals, 3 * T, red)) return;
  if (t < T) {
    const double rr_old = cs->orr[t];
    cs->orr[t] = vals[t];
    int act = 0;
    if (cs->oactive[t] && !first)
      cs->stall[t] = refine_stall_count(rr_old, vals[t], cs->stall[t], stall_ratio2);
    if (cs->oactive[t]) {
      if (!first && vals[t] <= rtol2 * cs->obnorm2[t]) {
        cs->oactive[t] = 0;
      } else if (refine_hand_to_fp64(cs->stall[t])) {
        cs->oactive[t] = 0;   // FP32 no longer reduces the residual: FP64 from here
        cs->fb[t] = 1;
      } else if (cs->refine[t] >= max_refine) {
        cs->oactive[t] = 0;
        cs->status[t] = kStNoconv;
      } else if (vals[2 * T + t] > 0.0) {
        act = 1;
        cs->refine[t] += 1;
      } else {
        cs->oactive[t] = 0;   // residual rounds to zero in FP32: nothing left to add
      }
    }
    cs->active[t] = act;
    cs->bnorm2[t] = vals[2 * T + t];
    cs->rho[t] = vals[T + t];
    cs->it_cur[t] = 0;
    // inner tolerance: inner_rtol, relaxed to what this step still needs
    // (a reduction to 0.3 rtol ||delta_bar|| / ||r||) when that is less
    const double need2 = vals[t] > 0.0 ? 0.09 * rtol2 * cs->obnorm2[t] / vals[t] : 0.0;
    cs->itol2[t] = need2 > irtol2 ? (need2 < 0.25 ? need2 : 0.25) : irtol2;
    cs->alpha[t] = 0.0;
    cs->beta[t] = 0.0;
  }
  if (t == 0) cs->xseq = cs->xdone = 0;
  recount_active(cs, T);
}

// x64 += x32 (x32 is zero on pairs whose inner solve did not run; pairs
// that failed keep their last good x).
template <int T>
__global__ __launch_bounds__(kBS) void k_accum(long cap, double* x64, const float* x32,
                                               const ColState* cs) {
  const int t = threadIdx.x;
  for (long e = (long)blockIdx.x * kBS + t; e < cap; e += (long)gridDim.x * kBS) {
    const int c = (int)(e % T);
    if (cs->status[c] == kStOk) x64[e] += (double)x32[e];
  }
}

// x -= mean (per component), optionally copied to the caller's X.
template <int T>
__global__ __launch_bounds__(kBS) void k_xfinal(int n, double* x64, MeanSrc m, double* X,
                                                long ldx) {
  const int t = threadIdx.x;
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * kBS + t; e < tot; e += (long)gridDim.x * kBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    const double v = x64[e] - mean_of(m, i, c);
    x64[e] = v;
    if (X) X[i * ldx + c] = v;
  }
}

// Warm start: x64 = X - mean is copied in (the caller's guess), b is kept.
template <int T>
__global__ __launch_bounds__(kBS) void k_xload(int n, double* x64, const double* X, long ldx) {
  const int t = threadIdx.x;
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * kBS + t; e < tot; e += (long)gridDim.x * kBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    x64[e] = X[i * ldx + c];
  }
}

// FP64 restart from the true residual held in r64: p = D^-1 r, q = 0,
// rho = r^T D^-1 r; CG resumes on the pairs still open.
template <int T>
__global__ __launch_bounds__(kBS) void k_restart(int n, long cap, const double* r64, double* p64,
                                                 double* q64, const double* invd, ColState* cs,
                                                 GridRed red) {
  __shared__ double sh[kBS];
  __shared__ double vals[kMaxTile];
  const int t = threadIdx.x;
  double acc[1][1] = {{0.0}};
  for (long e = (long)blockIdx.x * kBS + t; e < cap; e += (long)gridDim.x * kBS) {
    const long i = e / T;
    double z = 0.0;
    if (i < n) {
      z = r64[e] * invd[i];
      acc[0][0] += r64[e] * z;
    }
    p64[e] = z;                              // p0 = z0 = D^-1 r0
    q64[e] = 0.0;
  }
  block_reduce_cols<kBS, 1, 1>(acc, T, sh);
  if (t < T) vals[t] = sh[t];
  __syncthreads();
  if (!grid_reduce<kBS>(vals, T, red)) return;
  if (t < T) {
    cs->rho[t] = vals[t];
    cs->active[t] = cs->oactive[t] && vals[t] > 0.0;
    cs->bnorm2[t] = cs->obnorm2[t];
    cs->itol2[t] = 0.0;
    cs->it_cur[t] = 0;
    cs->alpha[t] = 0.0;
    cs->beta[t] = 0.0;
  }
  if (t == 0) cs->xseq = cs->xdone = 0;
  recount_active(cs, T);
}

// After a residual pass: open pairs are those whose true relative residual
// is still above rtol (FP64 restart logic).
__global__ void k_check(int T, double rtol2, ColState* cs) {
  const int t = threadIdx.x;
  if (t < T) {
    const double rr = cs->dots[2][t];
    cs->oactive[t] = (cs->status[t] == kStOk && cs->obnorm2[t] > 0.0 && rr > rtol2 * cs->obnorm2[t]);
  }
  recount_active(cs, T);
}

// Outer convergence right after a residual pass on a connected graph, from
// the pass's own dots: ||r - mean||^2 = r.r - n mean^2.  Closes the pairs
// that converged and those out of refinement steps, so the host can stop
// without setting up another inner solve.
__global__ void k_outer_check(int T, int n, double rtol2, int max_refine, ColState* cs) {
  const int t = threadIdx.x;
  if (t < T && cs->oactive[t]) {
    const double m = cs->dots[3][t] / (double)n;
    const double rr = cs->dots[2][t] - (double)n * m * m;
    if (rr <= rtol2 * cs->obnorm2[t]) {
      cs->oactive[t] = 0;
    } else if (cs->refine[t] >= max_refine) {
      cs->oactive[t] = 0;
      cs->status[t] = kStNoconv;
    }
  }
  recount_active(cs, T);
}

// After an inner FP32 solve: a pair whose solve ran out of iterations
// (status NOCONV from the inner CG; k_accum kept its last good x) is handed
// to the FP64 solver instead of being closed, like a stalled one.
__global__ void k_inner_failed_to_fp64(int T, int max_iter, ColState* cs) {
  const int t = threadIdx.x;
  if (t < T && cs->status[t] == kStNoconv && cs->it_cur[t] >= max_iter) {
    cs->status[t] = kStOk;
    cs->fb[t] = 1;
  }
  recount_active(cs, T);
}

// Open the pairs handed to the FP64 solver (and only those): the FP64 CG
// restarts from the true residual r = delta_bar - L x of their current x.
__global__ void k_fp64_open(int T, ColState* cs) {
  const int t = threadIdx.x;
  if (t < T) {
    cs->oactive[t] = cs->fb[t];
    if (cs->fb[t]) cs->fbdone[t] = 1;
    cs->fb[t] = 0;
  }
  recount_active(cs, T);
}

// d^2 = delta_bar^T x + x^T r from the last residual pass; d = sqrt(max(d^2, 0)).
// shift_n > 0: that pass saw x before its mean was removed (connected graph
// of shift_n nodes).  Shifting x by -m (m = sum x / n) leaves r unchanged
// (L 1 = 0) and changes delta_bar^T x by -m sum(delta_bar) = 0, so only x^T r
// changes, by -m sum(r).
__global__ void k_finish(int T, int mark_open_noconv, ColState* cs, double* d_out,
                         nvd_pair_info* info, int shift_n, int out_dsq) {
  const int t = threadIdx.x;
  if (t >= T) return;
  const double bx = cs->dots[0][t];
  double xr = cs->dots[1][t];
  if (shift_n > 0) xr -= cs->dots[4][t] / (double)shift_n * cs->dots[3][t];
  const double rr = cs->dots[2][t];
  const double bb = cs->obnorm2[t];
  double dsq = bx + xr;
  double rel = 0.0;
  if (bb > 0.0) {
    rel = sqrt(rr / bb);
  } else {
    dsq = 0.0;
  }
  int st = cs->status[t];
  if (mark_open_noconv && st == kStOk && cs->oactive[t]) st = kStNoconv;
  const double dsq0 = dsq > 0.0 ? dsq : 0.0;
  d_out[t] = out_dsq ? dsq0 : sqrt(dsq0);
  nvd_pair_info pi;
  pi.status = st;
  pi.iters = cs->iters[t];
  pi.refine_steps = cs->refine[t];
  pi.flags = cs->fbdone[t] ? NVD_INFO_FP64_FALLBACK : 0;
  pi.rel_res = rel;
  pi.dsq_plain = bb > 0.0 ? bx : 0.0;
  pi.dsq = dsq;
  info[t] = pi;
}

// delta_bar written to the caller's buffer (the stand-alone projection entry
// point); norms[c] = ||delta_bar_c||.
template <int T>
__global__ __launch_bounds__(kBS) void k_proj_out(int n, ProjSrc src, MeanSrc m, double* D,
                                                  long ldd, double* norms, GridRed red) {
  __shared__ double sh[kBS];
  __shared__ double vals[kMaxTile];
  const int t = threadIdx.x;
  double acc[1][1] = {{0.0}};
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * kBS + t; e < tot; e += (long)gridDim.x * kBS) {
    const long i = e / T;
    const int c = (int)(e % T);
    const double v = src.a[i * src.lda + c] - src.b[i * src.ldb + c] - mean_of(m, i, c);
    D[i * ldd + c] = v;
    acc[0][0] += v * v;
  }
  block_reduce_cols<kBS, 1, 1>(acc, T, sh);
  if (t < T) vals[t] = sh[t];
  __syncthreads();
  if (!grid_reduce<kBS>(vals, T, red)) return;
  if (t < T && norms) norms[t] = sqrt(vals[t]);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
#define NVD_TILE_SWITCH(T, CALL)             \
  switch (T) {                               \
    case 1: { constexpr int TT = 1; CALL; } break;   \
    case 2: { constexpr int TT = 2; CALL; } break;   \
    case 4: { constexpr int TT = 4; CALL; } break;   \
    case 8: { constexpr int TT = 8; CALL; } break;   \
    case 16: { constexpr int TT = 16; CALL; } break; \
    case 32: { constexpr int TT = 32; CALL; } break; \
    case 64: { constexpr int TT = 64; CALL; } break; \
    default: break;                          \
  }

// Blocks of the streaming kernels (grid-stride loops), and of those that end
// in a grid-wide reduction (fewer: every block adds a partial to the
// reduction's tail); build-time knobs.  Measured on a 10^6-node tile of 32
// FP32 columns: 1024 / 768 against 2048 for both took the iteration's two
// vector kernels from 5.5 to 6.0 TB/s.
#ifndef NVD_STREAM_GRID
#define NVD_STREAM_GRID 1024
#endif
#ifndef NVD_REDUCE_GRID
#define NVD_REDUCE_GRID 768
#endif

static int stream_grid(long cap) {
  long g = (cap + kBS - 1) / kBS;
  if (g > NVD_STREAM_GRID) g = NVD_STREAM_GRID;
  if (g < 1) g = 1;
  return (int)g;
}

static int reduce_grid(long cap) {
  long g = (cap + kBS - 1) / kBS;
  if (g > NVD_REDUCE_GRID) g = NVD_REDUCE_GRID;
  if (g < 1) g = 1;
  return (int)g;
}

static size_t padded_cap(int n, int T) { return (((size_t)n * T + 15) / 16) * 16; }

struct PollWords {
  int n_active, n_oactive, it_max, n_fb;
  double worst;
};
static_assert(offsetof(ColState, worst) - offsetof(ColState, n_active) == offsetof(PollWords, worst),
              "the polled words must be laid out as in ColState");

static nvd_status poll(Workspace* ws, hipStream_t s, int* n_active, int* n_oactive,
                       PollWords* all = nullptr) {
  NVD_HIP(hipMemcpyAsync(ws->h_pinned, &ws->cs->n_active, sizeof(PollWords),
                         hipMemcpyDeviceToHost, s));
  NVD_HIP(hipStreamSynchronize(s));
  const PollWords* pw = reinterpret_cast<const PollWords*>(ws->h_pinned);
  if (n_active) *n_active = pw->n_active;
  if (n_oactive) *n_oactive = pw->n_oactive;
  if (all) *all = *pw;
  return NVD_OK;
}

// The explicit preconditioner solve z = M^-1 r: the spanning forest's
// L_T^+, or the approximate-Cholesky factor's (F D F^T)^-1.
static nvd_status z_solve(DevGraph* g, const SolveParams& sp, int prec, int T, const void* r, void* z,
                          hipStream_t s) {
  return sp.achol ? achol_solve(g, prec, T, r, z, s) : tree_solve(g, prec, T, r, z, s);
}

// Start of a CG run with an explicit preconditioner solve on r: p = z =
// M^-1 r, rho = r^T z.
template <typename V>
static nvd_status tree_start(DevGraph* g, Workspace* ws, int T, const V* r, V* p,
                             const SolveParams& sp, hipStream_t s) {
  const long cap = (long)padded_cap(g->n, T);
  const int rgrid = reduce_grid(cap / Vec16<V>::N);
  NVD_TRY(z_solve(g, sp, sizeof(V) == 8 ? 0 : 1, T, r, p, s));
  NVD_TILE_SWITCH(T, (k_rz<V, TT, 0><<<rgrid, kBS, 0, s>>>(cap, r, p, ws->cs, ws->red)));
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

template <typename V>
static nvd_status cg_loop(DevGraph* g, Workspace* ws, int T, V* x, V* r, V* p, V* q,
                          const V* invd, double rtol2, int max_iter, const SolveParams& sp,
                          hipStream_t s) {
  const long cap = (long)padded_cap(g->n, T);
  const int sgrid = stream_grid(cap / Vec16<V>::N);
  const int rgrid = reduce_grid(cap / Vec16<V>::N);
  SpmmCall sc{};
  sc.g = g;
  sc.prec = sizeof(V) == 8 ? 0 : 1;
  sc.T = T;
  sc.nl = sp.nl;
  sc.grid = sp.grid;
  sc.x = p;
  sc.ldx = T;
  sc.y = q;
  sc.ldy = T;
  sc.cs = ws->cs;
  sc.epi = EPI_CG;
  const double sv = (double)sizeof(V);
  const double upd_bytes = (3.0 * T * sv + sv) * g->n;   // r, q in; r out; 1/deg
  const double dir_bytes = (5.0 * T * sv + sv) * g->n;   // x, r, p in; x, p out; 1/deg
  // Iterations are enqueued in chunks; after each chunk the host reads four
  // words (active count, largest iteration count, worst residual ratio) and
  // sizes the next chunk from the observed decay of the worst residual, so
  // that few launches run after the last column has converged.
  int done = 0;
  int chunk = 6;
  int it0 = 0;                 // it_max at the start of the chunk
  double prev_worst = -1.0;
  int prev_it = 0;
  std::vector<int> ids;
  while (done < max_iter) {
    const int todo = std::min(chunk, max_iter - done);
    ids.clear();
    for (int it = 0; it < todo; ++it) {
      NVD_TRY(launch_apply(sc, ws->red, s));
      ids.push_back(prof_last_id());
      int pid = prof_begin(s, sizeof(V) == 8 ? PK_UPD64 : PK_UPD32, upd_bytes);
      if (sp.tree) {
        NVD_TILE_SWITCH(T, (k_update<V, TT, true><<<rgrid, kBS, 0, s>>>(
                               g->n, cap, r, q, invd, rtol2, max_iter, ws->cs, ws->red)));
      } else {
        NVD_TILE_SWITCH(T, (k_update<V, TT><<<rgrid, kBS, 0, s>>>(g->n, cap, r, q, invd, rtol2,
                                                                  max_iter, ws->cs, ws->red)));
      }
      prof_end(s, pid);
      ids.push_back(pid);
      pid = prof_begin(s, sizeof(V) == 8 ? PK_DIR64 : PK_DIR32, dir_bytes);
      if (sp.tree) {
        // z = M^-1 r into q (free until the next apply), then beta and p
        NVD_TRY(z_solve(g, sp, sizeof(V) == 8 ? 0 : 1, T, r, q, s));
        NVD_TILE_SWITCH(T, (k_rz<V, TT, 1><<<rgrid, kBS, 0, s>>>(cap, r, q, ws->cs, ws->red)));
        NVD_TILE_SWITCH(T, (k_direction_z<V, TT><<<sgrid, kBS, 0, s>>>(cap, x, p, q, ws->cs)));
      } else {
        NVD_TILE_SWITCH(T, (k_direction<V, TT><<<sgrid, kBS, 0, s>>>(g->n, cap, x, p, r, invd, ws->cs)));
      }
      prof_end(s, pid);
      ids.push_back(pid);
    }
    NVD_HIP(hipGetLastError());
    done += todo;
    PollWords pw{};
    NVD_TRY(poll(ws, s, nullptr, nullptr, &pw));
    // launches past the last active iteration returned at once: not timed work
    const int ran = std::max(0, std::min(todo, pw.it_max - it0));
    for (size_t k = (size_t)ran * 3; k < ids.size(); ++k) prof_mark_idle(ids[k]);
    it0 = pw.it_max;
    if (pw.n_active == 0) break;
    int next = 8;
    if (prev_worst > 0.0 && pw.worst > 0.0 && pw.worst < prev_worst && pw.it_max > prev_it) {
      const double rate = std::log(pw.worst / prev_worst) / (double)(pw.it_max - prev_it);
      const double need = std::log(1.0 / pw.worst) / rate;   // iterations to reach ratio 1
      next = (int)std::ceil(need * 1.05) + 1;
    }
    prev_worst = pw.worst;
    prev_it = pw.it_max;
    chunk = std::max(1, std::min(next, 64));
  }
  return NVD_OK;
}

// ---------------------------------------------------------------------------
// timing of one CG iteration, for the autotuner
// ---------------------------------------------------------------------------
// The vector passes of an iteration cost more per byte once the tile's
// vectors no longer fit in the last-level cache, so the tile is chosen on
// whole iterations (apply, update, direction), not on the apply alone.  The
// iteration runs on the workspace vectors with a private column state that
// keeps every column active: r = 1, alpha = 0 (x and r stay put) and a huge
// rho (beta ~ 0, so p stays bounded), and a negative ||b||^2 so that no
// column ever counts as converged.
__global__ void k_tune_state(int T, ColState* cs) {
  const int t = threadIdx.x;
  if (t < T) {
    cs->rho[t] = 1e300;
    cs->alpha[t] = 0.0;
    cs->beta[t] = 0.0;
    cs->bnorm2[t] = -1.0;
    cs->itol2[t] = 0.0;
    cs->active[t] = 1;
    cs->oactive[t] = 1;
    cs->it_cur[t] = 0;
    cs->iters[t] = 0;
    cs->status[t] = kStOk;
  }
  if (t == 0) {
    cs->n_active = T;
    cs->n_oactive = T;
    cs->it_max = 0;
    cs->xseq = cs->xdone = 0;
  }
}

template <typename V>
__global__ void k_tune_fill(V* v, long cap, V val) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < cap; i += (long)gridDim.x * blockDim.x)
    v[i] = val;
}

template <typename V>
static nvd_status enqueue_tune_iteration(DevGraph* g, Workspace* ws, int T, int nl, ColState* tcs,
                                         hipStream_t s) {
  const long cap = (long)padded_cap(g->n, T);
  const int sgrid = stream_grid(cap / Vec16<V>::N);
  V* x;
  V* r;
  V* p;
  V* q;
  const V* invd;
  if constexpr (sizeof(V) == 8) {
    x = ws->x64; r = ws->r64; p = ws->p64; q = ws->q64; invd = g->invd64;
  } else {
    x = ws->x32; r = ws->r32; p = ws->p32; q = ws->q32; invd = g->invd32;
  }
  k_tune_state<<<1, kMaxTile, 0, s>>>(T, tcs);
  SpmmCall sc{};
  sc.g = g;
  sc.prec = sizeof(V) == 8 ? 0 : 1;
  sc.T = T;
  sc.nl = nl;
  sc.x = p;
  sc.ldx = T;
  sc.y = q;
  sc.ldy = T;
  sc.cs = tcs;
  sc.epi = EPI_PLAIN;
  NVD_TRY(launch_apply(sc, ws->red, s));
  NVD_TILE_SWITCH(T, (k_update<V, TT><<<reduce_grid(cap / Vec16<V>::N), kBS, 0, s>>>(g->n, cap, r, q, invd, 1.0,
                                                            0x7fffffff, tcs, ws->red)));
  NVD_TILE_SWITCH(T, (k_direction<V, TT><<<sgrid, kBS, 0, s>>>(g->n, cap, x, p, r, invd, tcs)));
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

template <typename V>
static nvd_status time_iteration_t(DevGraph* g, int T, int nl, hipStream_t s, float* ms) {
  Workspace* ws = g->ws;
  const long cap = (long)padded_cap(g->n, T);
  ColState* tcs = nullptr;
  NVD_HIP(hipMalloc(&tcs, sizeof(ColState)));
  hipEvent_t a = nullptr, b = nullptr;
  nvd_status st = NVD_OK;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) st = NVD_E_DEVICE;
  if (st == NVD_OK) {
    // r = 1 on the n x T tile, padding left at zero
    V* r = sizeof(V) == 8 ? (V*)ws->r64 : (V*)ws->r32;
    k_tune_fill<V><<<1024, kBS, 0, s>>>(r, (long)g->n * T, (V)1);
    st = enqueue_tune_iteration<V>(g, ws, T, nl, tcs, s);     // warm-up
  }
  const int reps = 3;
  if (st == NVD_OK && hipEventRecord(a, s) != hipSuccess) st = NVD_E_DEVICE;
  for (int i = 0; i < reps && st == NVD_OK; ++i) st = enqueue_tune_iteration<V>(g, ws, T, nl, tcs, s);
  if (st == NVD_OK && hipEventRecord(b, s) != hipSuccess) st = NVD_E_DEVICE;
  if (st == NVD_OK && hipEventSynchronize(b) != hipSuccess) st = NVD_E_DEVICE;
  float t = 0.0f;
  if (st == NVD_OK && hipEventElapsedTime(&t, a, b) != hipSuccess) st = NVD_E_DEVICE;
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  // leave the vectors zero, as allocated
  V* vs[4] = {sizeof(V) == 8 ? (V*)ws->x64 : (V*)ws->x32, sizeof(V) == 8 ? (V*)ws->r64 : (V*)ws->r32,
              sizeof(V) == 8 ? (V*)ws->p64 : (V*)ws->p32, sizeof(V) == 8 ? (V*)ws->q64 : (V*)ws->q32};
  for (V* v : vs) k_tune_fill<V><<<1024, kBS, 0, s>>>(v, cap, (V)0);
  if (hipStreamSynchronize(s) != hipSuccess && st == NVD_OK) st = NVD_E_DEVICE;
  (void)hipFree(tcs);
  *ms = t / reps;
  if (st != NVD_OK) set_error("autotuner: iteration timing failed");
  return st;
}

nvd_status time_cg_iteration(DevGraph* g, int prec, int T, int nl, hipStream_t s, float* ms) {
  return prec == 0 ? time_iteration_t<double>(g, T, nl, s, ms) : time_iteration_t<float>(g, T, nl, s, ms);
}

static nvd_status mean_into(DevGraph* g, Workspace* ws, int T, ProjSrc src, MeanSrc* m,
                            hipStream_t s) {
  *m = MeanSrc{};
  m->n = g->n;
  if (g->n_comp == 1) {
    const int grid = stream_grid((long)g->n * T);
    NVD_TILE_SWITCH(T, (k_colsum<TT><<<grid, kBS, 0, s>>>(g->n, src, ws->cs, ws->red)));
    m->colmean = ws->cs->mean;
  } else {
    const int grid = std::min(g->n_comp, 4096);
    NVD_TILE_SWITCH(T, (k_comp_mean<TT><<<grid, kBS, 0, s>>>(g->n_comp, g->comp_perm, g->comp_off,
                                                            src, ws->comp_mean)));
    m->cmean = ws->comp_mean;
    m->comp = g->comp;
  }
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

nvd_status project_tile(DevGraph* g, int T, const double* P, const double* Q, int64_t ld,
                        double* Dbar, int64_t ldd, double* norms, hipStream_t s) {
  NVD_TRY(ensure_workspace(g, T, false));
  Workspace* ws = g->ws;
  MeanSrc m{};
  NVD_TRY(mean_into(g, ws, T, ProjSrc{P, ld, Q, ld}, &m, s));
  const int grid = stream_grid((long)g->n * T);
  NVD_TILE_SWITCH(T, (k_proj_out<TT><<<grid, kBS, 0, s>>>(g->n, ProjSrc{P, ld, Q, ld}, m, Dbar, ldd,
                                                          norms, ws->red)));
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

// Solve pairs [c0, c0+T) of the caller's P, Q, in the graph's cached
// workspace (allocated or grown here).
nvd_status solve_tile(DevGraph* g, int T, const double* P, const double* Q, int64_t ld,
                      const SolveParams& sp, double* d_out, double* X, int64_t ldx,
                      nvd_pair_info* info_dev, hipStream_t s) {
  NVD_TRY(ensure_workspace(g, T, sp.precision == NVD_MIXED));
  if (sp.achol)
    NVD_TRY(ensure_achol(g));
  else if (sp.tree)
    NVD_TRY(ensure_tree(g, T));
  return solve_tile_ws(g, g->ws, T, P, Q, ld, sp, d_out, X, ldx, info_dev, s);
}

// The same in a given workspace, which must hold tile T (and the FP32
// vectors in mixed precision); allocates nothing.
nvd_status solve_tile_ws(DevGraph* g, Workspace* ws, int T, const double* P, const double* Q,
                         int64_t ld, const SolveParams& sp, double* d_out, double* X,
                         int64_t ldx, nvd_pair_info* info_dev, hipStream_t s) {
  const bool mixed = sp.precision == NVD_MIXED;
  const int n = g->n;
  const long cap = (long)padded_cap(n, T);
  const int grid = stream_grid(cap);
  const double rtol2 = sp.rtol * sp.rtol;

  // (a2) delta_bar = (P - Q) minus its per-component mean
  MeanSrc m{};
  NVD_TRY(mean_into(g, ws, T, ProjSrc{P, ld, Q, ld}, &m, s));
  NVD_TILE_SWITCH(T, (k_proj_init<TT><<<grid, kBS, 0, s>>>(
                         n, cap, ProjSrc{P, ld, Q, ld}, m, g->invd64, ws->b64, ws->x64, ws->r64,
                         ws->p64, ws->q64, mixed ? 0 : 1, ws->cs, ws->red)));
  NVD_HIP(hipGetLastError());
  if (sp.tree && !mixed) NVD_TRY(tree_start<double>(g, ws, T, ws->r64, ws->p64, sp, s));

  SpmmCall resid{};
  resid.g = g;
  resid.prec = 0;
  resid.T = T;
  resid.nl = sp.nl;
  resid.grid = sp.grid;
  resid.x = ws->x64;
  resid.ldx = T;
  resid.y = ws->r64;
  resid.ldy = T;
  resid.b = ws->b64;
  resid.ldb = T;
  resid.cs = ws->cs;
  resid.epi = EPI_RESID;

  bool have_x = false;
  if (sp.warm && X) {
    NVD_TILE_SWITCH(T, (k_xload<TT><<<grid, kBS, 0, s>>>(n, ws->x64, X, ldx)));
    NVD_HIP(hipGetLastError());
    have_x = true;
  }

  // FP64 CG from the restart state set up by the caller (k_restart, or
  // k_proj_init), then the true residual, with up to two restarts from it;
  // ends with x mean-zero and a residual pass of the final x.
  auto fp64_cg = [&]() -> nvd_status {
    int restarts = 0;
    for (;;) {
      NVD_TRY(cg_loop<double>(g, ws, T, ws->x64, ws->r64, ws->p64, ws->q64, g->invd64, rtol2,
                              sp.max_iter, sp, s));
      // x mean-zero, true residual, restart if needed
      MeanSrc mx{};
      NVD_TRY(mean_into(g, ws, T, ProjSrc{ws->x64, T, nullptr, 0}, &mx, s));
      NVD_TILE_SWITCH(T, (k_xfinal<TT><<<grid, kBS, 0, s>>>(n, ws->x64, mx, nullptr, 0)));
      NVD_TRY(launch_apply(resid, ws->red, s));
      k_check<<<1, 64, 0, s>>>(T, rtol2, ws->cs);
      NVD_HIP(hipGetLastError());
      int no = 0;
      NVD_TRY(poll(ws, s, nullptr, &no));
      if (no == 0 || restarts >= 2) break;
      ++restarts;
      NVD_TILE_SWITCH(T, (k_restart<TT><<<grid, kBS, 0, s>>>(n, cap, ws->r64, ws->p64, ws->q64,
                                                             g->invd64, ws->cs, ws->red)));
      NVD_HIP(hipGetLastError());
      if (sp.tree) NVD_TRY(tree_start<double>(g, ws, T, ws->r64, ws->p64, sp, s));
    }
    return NVD_OK;
  };

  int shift_n = 0;   // > 0: x's mean is removed after the last residual pass
  bool fp64_finish = !mixed;   // the FP64 solver ran last (open pairs are NOCONV)
  if (!mixed) {
    if (have_x) {
      // r = delta_bar - L x0, then CG from there
      NVD_TRY(launch_apply(resid, ws->red, s));
      NVD_TILE_SWITCH(T, (k_restart<TT><<<grid, kBS, 0, s>>>(n, cap, ws->r64, ws->p64, ws->q64,
                                                             g->invd64, ws->cs, ws->red)));
      NVD_HIP(hipGetLastError());
      if (sp.tree) NVD_TRY(tree_start<double>(g, ws, T, ws->r64, ws->p64, sp, s));
    }
    NVD_TRY(fp64_cg());
  } else {
    const double irtol2 = sp.inner_rtol * sp.inner_rtol;
    // NVD_REFINE_STALL_RATIO2 (in [0, 1]) replaces the stagnation rule's
    // ratio: 0 treats every outer step as stalled, which makes the hand-over
    // to the FP64 solver testable on any graph
    double stall_ratio2 = kStallRatio2;
    if (const char* e = std::getenv("NVD_REFINE_STALL_RATIO2")) {
      const double v = std::strtod(e, nullptr);
      if (v >= 0.0 && v <= 1.0) stall_ratio2 = v;
    }
    const bool connected = g->n_comp == 1;
    bool first = !have_x;
    bool resid_current = false;   // the last residual pass saw the current x
    PollWords pw{};               // the loop leaves by a break right after a poll
    bool polled = false;
    for (int step = 0; step <= sp.max_refine; ++step) {
      MeanSrc mr{};
      const double* src = ws->b64;
      if (!first) {
        // (a7) FP64 outer residual r = delta_bar - L x, projected
        NVD_TRY(launch_apply(resid, ws->red, s));
        resid_current = true;
        if (connected) {
          mr.n = n;
          mr.dots_sum = ws->cs->dots[3];
          k_outer_check<<<1, 64, 0, s>>>(T, n, rtol2, sp.max_refine, ws->cs);
          NVD_HIP(hipGetLastError());
          NVD_TRY(poll(ws, s, nullptr, nullptr, &pw));
          if (pw.n_oactive == 0) {
            polled = true;
            break;
          }
        } else {
          NVD_TRY(mean_into(g, ws, T, ProjSrc{ws->r64, T, nullptr, 0}, &mr, s));
        }
        src = ws->r64;
      }
      k_inner_init_any<<<grid, kBS, 0, s>>>(T, n, cap, src, mr, g->invd32, ws->x32, ws->r32,
                                            ws->p32, ws->q32, rtol2, irtol2, sp.max_refine,
                                            first ? 1 : 0, stall_ratio2, ws->cs, ws->red);
      NVD_HIP(hipGetLastError());
      if (sp.tree) NVD_TRY(tree_start<float>(g, ws, T, ws->r32, ws->p32, sp, s));
      if (first || !connected) {
        NVD_TRY(poll(ws, s, nullptr, nullptr, &pw));
        if (pw.n_oactive == 0) {
          polled = true;
          break;
        }
      }
      first = false;
      // (an inner set-up that closed every pair leaves nothing active: the
      // first chunk of the loop returns at once)
      NVD_TRY(cg_loop<float>(g, ws, T, ws->x32, ws->r32, ws->p32, ws->q32, g->invd32, irtol2,
                             sp.max_iter, sp, s));
      NVD_TILE_SWITCH(T, (k_accum<TT><<<grid, kBS, 0, s>>>(cap, ws->x64, ws->x32, ws->cs)));
      k_inner_failed_to_fp64<<<1, 64, 0, s>>>(T, sp.max_iter, ws->cs);
      NVD_HIP(hipGetLastError());
      resid_current = false;
    }
    // pairs on which FP32 stalled (or ran out of inner iterations) are
    // finished by the FP64 solver, from their current x (the count comes
    // with the poll that ended the loop, else a poll of its own)
    if (!polled) NVD_TRY(poll(ws, s, nullptr, nullptr, &pw));
    if (pw.n_fb > 0) {
      NVD_TRY(launch_apply(resid, ws->red, s));
      k_fp64_open<<<1, 64, 0, s>>>(T, ws->cs);
      NVD_TILE_SWITCH(T, (k_restart<TT><<<grid, kBS, 0, s>>>(n, cap, ws->r64, ws->p64, ws->q64,
                                                             g->invd64, ws->cs, ws->red)));
      NVD_HIP(hipGetLastError());
      if (sp.tree) NVD_TRY(tree_start<double>(g, ws, T, ws->r64, ws->p64, sp, s));
      NVD_TRY(fp64_cg());
      fp64_finish = true;
    } else if (connected && resid_current) {
      // the last residual pass is that of the final x: its dots give the
      // distance once x's mean is accounted for (k_finish); x itself is
      // shifted only where it is returned
      shift_n = n;
    } else {
      MeanSrc mx{};
      NVD_TRY(mean_into(g, ws, T, ProjSrc{ws->x64, T, nullptr, 0}, &mx, s));
      NVD_TILE_SWITCH(T, (k_xfinal<TT><<<grid, kBS, 0, s>>>(n, ws->x64, mx, nullptr, 0)));
      NVD_TRY(launch_apply(resid, ws->red, s));
    }
  }
  // (a8) quadratic form, distances, per-pair info; copy x out
  if (X) {
    MeanSrc xm{};
    xm.n = n;
    if (shift_n > 0) xm.dots_sum = ws->cs->dots[4];
    NVD_TILE_SWITCH(T, (k_xfinal<TT><<<grid, kBS, 0, s>>>(n, ws->x64, xm, X, ldx)));
  }
  k_finish<<<1, 64, 0, s>>>(T, fp64_finish ? 1 : 0, ws->cs, d_out, info_dev, shift_n,
                            sp.out_dsq ? 1 : 0);
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

}  // namespace nvd
