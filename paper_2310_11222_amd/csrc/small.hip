// One launch per tile for small and mid-size connected graphs: the whole
// Jacobi-PCG solve of nvd_distances (projection, CG iterations, FP64
// restarts or the mixed refinement with its stagnation guard, the quadratic
// form and the per-pair info) in one kernel, with barriers where the
// multi-kernel path has kernel boundaries and host polls.
//
// On a graph of a few thousand nodes every kernel of the multi-kernel path
// is a few microseconds of work behind a launch, and the host reads the
// convergence state between chunks of iterations: a 1e3-node solve of ~25
// iterations costs ~0.7 ms, almost all of it launch gaps and polls.
//
// Small graphs run in a single 1024-thread block.  Mid-size graphs (up to
// about a million vector elements) run as one cooperative launch of a few
// dozen such blocks that meet at grid barriers: reductions go through
// per-block partials written with coherent stores and summed in block
// order by every block, so all blocks hold the same scalars and take the
// same decisions; before a vector written by one block is gathered by
// another (p before the Laplacian apply, x before the FP64 residual) the
// barrier also releases the writer's L2 lines and invalidates the reader's.
// Waits are bounded: a barrier that gives up sets a failure word, after
// which every block leaves its loops and the pairs report NVD_E_DEVICE.
//
// Every sum has a fixed order, so results repeat bit for bit.  The
// arithmetic is that of the multi-kernel path (same recurrences, same
// stopping rules, same edge-difference form of L x), so the results agree
// up to the order of floating-point sums.
#include <algorithm>
#include <cstdlib>
#include <vector>

#include "device_common.hpp"
#include "refine_guard.hpp"

namespace nvd {

constexpr int kSmallBS = 1024;
// Vector elements (n * T) up to which the single launch is used; each thread
// holds up to kMaxEPT elements of the CG vectors in registers.  One block
// covers up to kSmallBS * kMaxEPT elements; above that, one element per
// thread while that takes at most kMidBlocksOne blocks, then kMaxEPT.
constexpr long kMidVec = 1L << 18;
// Rows with more neighbours than this are walked by a whole wave (64 lanes
// over the neighbour list, summed by shuffles in a fixed order) instead of
// one thread, so that a hub does not set the length of every phase.
constexpr int kHeavyDeg = 32;
// The single launch is used only where every row left to one thread has at
// most this many neighbours.
constexpr int kMaxThreadDeg = 64;
constexpr int kMaxEPT = 2;
constexpr int kMidBlocksOne = 128;
constexpr int kMidMaxBlocks = 256;
// Polls of a grid barrier before it gives up (a few seconds).
constexpr unsigned kMidSpinLimit = 1u << 22;

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
  // rows with more than kHeavyDeg neighbours, walked by a whole wave
  const int* heavy;    // [n_heavy] row ids
  int n_heavy;
  int heavy_deg;       // rows with more neighbours are heavy (a prefix of `heavy`)
  double* hq;          // [n][T] their q = L p (coherent stores)
  // multi-block launches only
  double* part;        // [2][blocks][kRedStride] reduction partials
  unsigned* sync;      // [0] barrier arrivals, [1] failure word
  unsigned spin_limit;
};

struct SmallState {
  double rho[kMaxTile], alpha[kMaxTile], beta[kMaxTile], bnorm2[kMaxTile], obnorm2[kMaxTile];
  double itol2[kMaxTile], orr[kMaxTile], mean[kMaxTile];
  double dots[5][kMaxTile];
  int active[kMaxTile], oactive[kMaxTile], iters[kMaxTile], it_cur[kMaxTile], status[kMaxTile];
  int refine[kMaxTile], stall[kMaxTile], fb[kMaxTile], fbdone[kMaxTile];
  int count;
  unsigned epoch;      // grid barriers passed (the same in every block)
  int failed;          // a grid barrier gave up
};

__device__ __forceinline__ long elem0() { return (long)blockIdx.x * kSmallBS + threadIdx.x; }
__device__ __forceinline__ long elem_step() { return (long)gridDim.x * kSmallBS; }

// Barrier over the whole launch (a block barrier when it is one block).
// With `fence`, vector writes of this block are released to every XCD and
// this block's caches are invalidated before it reads other blocks' writes.
__device__ __forceinline__ void small_sync(const SmallArgs& a, SmallState& S, bool fence) {
  if (gridDim.x == 1) {
    __syncthreads();
    return;
  }
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) {
    if (fence) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    S.epoch += 1;
    if (!S.failed) {
      const unsigned target = S.epoch * gridDim.x;
      __hip_atomic_fetch_add(a.sync, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      for (unsigned spins = 0;; ++spins) {
        if (__hip_atomic_load(a.sync, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
        if (__hip_atomic_load(a.sync + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
            spins >= a.spin_limit) {
          __hip_atomic_store(a.sync + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          S.failed = 1;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    if (fence) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

// Column sums of ND per-thread values: thread t holds column t % T (the
// block size is a multiple of T).  out[d * kMaxTile + c], in a fixed order:
// lanes of a wave by xor shuffles, the 16 waves in wave order, then (several
// blocks) the block sums in block order, the same in every block.  With
// `fence` the grid barrier also publishes this block's vector writes.
template <int ND, int T>
__device__ __forceinline__ void small_reduce(const double (&acc)[ND], const SmallArgs& a,
                                             SmallState& S, double* sh, double* out,
                                             bool fence = false) {
  constexpr int NW = kSmallBS / 64;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  double v[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) v[d] = acc[d];
#pragma unroll
  for (int off = 32; off >= T; off >>= 1) {
#pragma unroll
    for (int d = 0; d < ND; ++d) v[d] += __shfl_xor(v[d], off, 64);
  }
  if (lane < T) {
#pragma unroll
    for (int d = 0; d < ND; ++d) sh[(d * NW + wv) * T + lane] = v[d];
  }
  __syncthreads();
  double tot = 0.0;
  if (t < ND * T) {
    const int d = t / T, c = t % T;
    for (int w = 0; w < NW; ++w) tot += sh[(d * NW + w) * T + c];
  }
  if (gridDim.x == 1) {
    if (t < ND * T) out[(t / T) * kMaxTile + (t % T)] = tot;
    __syncthreads();
    return;
  }
  // Partials alternate between two buffers by barrier parity: a block writes
  // a buffer again only after every block has passed the barrier that
  // follows the reads of its previous contents.
  double* buf = a.part + (size_t)(S.epoch & 1u) * gridDim.x * kRedStride;
  if (t < ND * T) st_agent(&buf[(size_t)blockIdx.x * kRedStride + t], tot);
  small_sync(a, S, fence);
  double* sum = sh + kSmallBS;
  sum_rows_fixed<kSmallBS>(buf, gridDim.x, ND * T, sh, sum);
  if (t < ND * T) out[(t / T) * kMaxTile + (t % T)] = sum[t];
  __syncthreads();
}

// Number of columns whose flag is set (thread 0 counts; all threads read);
// zero once a grid barrier has failed, so that every loop ends.
__device__ __forceinline__ int small_count(SmallState& S, const int* flag, int T) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int k = 0;
    for (int c = 0; c < T; ++c) k += flag[c];
    S.count = S.failed ? 0 : k;
  }
  __syncthreads();
  return S.count;
}

// The direction of a CG iteration, p = z + beta p_old, in one rounding
// (the owner of an element and every neighbour that gathers it compute the
// same value bit for bit).
__device__ __forceinline__ float pdir(float z, float be, float po) { return __builtin_fmaf(be, po, z); }
__device__ __forceinline__ double pdir(double z, double be, double po) { return __builtin_fma(be, po, z); }

// Row i of L applied to this iteration's direction, in edge differences:
// sum_j w_ij (p_i - p_j), where every neighbour's p_j = z_j + beta p_old_j is
// formed from z and the previous direction as it is gathered, so that no
// barrier separates the direction update from the apply (p_old is not read
// when beta is zero: a fresh start, p = z).  Column indices are loaded 8 (4
// in FP64) at a time ahead of their gathers.
template <typename V, int T, bool UNIT>
__device__ __forceinline__ V small_row_apply(const SmallArgs& a, const V* __restrict__ w, int lo,
                                             int hi, int c, V pi, const V* __restrict__ z,
                                             const V* __restrict__ pold, V be) {
  constexpr int U = sizeof(V) == 8 ? 4 : 8;   // entries per step (registers)
  V sum = (V)0;
  const bool use_old = be != (V)0;
  for (int j = lo; j < hi; j += U) {
    const int m = hi - j;
    int cj[U];
    V wj[U], zj[U], oj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      cj[u] = u < m ? a.ci[j + u] : 0;
      wj[u] = UNIT ? (V)1 : (u < m ? w[j + u] : (V)0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      zj[u] = u < m ? z[(long)cj[u] * T + c] : (V)0;
      oj[u] = (u < m && use_old) ? pold[(long)cj[u] * T + c] : (V)0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (u < m) sum += wj[u] * (pi - pdir(zj[u], be, oj[u]));
  }
  return sum;
}

// Sum over the lanes of a wave (xor shuffles, fixed order; every lane gets
// the total).
template <typename V>
__device__ __forceinline__ V wave_sum(V v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Heavy rows of the CG apply: wave w of the launch takes the (row, column)
// pairs w, w + waves, ...; q goes to hq with a coherent store (its owner
// reads it after the next barrier) and p_i q_i joins the partial of p^T q
// of lane c, the lane that holds column c.  p_i is formed from z and the previous direction as the owner
// forms it.
template <typename V, int T, bool UNIT>
__device__ __forceinline__ double small_heavy_apply(const SmallArgs& a, const V* __restrict__ w,
                                                    const V* __restrict__ z,
                                                    const V* __restrict__ pold,
                                                    const SmallState& S) {
  const int lane = threadIdx.x & 63;
  const int gw = blockIdx.x * (kSmallBS / 64) + (threadIdx.x >> 6);
  const int nw = gridDim.x * (kSmallBS / 64);
  double acc = 0.0;
  for (int h = gw; h < a.n_heavy * T; h += nw) {
    const int c = h % T;
    if (!S.active[c]) continue;
    const long i = a.heavy[h / T];
    const V be = (V)S.beta[c];
    const bool use_old = be != (V)0;
    const V pi = pdir(z[i * T + c], be, use_old ? pold[i * T + c] : (V)0);
    const int lo = a.rp[i], hi = a.rp[i + 1];
    V sum = (V)0;
    for (int j = lo + lane; j < hi; j += 64) {
      const long cj = a.ci[j];
      const V pj = pdir(z[cj * T + c], be, use_old ? pold[cj * T + c] : (V)0);
      sum += (UNIT ? (V)1 : w[j]) * (pi - pj);
    }
    sum = wave_sum(sum);
    if (lane == c) {   // lane c's partials belong to column c
      st_agent(&a.hq[i * T + c], (double)sum);
      acc += (double)pi * (double)sum;
    }
  }
  return acc;
}

// r = b - L x in FP64 and its dots: b^T x, x^T r, r^T r, sum r, sum x
// (S.dots[0..4]); heavy rows are summed by waves, which add their dots to
// the partials of the lane that holds the row's column.
template <int T, bool UNIT>
__device__ __forceinline__ void small_resid(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  small_sync(a, S, true);   // x is gathered
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const long nT = (long)a.n * T;
  for (long e = elem0(); e < nT; e += elem_step()) {
    const long i = e / T;
    const int c = (int)(e % T);
    const int lo = a.rp[i], hi = a.rp[i + 1];
    if (hi - lo > a.heavy_deg) continue;
    const double xi = a.x64[e];
    double sum = 0.0;
    for (int j = lo; j < hi; ++j)
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
  {
    const int lane = threadIdx.x & 63;
    const int gw = blockIdx.x * (kSmallBS / 64) + (threadIdx.x >> 6);
    const int nw = gridDim.x * (kSmallBS / 64);
    for (int h = gw; h < a.n_heavy * T; h += nw) {
      const int c = h % T;
      const long i = a.heavy[h / T];
      const long e = i * T + c;
      const double xi = a.x64[e];
      double sum = 0.0;
      for (int j = a.rp[i] + lane; j < a.rp[i + 1]; j += 64)
        sum += (UNIT ? 1.0 : a.w64[j]) * (xi - a.x64[(long)a.ci[j] * T + c]);
      sum = wave_sum(sum);
      if (lane == c) {   // lane c's partials belong to column c
        const double bb = a.b64[e];
        const double rr = bb - sum;
        a.r64[e] = rr;
        acc[0] += bb * xi;
        acc[1] += xi * rr;
        acc[2] += rr * rr;
        acc[3] += rr;
        acc[4] += xi;
      }
    }
  }
  small_reduce<5, T>(acc, a, S, sh, red, true);   // r of heavy rows is read by their owners
  if (threadIdx.x < T) {
#pragma unroll
    for (int d = 0; d < 5; ++d) S.dots[d][threadIdx.x] = red[d * kMaxTile + threadIdx.x];
  }
  __syncthreads();
}

// x -= its column mean (one component).
template <int T>
__device__ __forceinline__ void small_center_x(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  double acc[1] = {0.0};
  const long nT = (long)a.n * T;
  for (long e = elem0(); e < nT; e += elem_step()) acc[0] += a.x64[e];
  small_reduce<1, T>(acc, a, S, sh, red);
  if (threadIdx.x < T) S.mean[threadIdx.x] = red[threadIdx.x] / (double)a.n;
  __syncthreads();
  for (long e = elem0(); e < nT; e += elem_step()) a.x64[e] -= S.mean[e % T];
  __syncthreads();
}

// CG iterations (preconditioner D) until no column is active, from x and
// r in memory and a fresh direction p = D^-1 r (rho = r^T D^-1 r set by the
// caller): as cg_loop with k_spmm (EPI_CG), k_update and k_direction, with
// each thread's EPT elements of x, r, p, z, q held in registers.  Two
// barriers per iteration: the sum p^T q (alpha), and the sums r^T z, r^T r
// (beta), whose barrier also publishes z and p for the next apply.  z lives
// in q's buffer; the directions alternate between p's and r's buffers (r is
// read once, before the first barrier).  On return x is in memory; r, p and
// q hold scratch.
template <typename V, int T, bool UNIT, int EPT>
__device__ __forceinline__ void small_cg(const SmallArgs& a, const V* w, const V* invd, V* x, V* r, V* p, V* q,
                         double rtol2, SmallState& S, double* sh, double* red) {
  const int t = threadIdx.x;
  const int c = t % T;
  const long nT = (long)a.n * T;
  V xr[EPT], rv[EPT], pr[EPT], zr[EPT], qv[EPT], id[EPT];
  long ev[EPT];
  int lo[EPT], hi[EPT];
  bool hv[EPT];
#pragma unroll
  for (int j = 0; j < EPT; ++j) {
    ev[j] = elem0() + (long)j * elem_step();
    xr[j] = rv[j] = pr[j] = zr[j] = qv[j] = id[j] = (V)0;
    lo[j] = hi[j] = 0;
    hv[j] = false;
    if (ev[j] < nT) {
      lo[j] = a.rp[ev[j] / T];
      hi[j] = a.rp[ev[j] / T + 1];
      hv[j] = hi[j] - lo[j] > a.heavy_deg;
      xr[j] = x[ev[j]];
      rv[j] = r[ev[j]];
      id[j] = invd[ev[j] / T];
      zr[j] = rv[j] * id[j];
      q[ev[j]] = zr[j];
    }
  }
  if (t < T) S.beta[t] = 0.0;
  V* const z = q;
  bool cur = false;        // directions: read p, write r; then the other way

  small_sync(a, S, true);   // z is gathered
  for (int it = 0; it < a.max_iter; ++it) {
    if (small_count(S, S.active, T) == 0) break;
    {
      const V be = (V)S.beta[c];
      const bool act = S.active[c] != 0;
      const V* pold = cur ? r : p;
      V* pnew = cur ? p : r;
      double acc[1] = {0.0};
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (act && ev[j] < nT) {
          pr[j] = pdir(zr[j], be, pr[j]);
          pnew[ev[j]] = pr[j];
          if (!hv[j]) {
            qv[j] = small_row_apply<V, T, UNIT>(a, w, lo[j], hi[j], c, pr[j], z, pold, be);
            acc[0] += (double)pr[j] * (double)qv[j];
          }
        }
      }
      if (a.n_heavy > 0) acc[0] += small_heavy_apply<V, T, UNIT>(a, w, z, pold, S);
      small_reduce<1, T>(acc, a, S, sh, red);
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
      const bool act = S.active[c] != 0;
      double acc[2] = {0.0, 0.0};
#pragma unroll
      for (int j = 0; j < EPT; ++j) {
        if (act && ev[j] < nT) {
          if (hv[j]) qv[j] = (V)ld_agent(&a.hq[ev[j]]);
          xr[j] += al * pr[j];
          rv[j] -= al * qv[j];
          zr[j] = rv[j] * id[j];
          z[ev[j]] = zr[j];
          const double rd = (double)rv[j];
          acc[0] += rd * rd * (double)id[j];
          acc[1] += rd * rd;
        }
      }
      small_reduce<2, T>(acc, a, S, sh, red, true);
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
    cur = !cur;
  }
#pragma unroll
  for (int j = 0; j < EPT; ++j)
    if (ev[j] < nT) x[ev[j]] = xr[j];
}

// FP64 CG from the restart state, then the true residual with up to two
// restarts from it; ends with x mean-zero and the residual of the final x.
template <int T, bool UNIT, int EPT>
__device__ __forceinline__ void small_fp64(const SmallArgs& a, SmallState& S, double* sh, double* red) {
  const int t = threadIdx.x;
  const long nT = (long)a.n * T;
  for (int restarts = 0;; ++restarts) {
    small_cg<double, T, UNIT, EPT>(a, a.w64, a.invd64, a.x64, a.r64, a.p64, a.q64, a.rtol2, S, sh, red);
    small_center_x<T>(a, S, sh, red);
    small_resid<T, UNIT>(a, S, sh, red);
    if (t < T)
      S.oactive[t] = S.status[t] == kStOk && S.obnorm2[t] > 0.0 && S.dots[2][t] > a.rtol2 * S.obnorm2[t];
    if (small_count(S, S.oactive, T) == 0 || restarts >= 2) break;
    // restart from the true residual: p = D^-1 r, rho = r^T D^-1 r
    double acc[1] = {0.0};
    for (long e = elem0(); e < nT; e += elem_step()) {
      const double z = a.r64[e] * a.invd64[e / T];
      a.p64[e] = z;
      acc[0] += a.r64[e] * z;
    }
    small_reduce<1, T>(acc, a, S, sh, red);
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

template <int T, bool UNIT, int EPT>
__global__ __launch_bounds__(kSmallBS) void k_small_solve(SmallArgs a) {
  __shared__ double sh[5 * kSmallBS];
  __shared__ double red[5 * kMaxTile];
  __shared__ SmallState S;
  const int t = threadIdx.x;
  const int c = t % T;
  const int n = a.n;
  const long nT = (long)n * T;
  if (t == 0) {
    S.epoch = 0u;
    S.failed = 0;
  }
  __syncthreads();
  // (a2) delta_bar = (P - Q) minus its mean (one component)
  {
    double acc[1] = {0.0};
    for (long e = elem0(); e < nT; e += elem_step()) {
      const long i = e / T;
      acc[0] += a.P[i * a.ld + c] - a.Q[i * a.ld + c];
    }
    small_reduce<1, T>(acc, a, S, sh, red);
    if (t < T) S.mean[t] = red[t] / (double)n;
    __syncthreads();
  }
  {
    const double m = S.mean[c];
    double acc[2] = {0.0, 0.0};
    for (long e = elem0(); e < nT; e += elem_step()) {
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
    small_reduce<2, T>(acc, a, S, sh, red);
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
    small_fp64<T, UNIT, EPT>(a, S, sh, red);
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
        for (long e = elem0(); e < nT; e += elem_step()) {
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
        small_reduce<3, T>(acc, a, S, sh, red);
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
      small_cg<float, T, UNIT, EPT>(a, a.w32, a.invd32, a.x32, a.r32, a.p32, a.q32, a.irtol2, S, sh, red);
      // x += c on the pairs whose inner solve ended well; a pair whose FP32
      // solve ran out of iterations goes to the FP64 solver instead
      {
        const int ok = S.status[c] == kStOk;
        for (long e = elem0(); e < nT; e += elem_step())
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
      for (long e = elem0(); e < nT; e += elem_step()) {
        const double z = a.r64[e] * a.invd64[e / T];
        a.p64[e] = z;
        acc[0] += a.r64[e] * z;
      }
      small_reduce<1, T>(acc, a, S, sh, red);
      if (t < T) {
        S.rho[t] = red[t];
        S.active[t] = S.oactive[t] && red[t] > 0.0;
        S.bnorm2[t] = S.obnorm2[t];
        S.itol2[t] = 0.0;
        S.it_cur[t] = 0;
      }
      __syncthreads();
      small_fp64<T, UNIT, EPT>(a, S, sh, red);
      fp64_finish = true;
    } else {
      small_center_x<T>(a, S, sh, red);
      small_resid<T, UNIT>(a, S, sh, red);
    }
  }
  // (a8) quadratic form, distances, per-pair info; x out
  if (a.X) {
    for (long e = elem0(); e < nT; e += elem_step()) a.X[(e / T) * a.ldx + (e % T)] = a.x64[e];
  }
  if (blockIdx.x == 0 && t < T) {
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
    if (S.failed) st = NVD_E_DEVICE;
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

// Heavy rows: those above kHeavyDeg neighbours (NVD_SMALL_HEAVY_DEG),
// longest first, built once per graph.
static nvd_status ensure_heavy(DevGraph* g) {
  int base = kHeavyDeg;
  if (const char* e = std::getenv("NVD_SMALL_HEAVY_DEG")) base = std::max(1, std::atoi(e));
  if (g->n_heavy >= 0 && g->heavy_base == base) return NVD_OK;
  if (g->heavy) (void)hipFree(g->heavy);
  g->heavy = nullptr;
  g->n_heavy = -1;
  std::vector<int> hv;
  for (int i = 0; i < g->n; ++i)
    if (g->h_rp[i + 1] - g->h_rp[i] > base) hv.push_back(i);
  auto deg = [&](int i) { return g->h_rp[i + 1] - g->h_rp[i]; };
  std::stable_sort(hv.begin(), hv.end(), [&](int x, int y) { return deg(x) > deg(y); });
  g->heavy_deg_desc.resize(hv.size());
  for (size_t q = 0; q < hv.size(); ++q) g->heavy_deg_desc[q] = deg(hv[q]);
  if (!hv.empty()) {
    NVD_HIP(hipMalloc((void**)&g->heavy, sizeof(int) * hv.size()));
    NVD_HIP(hipMemcpy(g->heavy, hv.data(), sizeof(int) * hv.size(), hipMemcpyHostToDevice));
  }
  g->n_heavy = (int)hv.size();
  g->heavy_base = base;
  return NVD_OK;
}

// The heavy rows of one launch: no more than one (row, column) pair per
// wave -- where many rows are long (dense graphs) only the longest are
// walked by waves.  The threshold is the degree of the first row left out,
// so that the rows above it are exactly a prefix of the list.
static void heavy_plan(const DevGraph* g, int nb, int T, int* heavy_deg, int* n_heavy) {
  *heavy_deg = g->heavy_base;
  *n_heavy = g->n_heavy;
  const int kmax = std::max(1, nb * (kSmallBS / 64) / T);
  if (g->n_heavy > kmax) {
    *heavy_deg = g->heavy_deg_desc[kmax];
    int h = 0;
    while (h < g->n_heavy && g->heavy_deg_desc[h] > *heavy_deg) ++h;
    *n_heavy = h;
  }
}

int small_blocks(DevGraph* g, int T, const SolveParams& sp) {
  if (g->n_comp != 1 || sp.tree || sp.achol || sp.warm) return 0;
  const char* e = std::getenv("NVD_SMALL");
  if (e && e[0] == '0') return 0;
  const long nT = (long)g->n * T;
  long mid_max = kMidVec;
  if (const char* m = std::getenv("NVD_MID_MAX_VEC")) mid_max = std::strtol(m, nullptr, 10);
  if (nT > std::min(mid_max, (long)kSmallBS * kMaxEPT * kMidMaxBlocks)) return 0;
  long nb;
  if (const char* b = std::getenv("NVD_MID_BLOCKS")) {
    nb = std::max(1L, std::strtol(b, nullptr, 10));
  } else {
    const long per_block = nT <= (long)kSmallBS * kMaxEPT ? (long)kSmallBS * kMaxEPT : kSmallBS;
    nb = (nT + per_block - 1) / per_block;
    if (nb > kMidBlocksOne) nb = (nT + (long)kSmallBS * kMaxEPT - 1) / ((long)kSmallBS * kMaxEPT);
  }
  if (nb > kMidMaxBlocks || nT > nb * (long)kSmallBS * kMaxEPT) return 0;
  // rows not walked by waves are walked by one thread each: beyond
  // kMaxThreadDeg neighbours the multi-kernel apply (lane groups per row)
  // is faster
  if (ensure_heavy(g) != NVD_OK) return 0;
  int heavy_deg = 0, n_heavy = 0;
  heavy_plan(g, (int)nb, T, &heavy_deg, &n_heavy);
  if (heavy_deg > kMaxThreadDeg && std::getenv("NVD_MID_BLOCKS") == nullptr) return 0;
  return (int)nb;
}

__global__ void k_small_reset(unsigned* sync) {
  if (threadIdx.x < 2) sync[threadIdx.x] = 0u;
}

// Blocks of k_small_solve<T, UNIT, EPT> that fit on the device at once.
template <int T, bool UNIT, int EPT>
static int small_resident() {
  static int cached = -1;
  if (cached >= 0) return cached;
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_small_solve<T, UNIT, EPT>), kSmallBS, 0) !=
          hipSuccess)
    return 0;
  cached = per_cu * cus;
  return cached;
}

template <int T, bool UNIT, int EPT>
static nvd_status launch_small_ept(const SmallArgs& a0, int nb, unsigned* sync, hipStream_t s) {
  SmallArgs a = a0;
  if (nb <= 1) {
    k_small_solve<T, UNIT, EPT><<<1, kSmallBS, 0, s>>>(a);
    NVD_HIP(hipGetLastError());
    return NVD_OK;
  }
  if (nb > small_resident<T, UNIT, EPT>()) {
    set_error("small solve: the multi-block launch does not fit on the device");
    return NVD_E_UNSUPPORTED;
  }
  k_small_reset<<<1, 64, 0, s>>>(sync);
  NVD_HIP(hipGetLastError());
  void* params[] = {&a};
  NVD_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_small_solve<T, UNIT, EPT>),
                                     dim3(nb), dim3(kSmallBS), params, 0, s));
  return NVD_OK;
}

// Elements per thread: the fewest register slots that cover n T with nb
// blocks (small_blocks guarantees that kMaxEPT do).
template <int T, bool UNIT>
static nvd_status launch_small(const SmallArgs& a, int nb, unsigned* sync, hipStream_t s) {
  const long nT = (long)a.n * T;
  if (nT <= (long)nb * kSmallBS) return launch_small_ept<T, UNIT, 1>(a, nb, sync, s);
  static_assert(kMaxEPT == 2, "one instantiation per register slot count");
  return launch_small_ept<T, UNIT, 2>(a, nb, sync, s);
}

nvd_status solve_small(DevGraph* g, int T, int nb, const double* P, const double* Q, int64_t ld,
                       const SolveParams& sp, double* d_out, double* X, int64_t ldx,
                       nvd_pair_info* info_dev, hipStream_t s) {
  const bool mixed = sp.precision == NVD_MIXED;
  NVD_TRY(ensure_workspace(g, T, mixed));
  Workspace* ws = g->ws;
  int heavy_deg = 0, n_heavy = 0;
  NVD_TRY(ensure_heavy(g));
  heavy_plan(g, nb, T, &heavy_deg, &n_heavy);
  if (g->n_heavy > 0 && !ws->hq) {
    NVD_HIP(hipMalloc((void**)&ws->hq, sizeof(double) * ws->cap_rows));
    ws->bytes += (int64_t)(sizeof(double) * ws->cap_rows);
    g->bytes += (int64_t)(sizeof(double) * ws->cap_rows);
  }
  SmallArgs a{};
  a.heavy = g->heavy;
  a.n_heavy = n_heavy;
  a.heavy_deg = heavy_deg;
  a.hq = ws->hq;
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
  a.part = ws->red.part1;
  a.sync = ws->msync;
  a.spin_limit = kMidSpinLimit;
  if (const char* e = std::getenv("NVD_MID_SPIN_LIMIT")) a.spin_limit = (unsigned)std::strtoul(e, nullptr, 10);
  const bool unit = !g->weighted;
#define NVD_SMALL_T(TT)                                                                  \
  case TT:                                                                               \
    return unit ? launch_small<TT, true>(a, nb, ws->msync, s)                            \
                : launch_small<TT, false>(a, nb, ws->msync, s);
  switch (T) {
    NVD_SMALL_T(1) NVD_SMALL_T(2) NVD_SMALL_T(4) NVD_SMALL_T(8) NVD_SMALL_T(16) NVD_SMALL_T(32)
    NVD_SMALL_T(64)
    default:
      set_error("small solve: tile must be a power of two up to 64");
      return NVD_E_ARG;
  }
#undef NVD_SMALL_T
}

}  // namespace nvd
