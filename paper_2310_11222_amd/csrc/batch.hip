// Batched distances: many graphs of uneven size, each with its own vector
// pairs, solved in ONE persistent cooperative launch (FP32 CG with FP64
// iterative refinement, or FP64 CG).
//
// Work plan (host, per call): blocks are resident for the whole launch.
// Graphs whose estimated work exceeds a block's fair share get a team of
// blocks of their own; each team member owns a row range balanced by
// rows + nonzeros, and the team meets at atomic barriers (bounded spins).
// All other graphs sit in a pool ordered by decreasing size, and single blocks
// take them one at a time from an atomic counter; blocks whose team has
// finished join the pool, so the launch drains without idle tails.
//
// Inside a team, the vectors other members gather (p of the inner CG, x of
// the outer residual) are written and read with agent-scope (coherent)
// accesses; team reductions go through a double-buffered scratch summed in
// rank order, so every member derives identical scalars and takes identical
// branches.  A graph solved by a single block uses plain accesses and
// __syncthreads only.
//
// Per graph and pair (the paper's section 3.1 distance through the solve of
// section 3.2): delta = p - q, mean removed (graphs in a batch are
// connected), FP64 outer residual r = delta_bar - L x, inner CG on
// L c = r - mean(r), x += c, and finally x made mean-zero and
// d^2 = delta_bar^T x + x^T (delta_bar - L x) in FP64.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "batch_internal.hpp"
#include "device_common.hpp"

namespace nvd {

constexpr int BBS = 512;                 // threads per block of the batched kernel
constexpr unsigned kSpinLimit = 1u << 26;  // bounded barrier wait (seconds), then give up

struct BGraph {
  int n, k, nnz, weighted;
  long rp_off;       // packed row pointers (n+1 local offsets)
  long nnz_off;      // packed col_idx / weights
  long v_off;        // packed vectors (n*T)
  long in_off;       // caller's P, Q, X (n*k, leading dimension k)
  int out_off;       // d_out / info (k entries)
  int long_off, n_long;  // packed list of rows with more than kLongRow neighbours
};

struct BatchArgs {
  int G, T, B;
  const BGraph* gd;
  const int* rp;
  const int* ci;
  const double* w64;
  const float* w32;
  const double* invd64;
  const float* invd32;
  const int* long_rows;
  double* b64;
  double* x64;
  double* r64;
  void* cv;   // inner vectors, V = float (mixed) or double (fp64)
  void* rv;
  void* pv;
  void* qv;
  const int* team_of_block;   // [B]
  const int* team_first;      // [nteams]
  const int* team_size;       // [nteams]
  const int* team_graph;      // [nteams] (-1: pooled single block)
  const int* pool;            // pooled graphs, largest first
  int n_pool;
  unsigned* pool_next;
  unsigned* team_ctr;         // [nteams]
  double* part;               // [2][B][kRedStride]
  const double* P;
  const double* Q;
  double* d_out;
  double* X;
  nvd_pair_info* info;
  double rtol2, irtol2;
  int max_iter, max_refine;
  int* err;
  unsigned spin_limit;        // polls of a team barrier before it gives up
  unsigned long long* trace;  // [2G] start/end wall-clock ticks per graph, or null
};

template <bool SH, typename V>
__device__ __forceinline__ V vld(const V* p) {
  if constexpr (SH)
    return __hip_atomic_load(const_cast<V*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    return *p;
}
template <bool SH, typename V>
__device__ __forceinline__ void vst(V* p, V v) {
  if constexpr (SH)
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  else
    *p = v;
}

struct Team {
  int S, rank, first;
  unsigned* ctr;
  unsigned epoch;
  double* part;
  int B;
  int parity;
  int* err;
  unsigned spin_limit;
};

// The launch's failure word: set by a barrier wait that gave up.  Once it is
// set every barrier returns at once and every solve loop exits, so the
// kernel ends after a bounded amount of work and the host reports the
// failure (the outputs of that call are then meaningless).
__device__ __forceinline__ bool team_failed(const Team& tm) {
  return __hip_atomic_load(tm.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

__device__ __forceinline__ void team_sync(Team& tm) {
  if (tm.S == 1) {
    __syncthreads();
    return;
  }
  wait_stores();
  __syncthreads();
  tm.epoch += 1;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(tm.ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = tm.epoch * (unsigned)tm.S;
    // at most spin_limit polls (0: give up at once, which makes the
    // failure path testable), and none once the launch has failed
    for (unsigned spins = 0;; ++spins) {
      if (spins >= tm.spin_limit) {
        __hip_atomic_store(tm.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      if (__hip_atomic_load(tm.ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target ||
          team_failed(tm))
        break;
      __builtin_amdgcn_s_sleep(2);
    }
  }
  __syncthreads();
}

// Team-wide sums of vals[0..ndt) (block sums on entry, team sums on exit).
__device__ __forceinline__ void team_reduce(Team& tm, double* vals, int ndt) {
  if (tm.S == 1) return;
  double* buf = tm.part + (size_t)tm.parity * tm.B * kRedStride;
  tm.parity ^= 1;
  for (int i = threadIdx.x; i < ndt; i += BBS)
    st_agent(&buf[(size_t)(tm.first + tm.rank) * kRedStride + i], vals[i]);
  team_sync(tm);
  double s = 0.0;
  const int i = threadIdx.x;
  if (i < ndt)
    for (int q = 0; q < tm.S; ++q) s += ld_agent(&buf[(size_t)(tm.first + q) * kRedStride + i]);
  __syncthreads();
  if (i < ndt) vals[i] = s;
  __syncthreads();
}

// Block sums by column of ND per-thread values (column t % T), then team sums.
template <int ND>
__device__ __forceinline__ void reduce_cols(Team& tm, double (&acc)[ND][1], int T, double* sh,
                                            double* vals) {
  block_reduce_cols<BBS, ND, 1>(acc, T, sh);
  if ((int)threadIdx.x < T) {
#pragma unroll
    for (int d = 0; d < ND; ++d) vals[d * T + threadIdx.x] = sh[d * BBS + threadIdx.x];
  }
  __syncthreads();
  team_reduce(tm, vals, ND * T);
}

// Column sums of ND dots when thread t holds N consecutive columns
// (t*N + v) % T, T a multiple of N: lanes holding the same columns are
// combined by shuffles, then the 8 waves' sums in wave order (fixed order).
// Needs 8*ND*T doubles of sh; result in vals[d*T + c].
template <int ND, int N>
__device__ __forceinline__ void block_reduce_vec(double (&acc)[ND][N], int T, double* sh,
                                                 double* vals) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int L = T / N;            // lanes with distinct column sets
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int v = 0; v < N; ++v) {
      double x = acc[d][v];
      for (int off = L; off < 64; off <<= 1) x += __shfl_xor(x, off, 64);
      acc[d][v] = x;
    }
  if (lane < L) {
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int v = 0; v < N; ++v) sh[(wave * ND + d) * T + lane * N + v] = acc[d][v];
  }
  __syncthreads();
  if (t < T) {
#pragma unroll
    for (int d = 0; d < ND; ++d) {
      double s = 0.0;
      for (int w = 0; w < BBS / 64; ++w) s += sh[(w * ND + d) * T + t];
      vals[d * T + t] = s;
    }
  }
  __syncthreads();
}

// Lane layout of the block SpMM: G = T*NL lanes per row; R rows carried at
// once per lane group (4 for the FP32 inner SpMM, 2 for the FP64 residual;
// more rows spill registers at 4 waves per SIMD); MB gathers per lane per
// batch.
template <int T, typename V = float>
struct BLanes {
  static constexpr int NL = T >= 16 ? 1 : (T == 8 ? 2 : (T == 4 ? 4 : 8));
  static constexpr int G = T * NL;
  static constexpr int R = sizeof(V) == 4 ? 4 : 2;
  static constexpr int MB = 4;
};

// Working storage of one block (kernel-level LDS, shared by both code paths).
struct Lds {
  double* sh;        // [4*BBS]
  double* sh_long;   // [BBS]
  double* vals;      // [4*kMaxTile]
  double *rho, *alpha, *beta, *bn2, *obn2, *mean, *itol2;   // [kMaxTile] each
  int *act, *oact, *it, *itc, *ref, *stat;          // [kMaxTile] each
  int* cnt;          // [2]: active, open
};

// Thread 0 folds the launch's failure word into a loop count (callers
// __syncthreads before reading it): a failed launch leaves its loops.
__device__ __forceinline__ int unless_failed(const Team& tm, int count) {
  return team_failed(tm) ? 0 : count;
}

// Laplacian apply on rows [lo, hi) of one graph.
//   EPI_CG:    y = L x (V), acc[0] += x.y          (x = p, y = q)
//   EPI_RESID: y = b - L x (double), acc = {sum y, y.y, b.x, x.y}
// Short rows: groups of G = T*NL lanes, R rows per group at once, neighbour
// indices loaded G at a time and shuffled out so gathers issue back to back.
template <typename V, int T, bool SH, int EPI, int ND>
__device__ __noinline__ void block_spmm(const BatchArgs& a, const BGraph& gd, int lo, int hi, const V* x,
                           V* y, const double* b, double (&acc)[ND][1], double* sh_long) {
  using LN = BLanes<T, V>;
  constexpr int NL = LN::NL;
  constexpr int G = LN::G;
  constexpr int R = LN::R;
  constexpr int RW = 64 / G;
  constexpr int MM = G / NL;
  constexpr int MB = MM < LN::MB ? MM : LN::MB;
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int g = lane / G;
  const int li = lane % G;
  const int c = li % T;
  const int j = li / T;
  const int* rp = a.rp + gd.rp_off;
  const int* ci = a.ci + gd.nnz_off;
  const bool unit = !gd.weighted;
  const V* wv = nullptr;
  if constexpr (sizeof(V) == 8)
    wv = reinterpret_cast<const V*>(a.w64 + gd.nnz_off);
  else
    wv = reinterpret_cast<const V*>(a.w32 + gd.nnz_off);
  constexpr int ROWS_PER_WAVE = RW * R;
  constexpr int ROWS_PER_STEP = (BBS / 64) * ROWS_PER_WAVE;
  for (int base = lo; base < hi; base += ROWS_PER_STEP) {
    int row[R], rs[R], deg[R];
    bool mine[R];
    V own[R];
    double bb[R];
    int maxdeg = 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      row[r] = base + wave * ROWS_PER_WAVE + r * RW + g;
      rs[r] = 0;
      deg[r] = -1;
      if (row[r] < hi) {
        rs[r] = rp[row[r]];
        deg[r] = rp[row[r] + 1] - rs[r];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      mine[r] = deg[r] >= 0 && deg[r] <= kLongRow;
      own[r] = mine[r] ? vld<SH>(&x[(long)row[r] * T + c]) : (V)0;
      bb[r] = 0.0;
      if constexpr (EPI == EPI_RESID) bb[r] = mine[r] ? b[(long)row[r] * T + c] : 0.0;
      if (!mine[r]) deg[r] = 0;
      maxdeg = deg[r] > maxdeg ? deg[r] : maxdeg;
    }
    V sum[R];
#pragma unroll
    for (int r = 0; r < R; ++r) sum[r] = (V)0;
    for (int off = 0; off < maxdeg; off += G) {
      int myc[R], cnt[R];
      V myw[R];
      int maxcnt = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        cnt[r] = deg[r] - off;
        cnt[r] = cnt[r] < 0 ? 0 : (cnt[r] > G ? G : cnt[r]);
        myc[r] = li < cnt[r] ? ci[rs[r] + off + li] : 0;
        myw[r] = unit ? (V)1 : (li < cnt[r] ? wv[rs[r] + off + li] : (V)0);
        maxcnt = cnt[r] > maxcnt ? cnt[r] : maxcnt;
      }
#pragma unroll
      for (int m0 = 0; m0 < MM; m0 += MB) {
        if (NL * m0 >= maxcnt) break;
        V xv[R][MB], ww[R][MB];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int m = 0; m < MB; ++m) {
            const int idx = j + NL * (m0 + m);
            const int col = __shfl(myc[r], idx, G);
            ww[r][m] = __shfl(myw[r], idx, G);
            // a slot past the row's end takes the row's own value: its
            // difference, whatever its weight, is zero
            xv[r][m] = idx < cnt[r] ? vld<SH>(&x[(long)col * T + c]) : own[r];
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int m = 0; m < MB; ++m) sum[r] += ww[r][m] * (own[r] - xv[r][m]);
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
#pragma unroll
      for (int off = T; off < G; off <<= 1) sum[r] += __shfl_xor(sum[r], off, 64);
    }
    if (j == 0) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (!mine[r]) continue;
        const V yv = sum[r];
        if constexpr (EPI == EPI_CG) {
          y[(long)row[r] * T + c] = yv;
          acc[0][0] += (double)own[r] * (double)yv;
        } else {
          const double rr = bb[r] - (double)yv;
          y[(long)row[r] * T + c] = (V)rr;
          acc[0][0] += rr;
          acc[1][0] += rr * rr;
          acc[2][0] += bb[r] * (double)own[r];
          acc[3][0] += (double)own[r] * rr;
        }
      }
    }
  }
  // rows with many neighbours: the whole block, BBS/T lanes per column
  const int* lr = a.long_rows + gd.long_off;
  constexpr int NJ = BBS / T;
  for (int q = 0; q < gd.n_long; ++q) {
    const int row = lr[q];
    if (row < lo || row >= hi) continue;      // uniform across the block
    const int rs = rp[row], re = rp[row + 1];
    const V xr = vld<SH>(&x[(long)row * T + t % T]);
    V sum = (V)0;
    for (int e = rs + t / T; e < re; e += NJ)
      sum += (unit ? (V)1 : wv[e]) * (xr - vld<SH>(&x[(long)ci[e] * T + t % T]));
    double part[1][1] = {{(double)sum}};
    block_reduce_cols<BBS, 1, 1>(part, T, sh_long);
    if (t < T) {
      const V own = vld<SH>(&x[(long)row * T + t]);
      const V yv = (V)sh_long[t];
      if constexpr (EPI == EPI_CG) {
        y[(long)row * T + t] = yv;
        acc[0][0] += (double)own * (double)yv;
      } else {
        const double bb = b[(long)row * T + t];
        const double rr = bb - (double)yv;
        y[(long)row * T + t] = (V)rr;
        acc[0][0] += rr;
        acc[1][0] += rr * rr;
        acc[2][0] += bb * (double)own;
        acc[3][0] += (double)own * rr;
      }
    }
    __syncthreads();
  }
}

// Row range of member `rank` of a team of S: balanced by rows + nonzeros.
__device__ __forceinline__ int split_row(const int* rp, int n, int rank, int S) {
  if (rank <= 0) return 0;
  if (rank >= S) return n;
  const long total = (long)rp[n] + n;
  const long target = total * rank / S;
  int lo = 0, hi = n;     // first row r with rp[r] + r >= target
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((long)rp[mid] + mid >= target)
      hi = mid;
    else
      lo = mid + 1;
  }
  return lo;
}

// Streaming loop over the block's elements e in [e0, e1) (row-major, T
// columns).  Single-block graphs use 16-byte vectors when T is a multiple of
// the vector width; shared (team) vectors use coherent scalar accesses.
template <typename V, int T, bool SH>
struct Stream {
  static constexpr int N = Vec16<V>::N;
  static constexpr bool VEC = !SH && (T % N == 0);
};

template <int T, typename V, bool SH>
__device__ __noinline__ void solve_graph(const BatchArgs& a, int gi, Team& tm, const Lds& L) {
  const BGraph gd = a.gd[gi];
  const int t = threadIdx.x;
  const int n = gd.n;
  if (a.trace && tm.rank == 0 && t == 0) a.trace[2 * gi] = wall_clock64();
  const int* rp = a.rp + gd.rp_off;
  const int lo = split_row(rp, n, tm.rank, tm.S);
  const int hi = split_row(rp, n, tm.rank + 1, tm.S);
  const long vo = gd.v_off;
  double* b64 = a.b64 + vo;
  double* x64 = a.x64 + vo;
  double* r64 = a.r64 + vo;
  V* cv = reinterpret_cast<V*>(a.cv) + vo;
  V* rv = reinterpret_cast<V*>(a.rv) + vo;
  V* pv = reinterpret_cast<V*>(a.pv) + vo;
  V* qv = reinterpret_cast<V*>(a.qv) + vo;
  const V* invd;
  if constexpr (sizeof(V) == 8)
    invd = reinterpret_cast<const V*>(a.invd64 + vo / T);
  else
    invd = reinterpret_cast<const V*>(a.invd32 + vo / T);
  const int k = gd.k;
  const double* Pg = a.P + gd.in_off;
  const double* Qg = a.Q + gd.in_off;
  double* sh = L.sh;
  double* vals = L.vals;
  // scalar element loop: thread t takes column c = t % T (BBS is a multiple of T)
  const int c = t % T;
  const long e0 = (long)lo * T + t;
  const long e1 = (long)hi * T;
  constexpr int STEP = BBS;

  // (1) delta = P - Q and its mean
  {
    double acc[1][1] = {{0.0}};
    for (long e = e0; e < e1; e += STEP) {
      const long i = e / T;
      const double d = c < k ? Pg[i * k + c] - Qg[i * k + c] : 0.0;
      b64[e] = d;
      acc[0][0] += d;
    }
    reduce_cols<1>(tm, acc, T, sh, vals);
    if (t < T) L.mean[t] = vals[t] / (double)n;
    __syncthreads();
  }
  // (2) delta_bar, ||delta_bar||^2, x = 0
  {
    double acc[1][1] = {{0.0}};
    const double mc = L.mean[c];
    for (long e = e0; e < e1; e += STEP) {
      const double v = b64[e] - mc;
      b64[e] = v;
      vst<SH>(&x64[e], 0.0);
      acc[0][0] += v * v;
    }
    reduce_cols<1>(tm, acc, T, sh, vals);
    if (t < T) {
      L.obn2[t] = vals[t];
      L.oact[t] = (t < k && vals[t] > 0.0) ? 1 : 0;
      L.it[t] = 0;
      L.ref[t] = 0;
      L.stat[t] = kStOk;
    }
    __syncthreads();
  }
  // (3) refinement
  for (int step = 0; step <= a.max_refine; ++step) {
    if (step > 0) {
      double acc[4][1] = {{0.0}, {0.0}, {0.0}, {0.0}};
      block_spmm<double, T, SH, EPI_RESID, 4>(a, gd, lo, hi, x64, r64, b64, acc, L.sh_long);
      reduce_cols<4>(tm, acc, T, sh, vals);
      if (t < T) {
        const double m = vals[t] / (double)n;
        L.mean[t] = m;
        const double rr = vals[T + t] - (double)n * m * m;   // ||r - mean||^2
        if (L.oact[t] && rr <= a.rtol2 * L.obn2[t]) L.oact[t] = 0;
      }
      __syncthreads();
    }
    if (t == 0) {
      int no = 0;
      for (int q = 0; q < T; ++q) {
        if (L.oact[q] && L.ref[q] >= a.max_refine) {
          L.oact[q] = 0;
          L.stat[q] = kStNoconv;
        }
        no += L.oact[q];
      }
      L.cnt[1] = unless_failed(tm, no);
    }
    __syncthreads();
    if (L.cnt[1] == 0) break;
    // inner set-up from r (or delta_bar on the first step)
    {
      double acc[2][1] = {{0.0}, {0.0}};
      const double mc = step > 0 ? L.mean[c] : 0.0;
      const bool open = L.oact[c] != 0;
      const double* src = step > 0 ? r64 : b64;
      for (long e = e0; e < e1; e += STEP) {
        const long i = e / T;
        const V rvv = open ? (V)(src[e] - mc) : (V)0;
        const V z = rvv * invd[i];
        rv[e] = rvv;
        cv[e] = (V)0;
        vst<SH>(&pv[e], z);
        acc[0][0] += (double)rvv * (double)z;
        acc[1][0] += (double)rvv * (double)rvv;
      }
      reduce_cols<2>(tm, acc, T, sh, vals);
      if (t < T) {
        L.rho[t] = vals[t];
        L.bn2[t] = vals[T + t];
        L.act[t] = (L.oact[t] && vals[T + t] > 0.0) ? 1 : 0;
        L.itc[t] = 0;
        if (L.oact[t]) L.ref[t] += 1;
        // inner tolerance relaxed to what this step still needs
        const double need2 = vals[T + t] > 0.0 ? 0.09 * a.rtol2 * L.obn2[t] / vals[T + t] : 0.0;
        L.itol2[t] = need2 > a.irtol2 ? (need2 < 0.25 ? need2 : 0.25) : a.irtol2;
      }
      __syncthreads();
    }
    // inner CG
    for (int it = 0; it < a.max_iter; ++it) {
      if (t == 0) {
        int na = 0;
        for (int q = 0; q < T; ++q) na += L.act[q];
        L.cnt[0] = unless_failed(tm, na);
      }
      __syncthreads();
      if (L.cnt[0] == 0) break;
      {
        double acc[1][1] = {{0.0}};
        block_spmm<V, T, SH, EPI_CG, 1>(a, gd, lo, hi, pv, qv, nullptr, acc, L.sh_long);
        reduce_cols<1>(tm, acc, T, sh, vals);
        if (t < T) {
          double al = 0.0;
          if (L.act[t]) {
            const double sg = vals[t];
            if (!(sg > 0.0) || !isfinite(sg)) {
              L.act[t] = 0;
              L.oact[t] = 0;
              L.stat[t] = kStBreak;
            } else {
              al = L.rho[t] / sg;
            }
          }
          L.alpha[t] = al;
        }
        __syncthreads();
      }
      {
        using S = Stream<V, T, SH>;
        constexpr int N = S::N;
        double acc[2][N];
#pragma unroll
        for (int v = 0; v < N; ++v) acc[0][v] = acc[1][v] = 0.0;
        if constexpr (S::VEC) {
          // U vectors per thread per pass: all loads issued before any use
          using VT = typename Vec16<V>::type;
          constexpr int U = 2;
          V al[N];
#pragma unroll
          for (int v = 0; v < N; ++v) al[v] = (V)L.alpha[(t * N + v) % T];
          const long i1 = (long)hi * T / N;
          // (c += alpha p is left to the direction phase, which reads p anyway)
          const VT* __restrict__ Q4 = reinterpret_cast<const VT*>(qv);
          VT* __restrict__ R4 = reinterpret_cast<VT*>(rv);
          for (long i0 = t; i0 < i1; i0 += (long)U * BBS) {
            VT qvv[U], rvv[U];
            V iv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const long i = i0 + (long)u * BBS;
              if (i < i1) {
                qvv[u] = Q4[i];
                rvv[u] = R4[i];
                iv[u] = invd[(i * N) / T];     // T >= N: one row per vector
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const long i = i0 + (long)u * BBS;
              if (i < i1) {
                V* qs = reinterpret_cast<V*>(&qvv[u]);
                V* rs = reinterpret_cast<V*>(&rvv[u]);
#pragma unroll
                for (int v = 0; v < N; ++v) {
                  rs[v] -= al[v] * qs[v];
                  const double rd = (double)rs[v];
                  acc[0][v] += rd * rd * (double)iv[u];
                  acc[1][v] += rd * rd;
                }
                R4[i] = rvv[u];
              }
            }
          }
        } else {
          const V al = (V)L.alpha[c];
          for (long e = e0; e < e1; e += STEP) {
            const long i = e / T;
            const V re = rv[e] - al * qv[e];
            rv[e] = re;
            const double rd = (double)re;
            acc[0][0] += rd * rd * (double)invd[i];
            acc[1][0] += rd * rd;
          }
        }
        // fold the N entries of a thread onto its columns, then reduce
        double acc1[2][1];
        if constexpr (S::VEC) {
          // vectors are used only by single-block graphs (lo = 0), so thread
          // t's entry v is column (t*N + v) % T
          block_reduce_vec<2, N>(acc, T, sh, vals);
          (void)acc1;
        } else {
          acc1[0][0] = acc[0][0];
          acc1[1][0] = acc[1][0];
          reduce_cols<2>(tm, acc1, T, sh, vals);
        }
        if (t < T) {
          double be = 0.0;
          if (L.act[t]) {
            const double rz = vals[t], rr = vals[T + t];
            L.it[t] += 1;
            L.itc[t] += 1;
            if (rr <= L.itol2[t] * L.bn2[t]) {
              L.act[t] = 0;
            } else if (L.itc[t] >= a.max_iter) {
              L.act[t] = 0;
            } else if (!(rz > 0.0) || !isfinite(rz)) {
              L.act[t] = 0;
              L.oact[t] = 0;
              L.stat[t] = kStBreak;
            } else {
              be = rz / L.rho[t];
              L.rho[t] = rz;
            }
          }
          L.beta[t] = be;
        }
        __syncthreads();
      }
      {
        using S = Stream<V, T, SH>;
        constexpr int N = S::N;
        if constexpr (S::VEC) {
          using VT = typename Vec16<V>::type;
          constexpr int U = 2;
          V al[N], be[N];
#pragma unroll
          for (int v = 0; v < N; ++v) {
            al[v] = (V)L.alpha[(t * N + v) % T];
            be[v] = (V)L.beta[(t * N + v) % T];
          }
          const long i1 = (long)hi * T / N;
          VT* __restrict__ P4 = reinterpret_cast<VT*>(pv);
          VT* __restrict__ C4 = reinterpret_cast<VT*>(cv);
          const VT* __restrict__ R4 = reinterpret_cast<const VT*>(rv);
          for (long i0 = t; i0 < i1; i0 += (long)U * BBS) {
            VT pvv[U], rvv[U], cvv[U];
            V iv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const long i = i0 + (long)u * BBS;
              if (i < i1) {
                pvv[u] = P4[i];
                rvv[u] = R4[i];
                cvv[u] = C4[i];
                iv[u] = invd[(i * N) / T];
              }
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
              const long i = i0 + (long)u * BBS;
              if (i < i1) {
                V* ps = reinterpret_cast<V*>(&pvv[u]);
                V* cs = reinterpret_cast<V*>(&cvv[u]);
                const V* rs = reinterpret_cast<const V*>(&rvv[u]);
#pragma unroll
                for (int v = 0; v < N; ++v) {
                  cs[v] += al[v] * ps[v];      // this iteration's step, old p
                  ps[v] = rs[v] * iv[u] + be[v] * ps[v];
                }
                C4[i] = cvv[u];
                P4[i] = pvv[u];
              }
            }
          }
        } else {
          const V al = (V)L.alpha[c];
          const V be = (V)L.beta[c];
          for (long e = e0; e < e1; e += STEP) {
            const long i = e / T;
            const V pe = vld<SH>(&pv[e]);
            cv[e] = cv[e] + al * pe;
            vst<SH>(&pv[e], rv[e] * invd[i] + be * pe);
          }
        }
        team_sync(tm);
      }
    }
    // x += c (FP64)
    for (long e = e0; e < e1; e += STEP) {
      if (L.stat[c] == kStOk) vst<SH>(&x64[e], vld<SH>(&x64[e]) + (double)cv[e]);
    }
    team_sync(tm);
  }
  // (4) x mean-zero, final FP64 residual and quadratic form
  {
    double acc[1][1] = {{0.0}};
    for (long e = e0; e < e1; e += STEP) acc[0][0] += vld<SH>(&x64[e]);
    reduce_cols<1>(tm, acc, T, sh, vals);
    if (t < T) L.mean[t] = vals[t] / (double)n;
    __syncthreads();
    const double mc = L.mean[c];
    for (long e = e0; e < e1; e += STEP) vst<SH>(&x64[e], vld<SH>(&x64[e]) - mc);
    team_sync(tm);
  }
  {
    double acc[4][1] = {{0.0}, {0.0}, {0.0}, {0.0}};
    block_spmm<double, T, SH, EPI_RESID, 4>(a, gd, lo, hi, x64, r64, b64, acc, L.sh_long);
    reduce_cols<4>(tm, acc, T, sh, vals);
  }
  if (tm.rank == 0 && t < k) {
    const double bb = L.obn2[t];
    const double bx = vals[2 * T + t], xr = vals[3 * T + t], rr = vals[T + t];
    double dsq = bb > 0.0 ? bx + xr : 0.0;
    a.d_out[gd.out_off + t] = sqrt(dsq > 0.0 ? dsq : 0.0);
    nvd_pair_info pi;
    pi.status = team_failed(tm) ? (int)NVD_E_DEVICE : L.stat[t];
    pi.iters = L.it[t];
    pi.refine_steps = L.ref[t];
    pi.flags = 0;
    pi.rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    pi.dsq_plain = bb > 0.0 ? bx : 0.0;
    pi.dsq = dsq;
    a.info[gd.out_off + t] = pi;
  }
  if (a.X) {
    for (long e = e0; e < e1; e += STEP) {
      const long i = e / T;
      if (c < k) a.X[gd.in_off + i * k + c] = vld<SH>(&x64[e]);
    }
  }
  if (a.trace && tm.rank == 0 && t == 0) a.trace[2 * gi + 1] = wall_clock64();
  __syncthreads();
}

template <int T, typename V>
__global__ __launch_bounds__(BBS, 4) void k_batch(BatchArgs a) {
  __shared__ double lds_d[4 * BBS + BBS + 4 * kMaxTile + 7 * kMaxTile];
  __shared__ int lds_i[6 * kMaxTile + 2];
  __shared__ int s_unit;
  Lds L;
  L.sh = lds_d;
  L.sh_long = lds_d + 4 * BBS;
  L.vals = L.sh_long + BBS;
  L.rho = L.vals + 4 * kMaxTile;
  L.alpha = L.rho + kMaxTile;
  L.beta = L.alpha + kMaxTile;
  L.bn2 = L.beta + kMaxTile;
  L.obn2 = L.bn2 + kMaxTile;
  L.mean = L.obn2 + kMaxTile;
  L.itol2 = L.mean + kMaxTile;
  L.act = lds_i;
  L.oact = lds_i + kMaxTile;
  L.it = lds_i + 2 * kMaxTile;
  L.itc = lds_i + 3 * kMaxTile;
  L.ref = lds_i + 4 * kMaxTile;
  L.stat = lds_i + 5 * kMaxTile;
  L.cnt = lds_i + 6 * kMaxTile;
  const int b = blockIdx.x;
  const int team = a.team_of_block[b];
  int gi = a.team_graph[team];
  Team tm;
  tm.S = a.team_size[team];
  tm.first = a.team_first[team];
  tm.rank = b - tm.first;
  tm.ctr = a.team_ctr + team;
  tm.epoch = 0;
  tm.part = a.part;
  tm.B = a.B;
  tm.parity = 0;
  tm.err = a.err;
  tm.spin_limit = a.spin_limit;
  if (gi >= 0) {
    if (tm.S > 1)
      solve_graph<T, V, true>(a, gi, tm, L);
    else
      solve_graph<T, V, false>(a, gi, tm, L);
  }
  // then the pool, one graph per block
  Team solo = tm;
  solo.S = 1;
  solo.rank = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned u = __hip_atomic_fetch_add(a.pool_next, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_unit = u < (unsigned)a.n_pool ? a.pool[u] : -1;
    }
    __syncthreads();
    const int u = s_unit;
    __syncthreads();
    if (u < 0) break;
    solve_graph<T, V, false>(a, u, solo, L);
  }
}

__global__ void k_batch_reset(unsigned* ctr, int nteams, unsigned* pool_next, int* err) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nteams) ctr[i] = 0u;
  if (i == 0) {
    *pool_next = 0u;
    *err = 0;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BatchPlan {
  int B = 0, nteams = 0;
  std::vector<int> team_of_block, team_first, team_size, team_graph, pool;
};

}  // namespace nvd

using namespace nvd;

extern "C" {

nvd_status nvd_batch_create(int32_t G, nvd_graph* const* graphs, void* stream, nvd_batch** out) {
  set_error("");
  if (!out || G < 1 || !graphs) {
    set_error("nvd_batch_create: bad argument");
    return NVD_E_ARG;
  }
  *out = nullptr;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  nvd_batch* b = new nvd_batch();
  b->G = G;
  b->it_est.assign(G, 20.0);
  for (int i = 0; i < G; ++i) {
    if (!graphs[i]) {
      delete b;
      set_error("nvd_batch_create: NULL graph");
      return NVD_E_ARG;
    }
    const DevGraph* g = graphs[i]->g;
    if (g->n_comp != 1) {
      delete b;
      set_error("nvd_batch_create: graph " + std::to_string(i) +
                " is not connected; batches take connected graphs (solve others with nvd_distances)");
      return NVD_E_UNSUPPORTED;
    }
    b->n.push_back(g->n);
    b->nnz.push_back(g->nnz);
    b->weighted.push_back(g->weighted ? 1 : 0);
    b->any_weighted |= g->weighted;
    b->rp_off.push_back(b->tot_rp);
    b->nnz_off.push_back(b->tot_nnz);
    b->node_off.push_back(b->tot_n);
    int nl = 0;
    for (int r = 0; r < g->n; ++r)
      if (g->h_rp[r + 1] - g->h_rp[r] > kLongRow) ++nl;
    b->long_off.push_back((int)b->tot_long);
    b->n_long.push_back(nl);
    b->tot_rp += g->n + 1;
    b->tot_nnz += g->nnz;
    b->tot_n += g->n;
    b->tot_long += nl;
  }
  if (b->tot_nnz >= INT32_MAX || b->tot_n >= INT32_MAX) {
    delete b;
    set_error("nvd_batch_create: packed sizes must stay below 2^31");
    return NVD_E_UNSUPPORTED;
  }
  nvd_status st = NVD_OK;
  auto chk = [&](nvd_status x) {
    if (st == NVD_OK) st = x;
  };
  chk(balloc(b, &b->rp, b->tot_rp));
  chk(balloc(b, &b->ci, b->tot_nnz));
  if (b->any_weighted) {
    chk(balloc(b, &b->w64, b->tot_nnz));
    chk(balloc(b, &b->w32, b->tot_nnz));
  }
  chk(balloc(b, &b->invd64, b->tot_n));
  chk(balloc(b, &b->invd32, b->tot_n));
  chk(balloc(b, &b->long_rows, b->tot_long));
  std::vector<int> lrows;
  lrows.reserve(b->tot_long);
  for (int i = 0; i < G && st == NVD_OK; ++i) {
    const DevGraph* g = graphs[i]->g;
    auto cp = [&](void* dst, const void* src, size_t bytes) {
      if (st == NVD_OK && bytes && hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) {
        set_error("nvd_batch_create: copy failed");
        st = NVD_E_DEVICE;
      }
    };
    cp(b->rp + b->rp_off[i], g->rp, sizeof(int) * (g->n + 1));
    cp(b->ci + b->nnz_off[i], g->ci, sizeof(int) * g->nnz);
    if (b->any_weighted) {
      if (g->weighted) {
        cp(b->w64 + b->nnz_off[i], g->w64, sizeof(double) * g->nnz);
        cp(b->w32 + b->nnz_off[i], g->w32, sizeof(float) * g->nnz);
      }
    }
    cp(b->invd64 + b->node_off[i], g->invd64, sizeof(double) * g->n);
    cp(b->invd32 + b->node_off[i], g->invd32, sizeof(float) * g->n);
    for (int r = 0; r < g->n; ++r)
      if (g->h_rp[r + 1] - g->h_rp[r] > kLongRow) lrows.push_back(r);
  }
  b->h_long_rows = lrows;
  if (st == NVD_OK && !lrows.empty() &&
      hipMemcpyAsync(b->long_rows, lrows.data(), sizeof(int) * lrows.size(), hipMemcpyHostToDevice, s) != hipSuccess)
    st = NVD_E_DEVICE;
  chk(balloc(b, &b->gd, G));
  chk(balloc(b, &b->pool_next, 1));
  chk(balloc(b, &b->err, 1));
  if (st == NVD_OK && hipHostMalloc((void**)&b->h_err, sizeof(int), hipHostMallocDefault) != hipSuccess)
    st = NVD_E_NOMEM;
  if (st == NVD_OK && hipStreamSynchronize(s) != hipSuccess) st = NVD_E_DEVICE;
  if (st != NVD_OK) {
    batch_free(b);
    delete b;
    return st;
  }
  *out = b;
  return NVD_OK;
}

nvd_status nvd_batch_destroy(nvd_batch* b) {
  if (!b) return NVD_OK;
  (void)hipDeviceSynchronize();
  batch_free(b);
  delete b;
  return NVD_OK;
}

}  // extern "C"

namespace nvd {

template <int T, typename V>
static nvd_status launch_batch(nvd_batch* b, const BatchArgs& a, hipStream_t s) {
  BatchArgs args = a;
  void* params[] = {&args};
  hipError_t e = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_batch<T, V>),
                                            dim3(a.B), dim3(BBS), params, 0, s);
  if (e != hipSuccess) {
    set_error(std::string("batched launch: ") + hipGetErrorString(e));
    return NVD_E_DEVICE;
  }
  return NVD_OK;
}

template <int T, typename V>
static int resident_blocks() {
  int dev = 0, per_cu = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&k_batch<T, V>), BBS, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// Teams for graphs above a block's fair share (up to three quarters of the
// blocks), the rest pooled largest first.
static BatchPlan make_plan(const nvd_batch* b, const std::vector<int>& ks, int T, int B) {
  BatchPlan pl;
  const int G = b->G;
  std::vector<double> w(G);
  double W = 0.0;
  for (int i = 0; i < G; ++i) {
    // per-iteration traffic x iterations (measured on the previous call)
    w[i] = (ks[i] > 0) ? ((double)b->nnz[i] + 3.0 * b->n[i]) * T * (b->it_est[i] + 4.0) : 0.0;
    W += w[i];
  }
  std::vector<int> order(G);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return w[x] > w[y]; });
  const double share = W / std::max(B, 1);
  int used = 0;
  std::vector<int> big;
  for (int gi : order) {
    if (w[gi] <= share) break;
    int S = (int)std::ceil(w[gi] / share);
    S = std::min(S, 64);
    if (used + S > (3 * B) / 4) break;
    big.push_back(gi);
    pl.team_graph.push_back(gi);
    pl.team_first.push_back(used);
    pl.team_size.push_back(S);
    for (int q = 0; q < S; ++q) pl.team_of_block.push_back((int)pl.team_first.size() - 1);
    used += S;
  }
  for (int bb = used; bb < B; ++bb) {
    pl.team_graph.push_back(-1);
    pl.team_first.push_back(bb);
    pl.team_size.push_back(1);
    pl.team_of_block.push_back((int)pl.team_first.size() - 1);
  }
  std::vector<char> isbig(G, 0);
  for (int gi : big) isbig[gi] = 1;
  for (int gi : order)
    if (!isbig[gi] && ks[gi] > 0) pl.pool.push_back(gi);
  pl.B = B;
  pl.nteams = (int)pl.team_first.size();
  return pl;
}

template <int T, typename V>
static nvd_status run_batch(nvd_batch* b, const std::vector<int>& ks, const double* P,
                            const double* Q, const nvd_opts& o, double* d_out, double* X,
                            nvd_pair_info* info_host, hipStream_t s) {
  const int G = b->G;
  const int B = std::min(resident_blocks<T, V>(), 2048);
  if (B < 1) {
    set_error("batched solver: no resident blocks");
    return NVD_E_DEVICE;
  }
  // workspace
  const size_t vsz = sizeof(V);
  if (b->cap_T < T || b->cap_vsize < (int)vsz) {
    void* ptrs[] = {b->b64, b->x64, b->r64, b->cv, b->rv, b->pv, b->qv};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    const size_t ne = (size_t)b->tot_n * T;
    NVD_TRY(balloc(b, &b->b64, ne));
    NVD_TRY(balloc(b, &b->x64, ne));
    NVD_TRY(balloc(b, &b->r64, ne));
    NVD_HIP(hipMalloc(&b->cv, ne * vsz));
    NVD_HIP(hipMalloc(&b->rv, ne * vsz));
    NVD_HIP(hipMalloc(&b->pv, ne * vsz));
    NVD_HIP(hipMalloc(&b->qv, ne * vsz));
    b->cap_T = T;
    b->cap_vsize = (int)vsz;
  }
  if (!b->part) NVD_TRY(balloc(b, &b->part, (size_t)2 * 2048 * kRedStride));
  int K = 0;
  std::vector<BGraph> gd(G);
  long in_off = 0;
  for (int i = 0; i < G; ++i) {
    BGraph& d = gd[i];
    d.n = b->n[i];
    d.k = ks[i];
    d.nnz = b->nnz[i];
    d.weighted = b->weighted[i];
    d.rp_off = b->rp_off[i];
    d.nnz_off = b->nnz_off[i];
    d.v_off = b->node_off[i] * T;
    d.in_off = in_off;
    d.out_off = K;
    d.long_off = b->long_off[i];
    d.n_long = b->n_long[i];
    in_off += (long)d.n * d.k;
    K += d.k;
  }
  if (b->info_cap < K) {
    if (b->info) (void)hipFree(b->info);
    NVD_TRY(balloc(b, &b->info, K));
    b->info_cap = K;
  }
  BatchPlan pl = make_plan(b, ks, T, B);
  std::vector<long> key = {T, (long)sizeof(V), (long)(intptr_t)P, (long)(intptr_t)Q,
                           (long)(intptr_t)d_out, (long)(intptr_t)X, B, o.max_iter, o.max_refine,
                           (long)std::llround(std::log10(o.rtol) * 1e6),
                           (long)std::llround(std::log10(o.inner_rtol) * 1e6)};
  key.insert(key.end(), ks.begin(), ks.end());
  const size_t plan_ints = (size_t)B + 3 * pl.nteams + pl.pool.size() + pl.nteams;
  if ((size_t)b->plan_cap < plan_ints) {
    if (b->plan_buf) (void)hipFree(b->plan_buf);
    NVD_TRY(balloc(b, &b->plan_buf, plan_ints));
    b->plan_cap = (int)plan_ints;
  }
  std::vector<int> hp;
  hp.reserve(plan_ints);
  hp.insert(hp.end(), pl.team_of_block.begin(), pl.team_of_block.end());
  hp.insert(hp.end(), pl.team_first.begin(), pl.team_first.end());
  hp.insert(hp.end(), pl.team_size.begin(), pl.team_size.end());
  hp.insert(hp.end(), pl.team_graph.begin(), pl.team_graph.end());
  hp.insert(hp.end(), pl.pool.begin(), pl.pool.end());
  hp.resize(plan_ints, 0);   // team counters follow (as unsigned)
  // the plan's sizes are baked into a captured launch: part of its key
  key.push_back(pl.nteams);
  key.push_back((long)pl.pool.size());
  key.insert(key.end(), hp.begin(), hp.end());
  NVD_HIP(hipMemcpyAsync(b->plan_buf, hp.data(), sizeof(int) * plan_ints, hipMemcpyHostToDevice, s));
  NVD_HIP(hipMemcpyAsync(b->gd, gd.data(), sizeof(BGraph) * G, hipMemcpyHostToDevice, s));
  int* pb = b->plan_buf;
  BatchArgs a{};
  a.G = G;
  a.T = T;
  a.B = B;
  a.gd = b->gd;
  a.rp = b->rp;
  a.ci = b->ci;
  a.w64 = b->w64;
  a.w32 = b->w32;
  a.invd64 = b->invd64;
  a.invd32 = b->invd32;
  a.long_rows = b->long_rows;
  a.b64 = b->b64;
  a.x64 = b->x64;
  a.r64 = b->r64;
  a.cv = b->cv;
  a.rv = b->rv;
  a.pv = b->pv;
  a.qv = b->qv;
  a.team_of_block = pb;
  a.team_first = pb + B;
  a.team_size = pb + B + pl.nteams;
  a.team_graph = pb + B + 2 * pl.nteams;
  a.pool = pb + B + 3 * pl.nteams;
  a.n_pool = (int)pl.pool.size();
  a.team_ctr = reinterpret_cast<unsigned*>(pb + B + 3 * pl.nteams + pl.pool.size());
  a.pool_next = b->pool_next;
  a.part = b->part;
  a.P = P;
  a.Q = Q;
  a.d_out = d_out;
  a.X = X;
  a.info = b->info;
  a.rtol2 = o.rtol * o.rtol;
  const bool mixed = o.precision == NVD_MIXED;
  a.irtol2 = mixed ? o.inner_rtol * o.inner_rtol : o.rtol * o.rtol;
  a.max_iter = o.max_iter;
  a.max_refine = mixed ? o.max_refine : std::max(2, std::min(o.max_refine, 3));
  a.err = b->err;
  // NVD_BATCH_SPIN_LIMIT: polls of a team barrier before it gives up (0 makes
  // the first barrier of a multi-block team fail: the failure path can then
  // be tested without a stalled team)
  a.spin_limit = kSpinLimit;
  if (const char* sl = std::getenv("NVD_BATCH_SPIN_LIMIT")) {
    const long v = std::strtol(sl, nullptr, 10);
    if (v >= 0 && v < (long)kSpinLimit) a.spin_limit = (unsigned)v;
    key.push_back((int)a.spin_limit);
  }
  const char* tr = std::getenv("NVD_BATCH_TRACE");
  if (tr && tr[0] == '1') {
    if (!b->trace) NVD_TRY(balloc(b, &b->trace, (size_t)2 * G));
    a.trace = b->trace;
    key.push_back(1);
  } else {
    a.trace = nullptr;
  }
  b->last_team_size.assign(G, 1);
  for (int q = 0; q < pl.nteams; ++q)
    if (pl.team_graph[q] >= 0) b->last_team_size[pl.team_graph[q]] = pl.team_size[q];
  // the launch sequence: counters reset by a kernel (no memset node), then
  // the persistent kernel
  auto enqueue = [&](hipStream_t q) -> nvd_status {
    k_batch_reset<<<(pl.nteams + 255) / 256, 256, 0, q>>>(a.team_ctr, pl.nteams, b->pool_next,
                                                          b->err);
    NVD_HIP(hipGetLastError());
    return launch_batch<T, V>(b, a, q);
  };
  const char* ge = std::getenv("NVD_BATCH_GRAPH");
  const bool use_graph = !(ge && ge[0] == '0') && !b->capture_failed;
  bool done = false;
  if (use_graph) {
    if (b->gexec && b->key == key) {
      NVD_HIP(hipGraphLaunch(b->gexec, s));
      ++b->replays;
      done = true;
    } else {
      batch_drop_graph(b);
      if (!b->cap_stream) NVD_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
      // the device plan was copied on s: make the capture stream wait for it
      NVD_HIP(hipStreamSynchronize(s));
      hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
      nvd_status st = e == hipSuccess ? enqueue(b->cap_stream) : NVD_E_DEVICE;
      hipGraph_t gr = nullptr;
      hipError_t e2 = hipStreamEndCapture(b->cap_stream, &gr);
      if (st == NVD_OK && e == hipSuccess && e2 == hipSuccess && gr) {
        if (hipGraphInstantiate(&b->gexec, gr, nullptr, nullptr, 0) == hipSuccess) {
          b->graph = gr;
          b->key = key;
          ++b->captures;
          NVD_HIP(hipGraphLaunch(b->gexec, s));
          done = true;
        } else {
          (void)hipGraphDestroy(gr);
        }
      } else if (gr) {
        (void)hipGraphDestroy(gr);
      }
      if (!done) {
        b->capture_failed = true;     // fall back to direct launches from now on
        (void)hipGetLastError();
      }
    }
  }
  if (!done) {
    NVD_TRY(enqueue(s));
    ++b->eager;
  }
  NVD_HIP(hipMemcpyAsync(b->h_err, b->err, sizeof(int), hipMemcpyDeviceToHost, s));
  if (info_host)
    NVD_HIP(hipMemcpyAsync(info_host, b->info, sizeof(nvd_pair_info) * K, hipMemcpyDeviceToHost, s));
  NVD_HIP(hipStreamSynchronize(s));
  if (*b->h_err) {
    set_error("batched solver: a team barrier timed out (blocks not co-resident?)");
    return NVD_E_DEVICE;
  }
  if (info_host) {
    int off = 0;
    for (int i = 0; i < G; ++i) {
      int itmax = 0;
      for (int j = 0; j < ks[i]; ++j) itmax = std::max(itmax, info_host[off + j].iters);
      if (itmax > 0) b->it_est[i] = itmax;
      off += ks[i];
    }
  }
  return NVD_OK;
}

}  // namespace nvd

extern "C" nvd_status nvd_batch_trace(const nvd_batch* b, int32_t G, int64_t* start_end,
                                      int32_t* team_size) {
  if (!b || !start_end || !team_size || G != b->G) {
    set_error("nvd_batch_trace: bad argument");
    return NVD_E_ARG;
  }
  if (!b->trace) {
    set_error("nvd_batch_trace: no trace recorded (set NVD_BATCH_TRACE=1 before the call)");
    return NVD_E_ARG;
  }
  NVD_HIP(hipMemcpy(start_end, b->trace, sizeof(int64_t) * 2 * G, hipMemcpyDeviceToHost));
  for (int i = 0; i < G; ++i) team_size[i] = b->last_team_size.empty() ? 1 : b->last_team_size[i];
  return NVD_OK;
}

extern "C" nvd_status nvd_batch_query(const nvd_batch* b, int64_t* captures, int64_t* replays,
                                      int64_t* eager) {
  if (!b || !captures || !replays || !eager) {
    set_error("nvd_batch_query: NULL argument");
    return NVD_E_ARG;
  }
  *captures = b->captures;
  *replays = b->replays;
  *eager = b->eager;
  return NVD_OK;
}

extern "C" nvd_status nvd_batch_distances(nvd_batch* b, const int32_t* k_per_graph,
                                          const double* P, const double* Q,
                                          const nvd_opts* opts, double* d_out, double* X_out,
                                          nvd_pair_info* info, void* stream) {
  set_error("");
  if (!b || !k_per_graph || !P || !Q || !d_out) {
    set_error("nvd_batch_distances: bad argument");
    return NVD_E_ARG;
  }
  nvd_opts o;
  nvd_opts_default(&o);
  o.precision = NVD_MIXED;
  o.rtol = 1e-8;
  if (opts) o = *opts;
  if (o.precision != NVD_FP64 && o.precision != NVD_MIXED) {
    set_error("nvd_batch_distances: bad precision");
    return NVD_E_ARG;
  }
  if (o.flags & (NVD_PRECOND_TREE | NVD_PRECOND_ACHOL)) {
    set_error("nvd_batch_distances: the tree preconditioner is not available for batches");
    return NVD_E_UNSUPPORTED;
  }
  if (!(o.rtol > 0 && o.rtol < 1 && o.inner_rtol > 0 && o.inner_rtol < 1) || o.max_iter < 1 ||
      o.max_refine < 1) {
    set_error("nvd_batch_distances: bad tolerances or iteration limits");
    return NVD_E_ARG;
  }
  std::vector<int> ks(b->G);
  int kmax = 0, K = 0;
  for (int i = 0; i < b->G; ++i) {
    ks[i] = k_per_graph[i];
    if (ks[i] < 1 || ks[i] > kMaxTile) {
      set_error("nvd_batch_distances: k_per_graph entries must be in 1..64");
      return NVD_E_ARG;
    }
    kmax = std::max(kmax, ks[i]);
    K += ks[i];
  }
  int T = 1;
  while (T < kmax) T *= 2;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  std::vector<nvd_pair_info> hinfo(K);
  nvd_status st = NVD_E_UNSUPPORTED;
  const bool mixed = o.precision == NVD_MIXED;
  if (!(o.flags & NVD_BATCH_PERSISTENT)) {
    st = run_sweep(b, ks, T, o, P, Q, d_out, X_out, hinfo.data(), s);
    T = 0;    // skip the persistent solver below
  }
#define NVD_BT(TT)                                                                          \
  case TT:                                                                                  \
    st = mixed ? run_batch<TT, float>(b, ks, P, Q, o, d_out, X_out, hinfo.data(), s)        \
               : run_batch<TT, double>(b, ks, P, Q, o, d_out, X_out, hinfo.data(), s);      \
    break;
  switch (T) {
    NVD_BT(1) NVD_BT(2) NVD_BT(4) NVD_BT(8) NVD_BT(16) NVD_BT(32) NVD_BT(64)
    default: break;   // T == 0: solved by the sweep
  }
#undef NVD_BT
  if (st != NVD_OK) return st;
  nvd_status agg = NVD_OK;
  for (int j = 0; j < K; ++j) {
    if (hinfo[j].status == NVD_E_BREAKDOWN) agg = NVD_E_BREAKDOWN;
    else if (hinfo[j].status == NVD_E_NOCONV && agg == NVD_OK) agg = NVD_E_NOCONV;
  }
  if (info) std::copy(hinfo.begin(), hinfo.end(), info);
  return agg;
}
