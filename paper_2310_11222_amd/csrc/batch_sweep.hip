// Batched distances, sweep solver: the graphs of a batch are one
// block-diagonal Laplacian, and every phase of the solve (apply, update,
// direction, projection, refinement) is one kernel that sweeps the rows of
// all graphs still open with the whole GPU.  Each graph keeps its own CG
// scalars per pair (the recurrences of the paper's section 3.2 solve are
// independent per graph and pair); only the passes over memory are shared.
//
// Rows are cut into chunks of at most kChunkRows rows of one graph (plus one
// chunk per row with more than kLongRow neighbours, applied by a whole
// block).  A block reduces its chunk's dot products, publishes them with
// coherent stores, and takes a ticket on the graph's arrival counter; the
// graph's last chunk to arrive sums all of the graph's chunk partials in
// chunk order (so results repeat bit for bit) and updates the graph's
// scalars.  Chunks of graphs that are done are skipped, so later iterations
// cost only what the open graphs need.
//
// Precision: FP32 inner CG with FP64 outer refinement (MIXED), or FP64 inner
// CG with residual restarts (FP64), as in the single-graph solver; the
// distance is d^2 = delta_bar^T x + x^T (delta_bar - L x) in FP64.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <cmath>
#include <vector>

#include "batch_internal.hpp"
#include "device_common.hpp"

namespace nvd {

constexpr int SBS = 256;          // threads per block of the sweep kernels
#ifndef NVD_CHUNK_ROWS
#define NVD_CHUNK_ROWS 1024
#endif
constexpr int kChunkRows = NVD_CHUNK_ROWS;   // rows per short chunk
// Blocks per sweep kernel at most.  One block per chunk is best measured:
// the dispatcher then balances the uneven chunk costs (long rows, skipped
// graphs) better than a grid-stride loop.
constexpr int kSweepGrid = 1 << 20;

struct SGraph {
  int n, k, weighted, first, nshort, nlong, out_off, pad;
  long rp_off, nnz_off, node_off, in_off;
};

// Per (graph, column) state, index g*T + c, and per-graph flags.
struct SState {
  double *rho, *alpha, *beta, *bn2, *obn2, *mean, *itol2;
  double* xm;        // mean of x seen by the graph's last residual pass
  int *act, *oact, *it, *itc, *ref, *stat;
  int* g_act;        // graph has an inner CG column running
  int* g_oact;       // graph has a pair not yet converged
  int* n_act;        // [2]: totals of act and oact (polled by the host)
  unsigned* tick;    // per-graph chunk arrival counters
  // c += alpha p runs in ks_direction for the iteration whose ks_update ran
  // on the graph: the graph's last chunk there advances xseq; a ks_update
  // that finds the graph inactive (and ks_accum) set xdone = xseq.
  int* xseq;
  int* xdone;
};

struct SArgs {
  int G, T, n_chunks, pstride;
  int xfirst[8], xcount[8];   // chunk range of each XCD's graphs
  const SGraph* sg;
  const int* ch_graph;
  const int* ch_lo;
  const int* ch_hi;      // -1: chunk is the single long row ch_lo
  const int* rp;
  const int* ci;
  const double* w64;
  const float* w32;
  const double* invd64;
  const float* invd32;
  double* b64;
  double* x64;
  double* r64;
  void* cv;
  void* rv;
  void* pv;
  void* qv;
  double* part;
  SState s;
  const double* P;
  const double* Q;
  double* d_out;
  double* X;
  nvd_pair_info* info;
  double rtol2, irtol2;
  int max_iter, max_refine;
};

// Chunk loop of a sweep kernel.  Blocks are dealt to the 8 XCDs round-robin
// (block b runs on XCD b % 8), and every graph's chunks sit in one XCD's
// range, so a graph is swept by the blocks of one XCD at about the same time
// and its gathered vector stays in that XCD's L2.  (Where blocks land
// elsewhere only speed changes: each chunk is still processed exactly once.)
#define SWEEP_CHUNKS(a, ch)                                                            \
  for (int sweep_j = (int)(blockIdx.x >> 3), sweep_x = (int)(blockIdx.x & 7), ch = 0; \
       sweep_j < (a).xcount[sweep_x] && ((ch = (a).xfirst[sweep_x] + sweep_j), true); \
       sweep_j += (int)(gridDim.x >> 3))

// ---------------------------------------------------------------------------
// chunk reductions
// ---------------------------------------------------------------------------
// Column sums over the block when entry v of thread t is column (t*N+v) % T:
// shuffles within each wave, then the waves in order.  sh holds
// (SBS/64)*ND*T doubles; the result is vals[d*T + c].
template <int ND, int N>
__device__ __forceinline__ void chunk_block_sum(double (&acc)[ND][N], int T, double* sh, double* vals) {
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int L = T / N;
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
      for (int w = 0; w < SBS / 64; ++w) s += sh[(w * ND + d) * T + t];
      vals[d * T + t] = s;
    }
  }
  __syncthreads();
}

// Publish the chunk's sums vals[0..ND*T) and arrive at graph g's counter.
// Returns true in the graph's last chunk of `count`, whose vals then hold the
// graph's totals summed over its chunks first .. first+count-1 in order.
template <int ND>
__device__ bool chunk_arrive(const SArgs& a, int ch, int g, int first, int count, double* vals,
                             double* red) {
  __shared__ int s_last;
  const int ndt = ND * a.T;
  for (int i = threadIdx.x; i < ndt; i += SBS) st_agent(&a.part[(size_t)ch * a.pstride + i], vals[i]);
  wait_stores();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (ticket(&a.s.tick[g]) == (unsigned)(count - 1));
  __syncthreads();
  if (!s_last) return false;
  sum_rows_fixed<SBS>(a.part + (size_t)first * a.pstride, count, ndt, red, vals, (size_t)a.pstride);
  if (threadIdx.x == 0) __hip_atomic_store(&a.s.tick[g], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return true;
}

// After a finaliser changed graph g's flags: recount them, keep the graph
// flags and the totals in step.
__device__ __forceinline__ void recount_graph(const SArgs& a, int g) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const int T = a.T;
    int na = 0, no = 0;
    for (int c = 0; c < T; ++c) {
      na += a.s.act[g * T + c];
      no += a.s.oact[g * T + c];
    }
    const int da = (na > 0) - a.s.g_act[g];
    const int dof = (no > 0) - a.s.g_oact[g];
    a.s.g_act[g] = na > 0;
    a.s.g_oact[g] = no > 0;
    if (da) atomicAdd(&a.s.n_act[0], da);
    if (dof) atomicAdd(&a.s.n_act[1], dof);
  }
  __syncthreads();
}

template <typename V>
__device__ __forceinline__ const V* invd_ptr(const SArgs& a) {
  if constexpr (sizeof(V) == 8)
    return reinterpret_cast<const V*>(a.invd64);
  else
    return reinterpret_cast<const V*>(a.invd32);
}

// Distance and info of pair t of graph g from the FP64 dots of a residual
// pass: d^2 = delta_bar^T x + x^T r (0 when delta_bar = 0).
__device__ __forceinline__ void write_pair(const SArgs& a, const SGraph& sg, int g, int t, double bx,
                                           double xr, double rr) {
  const int i = g * a.T + t;
  const double bb = a.s.obn2[i];
  const double dsq = bb > 0.0 ? bx + xr : 0.0;
  a.d_out[sg.out_off + t] = sqrt(dsq > 0.0 ? dsq : 0.0);
  nvd_pair_info pi;
  pi.status = a.s.stat[i];
  pi.iters = a.s.it[i];
  pi.refine_steps = a.s.ref[i];
  pi.flags = 0;
  pi.rel_res = bb > 0.0 ? sqrt(rr / bb) : 0.0;
  pi.dsq_plain = bb > 0.0 ? bx : 0.0;
  pi.dsq = dsq;
  a.info[sg.out_off + t] = pi;
}

// ---------------------------------------------------------------------------
// set-up: delta = P - Q, its mean, delta_bar, ||delta_bar||
// ---------------------------------------------------------------------------
__global__ void ks_reset(SArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < a.G) {
    a.s.g_act[i] = 0;
    a.s.g_oact[i] = 0;
    a.s.xseq[i] = 0;
    a.s.xdone[i] = 0;
  }
  if (i < 2) a.s.n_act[i] = 0;
}

template <int T>
__global__ __launch_bounds__(SBS) void ks_delta(SArgs a) {
  __shared__ double sh[(SBS / 64) * T];
  __shared__ double vals[kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  const int c = t % T;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const int k = sg.k;
    const double* Pg = a.P + sg.in_off;
    const double* Qg = a.Q + sg.in_off;
    double* b = a.b64 + sg.node_off * T;
    double acc[1][1] = {{0.0}};
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) {
      const long i = e / T;
      const double d = c < k ? Pg[i * k + c] - Qg[i * k + c] : 0.0;
      b[e] = d;
      acc[0][0] += d;
    }
    chunk_block_sum<1, 1>(acc, T, sh, vals);
    if (chunk_arrive<1>(a, ch, g, sg.first, sg.nshort, vals, red)) {
      if (t < T) a.s.mean[g * T + t] = vals[t] / (double)sg.n;
    }
    __syncthreads();
  }
}

template <int T>
__global__ __launch_bounds__(SBS) void ks_proj(SArgs a) {
  __shared__ double sh[(SBS / 64) * T];
  __shared__ double vals[kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  const int c = t % T;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    double* b = a.b64 + sg.node_off * T;
    double* x = a.x64 + sg.node_off * T;
    const double m = a.s.mean[g * T + c];
    double acc[1][1] = {{0.0}};
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) {
      const double v = b[e] - m;
      b[e] = v;
      x[e] = 0.0;
      acc[0][0] += v * v;
    }
    chunk_block_sum<1, 1>(acc, T, sh, vals);
    if (chunk_arrive<1>(a, ch, g, sg.first, sg.nshort, vals, red)) {
      if (t < T) {
        const int i = g * T + t;
        a.s.obn2[i] = vals[t];
        a.s.oact[i] = (t < sg.k && vals[t] > 0.0) ? 1 : 0;
        a.s.act[i] = 0;
        a.s.it[i] = 0;
        a.s.itc[i] = 0;
        a.s.ref[i] = 0;
        a.s.stat[i] = kStOk;
        a.s.mean[i] = 0.0;
        a.s.xm[i] = 0.0;
        // pairs with delta_bar = 0 are final now: d = 0, x = 0
        if (t < sg.k && !a.s.oact[i]) write_pair(a, sg, g, t, 0.0, 0.0, 0.0);
      }
      recount_graph(a, g);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Laplacian apply over chunks
//   EPI_CG:              q = L p (V), dot p.q -> alpha
//   EPI_RESID, ND == 5:  r = delta_bar - L x (FP64) on the open graphs; sum r,
//                        r.r, delta_bar.x, x.r, sum x -> outer check, and d of
//                        every pair of the graph for the current x (the mean
//                        of x accounted for: the graph's last pass is final)
//   EPI_RESID, ND == 4:  pass over every graph after x was made mean-zero:
//                        delta_bar.x, x.r -> d
// ---------------------------------------------------------------------------
template <typename V, int T, int EPI, int ND>
__global__ __launch_bounds__(SBS) void ks_spmm(SArgs a) {
  constexpr int W16 = 16 / (int)sizeof(V);
  constexpr int VW = T < W16 ? T : W16;
  constexpr int L = T / VW;
  constexpr int RW = 64 / L;
  constexpr int ROWS = (SBS / 64) * RW;
  constexpr int U = 8;
  using VV = typename VecOf<V, VW>::type;
  constexpr int SHN = (SBS / 64) * ND * T > SBS * VW ? (SBS / 64) * ND * T : SBS * VW;
  __shared__ double sh[SHN];
  __shared__ double vals[5 * kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wave = t >> 6;
  const int gl = lane / L;
  const int cv = lane % L;
  const V* xall;
  V* yall;
  if constexpr (EPI == EPI_CG) {
    xall = reinterpret_cast<const V*>(a.pv);
    yall = reinterpret_cast<V*>(a.qv);
  } else {
    xall = reinterpret_cast<const V*>(a.x64);
    yall = reinterpret_cast<V*>(a.r64);
  }
  SWEEP_CHUNKS(a, ch) {
    const int g = a.ch_graph[ch];
    if constexpr (EPI == EPI_CG) {
      if (!a.s.g_act[g]) continue;
    } else if constexpr (ND == 5) {
      if (!a.s.g_oact[g]) continue;
    }
    const SGraph sg = a.sg[g];
    const int* rp = a.rp + sg.rp_off;
    const int* ci = a.ci + sg.nnz_off;
    const bool unit = !sg.weighted;
    const V* wv;
    if constexpr (sizeof(V) == 8)
      wv = reinterpret_cast<const V*>(a.w64 + sg.nnz_off);
    else
      wv = reinterpret_cast<const V*>(a.w32 + sg.nnz_off);
    const V* x = xall + sg.node_off * T;
    V* y = yall + sg.node_off * T;
    const double* b = a.b64 + sg.node_off * T;
    double acc[ND][VW];
#pragma unroll
    for (int d = 0; d < ND; ++d)
#pragma unroll
      for (int v = 0; v < VW; ++v) acc[d][v] = 0.0;
    auto ldrow = [&](int row, int vi, V (&o)[VW]) {
      unpack<V, VW>(reinterpret_cast<const VV*>(x + (long)row * T)[vi], o);
    };
    // sum = (L x) of the row, accumulated as edge differences w (x_v - x_u)
    auto epilogue = [&](int row, int vi, const V (&sum)[VW], const V (&own)[VW]) {
      V yv[VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) yv[v] = sum[v];
      VV* yp = reinterpret_cast<VV*>(y + (long)row * T) + vi;
      if constexpr (EPI == EPI_CG) {
        __builtin_nontemporal_store(pack<V, VW>(yv), yp);
#pragma unroll
        for (int v = 0; v < VW; ++v) acc[0][v] += (double)own[v] * (double)yv[v];
      } else {
        using BV = typename VecOf<double, VW>::type;
        double bb[VW];
        unpack<double, VW>(reinterpret_cast<const BV*>(b + (long)row * T)[vi], bb);
        V rv[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) {
          const double rr = bb[v] - (double)yv[v];
          rv[v] = (V)rr;
          acc[0][v] += rr;
          acc[1][v] += rr * rr;
          acc[2][v] += bb[v] * (double)own[v];
          acc[3][v] += (double)own[v] * rr;
          if constexpr (ND == 5) acc[4][v] += (double)own[v];
        }
        __builtin_nontemporal_store(pack<V, VW>(rv), yp);
      }
    };
    const int lo = a.ch_lo[ch];
    const int hi = a.ch_hi[ch];
    if (hi >= 0) {
      for (int base = lo; base < hi; base += ROWS) {
        const int row = base + wave * RW + gl;
        int rs = 0, deg = 0;
        bool mine = false;
        if (row < hi) {
          rs = rp[row];
          const int d = rp[row + 1] - rs;
          mine = d <= kLongRow;
          deg = mine ? d : 0;
        }
        V own[VW];
        ldrow(mine ? row : lo, cv, own);
        V sum[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) sum[v] = (V)0;
        for (int e0 = 0; e0 < deg; e0 += U) {
          int col[U];
          V wt[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            col[u] = 0;
            wt[u] = (V)0;
            if (e0 + u < deg) {
              col[u] = NVD_CSR_LOAD(&ci[rs + e0 + u]);
              wt[u] = unit ? (V)1 : NVD_CSR_LOAD(&wv[rs + e0 + u]);
            }
          }
          VV xv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            xv[u] = VV{};
            if (e0 + u < deg) xv[u] = reinterpret_cast<const VV*>(x + (long)col[u] * T)[cv];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            V xs[VW];
            unpack<V, VW>(xv[u], xs);
#pragma unroll
            for (int v = 0; v < VW; ++v) sum[v] += wt[u] * (own[v] - xs[v]);
          }
        }
        if (mine) epilogue(row, cv, sum, own);
      }
    } else {
      // one long row: the whole block, SBS/L neighbour slots
      const int row = lo;
      const int rs = rp[row], re = rp[row + 1];
      constexpr int NJ = SBS / L;
      V sum[VW], xr[VW];
      ldrow(row, cv, xr);
#pragma unroll
      for (int v = 0; v < VW; ++v) sum[v] = (V)0;
      for (int e = rs + t / L; e < re; e += NJ) {
        V xs[VW];
        ldrow(ci[e], cv, xs);
        const V wt = unit ? (V)1 : wv[e];
#pragma unroll
        for (int v = 0; v < VW; ++v) sum[v] += wt * (xr[v] - xs[v]);
      }
      double pr[1][VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) pr[0][v] = (double)sum[v];
      block_reduce_cols<SBS, 1, VW>(pr, T, sh);
      if (t < L) {
        V tot[VW], own[VW];
#pragma unroll
        for (int v = 0; v < VW; ++v) tot[v] = (V)sh[t * VW + v];
        ldrow(row, t, own);
        epilogue(row, t, tot, own);
      }
      __syncthreads();
    }
    chunk_block_sum<ND, VW>(acc, T, sh, vals);
    if (chunk_arrive<ND>(a, ch, g, sg.first, sg.nshort + sg.nlong, vals, red)) {
      if (t < T) {
        const int i = g * T + t;
        if constexpr (EPI == EPI_CG) {
          double al = 0.0;
          if (a.s.act[i]) {
            const double sgm = vals[t];
            if (!(sgm > 0.0) || !isfinite(sgm)) {
              a.s.act[i] = 0;
              a.s.oact[i] = 0;
              a.s.stat[i] = kStBreak;
            } else {
              al = a.s.rho[i] / sgm;
            }
          }
          a.s.alpha[i] = al;
        } else if constexpr (ND == 5) {
          const double m = vals[t] / (double)sg.n;
          a.s.mean[i] = m;
          const double rr = vals[T + t] - (double)sg.n * m * m;   // ||r - mean||^2
          if (a.s.oact[i] && rr <= a.rtol2 * a.s.obn2[i]) a.s.oact[i] = 0;
          if (a.s.oact[i] && a.s.ref[i] >= a.max_refine) {
            a.s.oact[i] = 0;
            a.s.stat[i] = kStNoconv;
          }
          // x - mx has the same residual (L 1 = 0) and the same
          // delta_bar^T x (delta_bar sums to 0), so only x^T r moves
          const double mx = vals[4 * T + t] / (double)sg.n;
          a.s.xm[i] = mx;
          if (t < sg.k) write_pair(a, sg, g, t, vals[2 * T + t], vals[3 * T + t] - mx * vals[t], vals[T + t]);
        } else {
          if (t < sg.k) write_pair(a, sg, g, t, vals[2 * T + t], vals[3 * T + t], vals[T + t]);
        }
      }
      if constexpr (EPI == EPI_CG || ND == 5) recount_graph(a, g);
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// streaming passes over the rows of a chunk (elements e of the graph's
// row-major n x T block; thread t takes NE consecutive elements, columns
// (t*NE + v) % T)
// ---------------------------------------------------------------------------
template <typename V, int T>
struct SVec {
  static constexpr int N16 = 16 / (int)sizeof(V);
  static constexpr int NE = T >= N16 ? N16 : 1;
  using type = typename VecOf<V, NE>::type;
};

// Loads and stores of the streaming passes (update, direction):
// non-temporal.  Each vector is touched once per pass, and an XCD's share
// of the batch's vectors (tens of MB) does not stay in its 4 MB L2 from one
// pass to the next.  NVD_SWEEP_NT=0 builds plain accesses.
#ifndef NVD_SWEEP_NT
#define NVD_SWEEP_NT 1
#endif
template <typename VT>
__device__ __forceinline__ VT sw_ld(const VT* p) {
#if NVD_SWEEP_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename VT>
__device__ __forceinline__ void sw_st(const VT& v, VT* p) {
#if NVD_SWEEP_NT
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

// Inner set-up of an outer step for the open graphs: r = src - mean on open
// columns (0 elsewhere), c = 0, p = D^-1 r; rho = r^T D^-1 r, ||r||^2.
template <typename V, int T>
__global__ __launch_bounds__(SBS) void ks_inner_init(SArgs a, int first_step) {
  __shared__ double sh[(SBS / 64) * 2 * T];
  __shared__ double vals[2 * kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  const int c = t % T;
  const V* invd_all = invd_ptr<V>(a);
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    if (!a.s.g_oact[g]) continue;
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const long vo = sg.node_off * T;
    const double* src = (first_step ? a.b64 : a.r64) + vo;
    V* rv = reinterpret_cast<V*>(a.rv) + vo;
    V* cvv = reinterpret_cast<V*>(a.cv) + vo;
    V* pv = reinterpret_cast<V*>(a.pv) + vo;
    const V* invd = invd_all + sg.node_off;
    const bool open = a.s.oact[g * T + c] != 0;
    const double m = first_step ? 0.0 : a.s.mean[g * T + c];
    double acc[2][1] = {{0.0}, {0.0}};
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) {
      const long i = e / T;
      const V r = open ? (V)(src[e] - m) : (V)0;
      const V z = r * invd[i];
      rv[e] = r;
      cvv[e] = (V)0;
      pv[e] = z;
      acc[0][0] += (double)r * (double)z;
      acc[1][0] += (double)r * (double)r;
    }
    chunk_block_sum<2, 1>(acc, T, sh, vals);
    if (chunk_arrive<2>(a, ch, g, sg.first, sg.nshort, vals, red)) {
      if (t < T) {
        const int i = g * T + t;
        const double rr = vals[T + t];
        a.s.rho[i] = vals[t];
        a.s.bn2[i] = rr;
        a.s.act[i] = (a.s.oact[i] && rr > 0.0) ? 1 : 0;
        a.s.itc[i] = 0;
        if (a.s.oact[i]) a.s.ref[i] += 1;
        // inner tolerance relaxed to what this outer step still needs
        const double need2 = rr > 0.0 ? 0.09 * a.rtol2 * a.s.obn2[i] / rr : 0.0;
        a.s.itol2[i] = need2 > a.irtol2 ? (need2 < 0.25 ? need2 : 0.25) : a.irtol2;
      }
      recount_graph(a, g);
    }
    __syncthreads();
  }
}

// r -= alpha q; rho' = r^T D^-1 r, ||r||^2 -> beta, convergence (c += alpha p
// is left to ks_direction, which reads p anyway)
template <typename V, int T>
__global__ __launch_bounds__(SBS) void ks_update(SArgs a) {
  using SV = SVec<V, T>;
  constexpr int NE = SV::NE;
  using VT = typename SV::type;
  __shared__ double sh[(SBS / 64) * 2 * T];
  __shared__ double vals[2 * kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  const V* invd_all = invd_ptr<V>(a);
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    if (!a.s.g_act[g]) {
      // no iteration on this graph: nothing for ks_direction to add to c
      // (the graph's first chunk is a row chunk)
      if (ch == a.sg[g].first && t == 0) a.s.xdone[g] = a.s.xseq[g];
      continue;
    }
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const long vo = sg.node_off * T;
    const VT* Q4 = reinterpret_cast<const VT*>(reinterpret_cast<const V*>(a.qv) + vo);
    VT* R4 = reinterpret_cast<VT*>(reinterpret_cast<V*>(a.rv) + vo);
    const V* invd = invd_all + sg.node_off;
    V al[NE];
#pragma unroll
    for (int v = 0; v < NE; ++v) al[v] = (V)a.s.alpha[g * T + (t * NE + v) % T];
    double acc[2][NE];
#pragma unroll
    for (int v = 0; v < NE; ++v) acc[0][v] = acc[1][v] = 0.0;
    const long i1 = (long)hi * T / NE;
    for (long i = (long)lo * T / NE + t; i < i1; i += SBS) {
      V q[NE], r[NE];
      unpack<V, NE>(sw_ld(Q4 + i), q);
      unpack<V, NE>(sw_ld(R4 + i), r);
#pragma unroll
      for (int v = 0; v < NE; ++v) {
        r[v] -= al[v] * q[v];
        const double rd = (double)r[v];
        acc[0][v] += rd * rd * (double)invd[(i * NE + v) / T];
        acc[1][v] += rd * rd;
      }
      sw_st(pack<V, NE>(r), R4 + i);
    }
    chunk_block_sum<2, NE>(acc, T, sh, vals);
    if (chunk_arrive<2>(a, ch, g, sg.first, sg.nshort, vals, red)) {
      if (t < T) {
        const int i = g * T + t;
        double be = 0.0;
        if (a.s.act[i]) {
          const double rz = vals[t], rr = vals[T + t];
          a.s.it[i] += 1;
          a.s.itc[i] += 1;
          if (rr <= a.s.itol2[i] * a.s.bn2[i]) {
            a.s.act[i] = 0;
          } else if (a.s.itc[i] >= a.max_iter) {
            a.s.act[i] = 0;
          } else if (!(rz > 0.0) || !isfinite(rz)) {
            a.s.act[i] = 0;
            a.s.oact[i] = 0;
            a.s.stat[i] = kStBreak;
          } else {
            be = rz / a.s.rho[i];
            a.s.rho[i] = rz;
          }
        }
        a.s.beta[i] = be;
      }
      if (t == 0) a.s.xseq[g] += 1;
      recount_graph(a, g);
    }
    __syncthreads();
  }
}

// c += alpha p on graphs whose ks_update ran this iteration (columns that
// retired in it included; alpha is 0 on columns inactive at the apply), then
// p = D^-1 r + beta p on graphs still active.
template <typename V, int T>
__global__ __launch_bounds__(SBS) void ks_direction(SArgs a) {
  using SV = SVec<V, T>;
  constexpr int NE = SV::NE;
  using VT = typename SV::type;
  const int t = threadIdx.x;
  const V* invd_all = invd_ptr<V>(a);
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const bool xup = a.s.xseq[g] != a.s.xdone[g];
    const bool pup = a.s.g_act[g] != 0;
    if (!xup && !pup) continue;
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const long vo = sg.node_off * T;
    VT* P4 = reinterpret_cast<VT*>(reinterpret_cast<V*>(a.pv) + vo);
    VT* C4 = reinterpret_cast<VT*>(reinterpret_cast<V*>(a.cv) + vo);
    const VT* R4 = reinterpret_cast<const VT*>(reinterpret_cast<const V*>(a.rv) + vo);
    const V* invd = invd_all + sg.node_off;
    V al[NE], be[NE];
#pragma unroll
    for (int v = 0; v < NE; ++v) {
      al[v] = (V)a.s.alpha[g * T + (t * NE + v) % T];
      be[v] = (V)a.s.beta[g * T + (t * NE + v) % T];
    }
    const long i1 = (long)hi * T / NE;
    for (long i = (long)lo * T / NE + t; i < i1; i += SBS) {
      V p[NE];
      unpack<V, NE>(sw_ld(P4 + i), p);
      if (xup) {
        V cc[NE];
        unpack<V, NE>(sw_ld(C4 + i), cc);
#pragma unroll
        for (int v = 0; v < NE; ++v) cc[v] += al[v] * p[v];
        sw_st(pack<V, NE>(cc), C4 + i);
      }
      if (pup) {
        V r[NE];
        unpack<V, NE>(sw_ld(R4 + i), r);
#pragma unroll
        for (int v = 0; v < NE; ++v) p[v] = r[v] * invd[(i * NE + v) / T] + be[v] * p[v];
        sw_st(pack<V, NE>(p), P4 + i);
      }
    }
  }
}

// x += c (FP64) on the graphs that ran an inner solve this outer step
template <typename V, int T>
__global__ __launch_bounds__(SBS) void ks_accum(SArgs a) {
  const int t = threadIdx.x;
  const int c = t % T;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    // the inner loop is over: every c += alpha p has been applied
    if (ch == a.sg[g].first && t == 0) a.s.xdone[g] = a.s.xseq[g];
    if (!a.s.g_oact[g]) continue;
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const long vo = sg.node_off * T;
    double* x = a.x64 + vo;
    const V* cvv = reinterpret_cast<const V*>(a.cv) + vo;
    if (a.s.stat[g * T + c] != kStOk) continue;   // per thread: column fixed
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) x[e] += (double)cvv[e];
  }
}

// x made mean-zero: column sums, then subtraction
template <int T>
__global__ __launch_bounds__(SBS) void ks_xmean(SArgs a) {
  __shared__ double sh[(SBS / 64) * T];
  __shared__ double vals[kMaxTile];
  __shared__ double red[SBS];
  const int t = threadIdx.x;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    const double* x = a.x64 + sg.node_off * T;
    double acc[1][1] = {{0.0}};
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) acc[0][0] += x[e];
    chunk_block_sum<1, 1>(acc, T, sh, vals);
    if (chunk_arrive<1>(a, ch, g, sg.first, sg.nshort, vals, red)) {
      if (t < T) {
        a.s.mean[g * T + t] = vals[t] / (double)sg.n;
        a.s.xm[g * T + t] = 0.0;   // x is shifted in place
      }
    }
    __syncthreads();
  }
}

template <int T>
__global__ __launch_bounds__(SBS) void ks_xsub(SArgs a) {
  const int t = threadIdx.x;
  const int c = t % T;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const SGraph sg = a.sg[g];
    const int lo = a.ch_lo[ch];
    double* x = a.x64 + sg.node_off * T;
    const double m = a.s.mean[g * T + c];
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) x[e] -= m;
  }
}

// X (caller's layout: graph-major, n x k per graph) = x - (its mean where the
// last residual pass left it in x)
template <int T>
__global__ __launch_bounds__(SBS) void ks_xout(SArgs a) {
  const int t = threadIdx.x;
  const int c = t % T;
  SWEEP_CHUNKS(a, ch) {
    const int hi = a.ch_hi[ch];
    if (hi < 0) continue;
    const int g = a.ch_graph[ch];
    const SGraph sg = a.sg[g];
    if (c >= sg.k) continue;
    const int lo = a.ch_lo[ch];
    const double* x = a.x64 + sg.node_off * T;
    const double m = a.s.xm[g * T + c];
    for (long e = (long)lo * T + t; e < (long)hi * T; e += SBS) {
      const long i = e / T;
      a.X[sg.in_off + i * sg.k + c] = x[e] - m;
    }
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
// Graphs are dealt to the 8 XCDs so that every XCD gets about the same
// rows + nonzeros from each class of iteration counts (graphs in decreasing
// order of the iterations measured on the previous call, then of size, each
// to the least-loaded XCD): the open work stays balanced as graphs converge.
// The chunk table lists each XCD's graphs in turn; it is rebuilt when the
// assignment changes.  Results do not depend on it: a graph's chunks and
// their summation order are fixed by its rows alone.
static nvd_status build_chunks(nvd_batch* b, hipStream_t s) {
  const int G = b->G;
  std::vector<int> order(G);
  for (int g = 0; g < G; ++g) order[g] = g;
  auto size_of = [&](int g) { return (double)b->nnz[g] + 3.0 * b->n[g]; };
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    if (b->it_est[x] != b->it_est[y]) return b->it_est[x] > b->it_est[y];
    return size_of(x) > size_of(y);
  });
  std::vector<int> xcd(G, 0);
  double load[8] = {};
  for (int g : order) {
    int best = 0;
    for (int q = 1; q < 8; ++q)
      if (load[q] < load[best]) best = q;
    xcd[g] = best;
    load[best] += size_of(g);
  }
  if (b->ch_buf && xcd == b->ch_xcd) return NVD_OK;
  std::vector<int> cg, clo, chi;
  b->ch_first.assign(G, 0);
  b->ch_nshort.assign(G, 0);
  b->ch_nlong.assign(G, 0);
  for (int q = 0; q < 8; ++q) {
    b->xfirst[q] = (int)cg.size();
    for (int g : order) {
      if (xcd[g] != q) continue;
      b->ch_first[g] = (int)cg.size();
      const int n = b->n[g];
      for (int lo = 0; lo < n; lo += kChunkRows) {
        cg.push_back(g);
        clo.push_back(lo);
        chi.push_back(std::min(n, lo + kChunkRows));
      }
      b->ch_nshort[g] = (int)cg.size() - b->ch_first[g];
      for (int r = 0; r < b->n_long[g]; ++r) {
        cg.push_back(g);
        clo.push_back(b->h_long_rows[b->long_off[g] + r]);
        chi.push_back(-1);
      }
      b->ch_nlong[g] = b->n_long[g];
    }
    b->xcount[q] = (int)cg.size() - b->xfirst[q];
  }
  const size_t nc = cg.size();
  if (b->ch_buf && (size_t)b->n_chunks != nc) {
    (void)hipFree(b->ch_buf);
    b->ch_buf = nullptr;
  }
  if (!b->ch_buf) NVD_TRY(balloc(b, &b->ch_buf, 3 * nc));
  b->n_chunks = (int)nc;
  std::vector<int> h(3 * nc);
  std::copy(cg.begin(), cg.end(), h.begin());
  std::copy(clo.begin(), clo.end(), h.begin() + nc);
  std::copy(chi.begin(), chi.end(), h.begin() + 2 * nc);
  NVD_HIP(hipMemcpyAsync(b->ch_buf, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice, s));
  NVD_HIP(hipStreamSynchronize(s));
  b->ch_xcd = xcd;
  return NVD_OK;
}

static nvd_status poll_counts(nvd_batch* b, const SArgs& a, hipStream_t s, int* n_act, int* n_oact) {
  NVD_HIP(hipMemcpyAsync(b->h_poll, a.s.n_act, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  NVD_HIP(hipStreamSynchronize(s));
  *n_act = b->h_poll[0];
  *n_oact = b->h_poll[1];
  return NVD_OK;
}

// Inner iterations per captured chunk: kCapIters x (apply, update,
// direction).  The kernels skip graphs whose pairs have all converged, so a
// chunk that runs past the last active iteration costs only its launches.
constexpr int kCapIters = 8;

// Launches one captured chunk of inner iterations, capturing it first when
// no graph exists for these arguments (kernel arguments are fixed in the
// graph: the key is the whole argument block, the tile and the element type).
// *launched is false if capture is unavailable; the caller then launches the
// kernels directly.
template <int T, typename V>
static nvd_status launch_captured_chunk(nvd_batch* b, const SArgs& a, int grid, hipStream_t s,
                                        bool* launched) {
  *launched = false;
  if (b->sw_capture_failed) return NVD_OK;
  std::vector<unsigned char> key(sizeof(SArgs) + 3 * sizeof(int));
  std::memcpy(key.data(), &a, sizeof(SArgs));
  const int extra[3] = {T, (int)sizeof(V), grid};
  std::memcpy(key.data() + sizeof(SArgs), extra, sizeof(extra));
  if (!b->sw_exec || b->sw_key != key) {
    batch_drop_sweep_graph(b);
    if (!b->cap_stream) NVD_HIP(hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
    hipError_t e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeRelaxed);
    if (e == hipSuccess) {
      for (int it = 0; it < kCapIters; ++it) {
        ks_spmm<V, T, EPI_CG, 1><<<grid, SBS, 0, b->cap_stream>>>(a);
        ks_update<V, T><<<grid, SBS, 0, b->cap_stream>>>(a);
        ks_direction<V, T><<<grid, SBS, 0, b->cap_stream>>>(a);
      }
    }
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &gr);
    if (e == hipSuccess && e2 == hipSuccess && gr &&
        hipGraphInstantiate(&b->sw_exec, gr, nullptr, nullptr, 0) == hipSuccess) {
      b->sw_graph = gr;
      b->sw_key = key;
      ++b->captures;
    } else {
      if (gr) (void)hipGraphDestroy(gr);
      b->sw_exec = nullptr;
      b->sw_capture_failed = true;     // direct launches from now on
      (void)hipGetLastError();
      return NVD_OK;
    }
  } else {
    ++b->replays;
  }
  NVD_HIP(hipGraphLaunch(b->sw_exec, s));
  *launched = true;
  return NVD_OK;
}

template <int T, typename V>
static nvd_status sweep_t(nvd_batch* b, const std::vector<int>& ks, const nvd_opts& o,
                          const double* P, const double* Q, double* d_out, double* X,
                          nvd_pair_info* info_host, hipStream_t s) {
  const int G = b->G;
  NVD_TRY(build_chunks(b, s));
  // vectors (shared with the persistent solver's workspace)
  const size_t vsz = sizeof(V);
  if (b->cap_T < T || b->cap_vsize < (int)vsz) {
    void* ptrs[] = {b->b64, b->x64, b->r64, b->cv, b->rv, b->pv, b->qv};
    for (void* p : ptrs)
      if (p) (void)hipFree(p);
    b->b64 = b->x64 = b->r64 = nullptr;
    b->cv = b->rv = b->pv = b->qv = nullptr;
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
  // per-chunk partials and per-(graph, column) state
  const int pstride = 5 * T;
  const size_t need_part = (size_t)b->n_chunks * pstride;
  if (b->spart_cap < need_part) {
    if (b->spart) (void)hipFree(b->spart);
    b->spart = nullptr;
    NVD_TRY(balloc(b, &b->spart, need_part));
    b->spart_cap = need_part;
  }
  const size_t GT = (size_t)G * T;
  const size_t state_bytes = GT * (8 * sizeof(double) + 6 * sizeof(int)) + (size_t)G * 5 * sizeof(int) +
                             2 * sizeof(int) + 64;
  if (b->sstate_cap < state_bytes) {
    if (b->sstate) (void)hipFree(b->sstate);
    b->sstate = nullptr;
    NVD_TRY(balloc(b, &b->sstate, state_bytes));
    NVD_HIP(hipMemset(b->sstate, 0, state_bytes));   // arrival counters start at zero
    b->sstate_cap = state_bytes;
  }
  if (!b->h_poll && hipHostMalloc((void**)&b->h_poll, 2 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    set_error("batched sweep: pinned host allocation failed");
    return NVD_E_NOMEM;
  }
  // per-graph descriptors
  std::vector<SGraph> sg(G);
  int K = 0;
  long in_off = 0;
  for (int g = 0; g < G; ++g) {
    SGraph& d = sg[g];
    d.n = b->n[g];
    d.k = ks[g];
    d.weighted = b->weighted[g];
    d.first = b->ch_first[g];
    d.nshort = b->ch_nshort[g];
    d.nlong = b->ch_nlong[g];
    d.out_off = K;
    d.pad = 0;
    d.rp_off = b->rp_off[g];
    d.nnz_off = b->nnz_off[g];
    d.node_off = b->node_off[g];
    d.in_off = in_off;
    in_off += (long)d.n * d.k;
    K += d.k;
  }
  if (!b->sg_dev) {
    NVD_HIP(hipMalloc(&b->sg_dev, sizeof(SGraph) * G));
    b->bytes += (int64_t)(sizeof(SGraph) * G);
  }
  NVD_HIP(hipMemcpyAsync(b->sg_dev, sg.data(), sizeof(SGraph) * G, hipMemcpyHostToDevice, s));
  if (b->info_cap < K) {
    if (b->info) (void)hipFree(b->info);
    b->info = nullptr;
    NVD_TRY(balloc(b, &b->info, K));
    b->info_cap = K;
  }
  SArgs a{};
  a.G = G;
  a.T = T;
  a.n_chunks = b->n_chunks;
  a.pstride = pstride;
  for (int q = 0; q < 8; ++q) {
    a.xfirst[q] = b->xfirst[q];
    a.xcount[q] = b->xcount[q];
  }
  a.sg = reinterpret_cast<const SGraph*>(b->sg_dev);
  a.ch_graph = b->ch_buf;
  a.ch_lo = b->ch_buf + b->n_chunks;
  a.ch_hi = b->ch_buf + 2 * (size_t)b->n_chunks;
  a.rp = b->rp;
  a.ci = b->ci;
  a.w64 = b->w64;
  a.w32 = b->w32;
  a.invd64 = b->invd64;
  a.invd32 = b->invd32;
  a.b64 = b->b64;
  a.x64 = b->x64;
  a.r64 = b->r64;
  a.cv = b->cv;
  a.rv = b->rv;
  a.pv = b->pv;
  a.qv = b->qv;
  a.part = b->spart;
  {
    char* p = b->sstate;
    auto take_d = [&]() { double* r = reinterpret_cast<double*>(p); p += GT * sizeof(double); return r; };
    auto take_i = [&](size_t cnt) { int* r = reinterpret_cast<int*>(p); p += cnt * sizeof(int); return r; };
    a.s.rho = take_d();
    a.s.alpha = take_d();
    a.s.beta = take_d();
    a.s.bn2 = take_d();
    a.s.obn2 = take_d();
    a.s.mean = take_d();
    a.s.itol2 = take_d();
    a.s.xm = take_d();
    a.s.act = take_i(GT);
    a.s.oact = take_i(GT);
    a.s.it = take_i(GT);
    a.s.itc = take_i(GT);
    a.s.ref = take_i(GT);
    a.s.stat = take_i(GT);
    a.s.g_act = take_i(G);
    a.s.g_oact = take_i(G);
    a.s.tick = reinterpret_cast<unsigned*>(take_i(G));
    a.s.xseq = take_i(G);
    a.s.xdone = take_i(G);
    a.s.n_act = take_i(2);
  }
  a.P = P;
  a.Q = Q;
  a.d_out = d_out;
  a.X = X;
  a.info = b->info;
  const bool mixed = o.precision == NVD_MIXED;
  a.rtol2 = o.rtol * o.rtol;
  a.irtol2 = mixed ? o.inner_rtol * o.inner_rtol : o.rtol * o.rtol;
  a.max_iter = o.max_iter;
  a.max_refine = mixed ? o.max_refine : std::max(2, std::min(o.max_refine, 3));
  const char* ge = std::getenv("NVD_BATCH_GRAPH");
  const bool use_graph = !(ge && ge[0] == '0');
  // a multiple of 8 blocks (the same number on every XCD): one per chunk
  int xmax = 0;
  for (int q = 0; q < 8; ++q) xmax = std::max(xmax, b->xcount[q]);
  const int grid = 8 * std::max(1, std::min(xmax, kSweepGrid / 8));

  ks_reset<<<(G + 255) / 256, 256, 0, s>>>(a);
  ks_delta<T><<<grid, SBS, 0, s>>>(a);
  ks_proj<T><<<grid, SBS, 0, s>>>(a);
  NVD_HIP(hipGetLastError());
  // Every graph's results are written when its last pair closes: by the
  // projection (delta_bar = 0) or by a residual pass, which sees the final x.
  bool closed = false;
  for (int step = 0; step <= a.max_refine; ++step) {
    if (step > 0) ks_spmm<double, T, EPI_RESID, 5><<<grid, SBS, 0, s>>>(a);
    int n_act = 0, n_oact = 0;
    NVD_TRY(poll_counts(b, a, s, &n_act, &n_oact));
    if (n_oact == 0) {
      closed = true;
      break;
    }
    ks_inner_init<V, T><<<grid, SBS, 0, s>>>(a, step == 0 ? 1 : 0);
    int done = 0;
    int chunk = kCapIters;
    while (done < a.max_iter) {
      const int todo = std::min(chunk, a.max_iter - done);
      int it = 0;
      for (; use_graph && it + kCapIters <= todo; it += kCapIters) {
        bool launched = false;
        NVD_TRY((launch_captured_chunk<T, V>(b, a, grid, s, &launched)));
        if (!launched) break;
      }
      for (; it < todo; ++it) {
        ks_spmm<V, T, EPI_CG, 1><<<grid, SBS, 0, s>>>(a);
        ks_update<V, T><<<grid, SBS, 0, s>>>(a);
        ks_direction<V, T><<<grid, SBS, 0, s>>>(a);
      }
      NVD_HIP(hipGetLastError());
      done += todo;
      NVD_TRY(poll_counts(b, a, s, &n_act, &n_oact));
      if (n_act == 0) break;
      // chunks of whole captured sub-chunks, growing with the iterations seen
      chunk = std::min(4 * kCapIters, std::max(kCapIters, done / 2 / kCapIters * kCapIters));
    }
    ks_accum<V, T><<<grid, SBS, 0, s>>>(a);
  }
  if (!closed) {
    // pairs still open after the last step: results of the final x
    ks_xmean<T><<<grid, SBS, 0, s>>>(a);
    ks_xsub<T><<<grid, SBS, 0, s>>>(a);
    ks_spmm<double, T, EPI_RESID, 4><<<grid, SBS, 0, s>>>(a);
  }
  if (X) ks_xout<T><<<grid, SBS, 0, s>>>(a);
  NVD_HIP(hipGetLastError());
  if (info_host)
    NVD_HIP(hipMemcpyAsync(info_host, b->info, sizeof(nvd_pair_info) * K, hipMemcpyDeviceToHost, s));
  NVD_HIP(hipStreamSynchronize(s));
  ++b->sweeps;
  if (info_host) {
    int off = 0;
    for (int g = 0; g < G; ++g) {
      int itmax = 0;
      for (int j = 0; j < ks[g]; ++j) itmax = std::max(itmax, info_host[off + j].iters);
      if (itmax > 0) b->it_est[g] = itmax;
      off += ks[g];
    }
  }
  return NVD_OK;
}

nvd_status run_sweep(nvd_batch* b, const std::vector<int>& ks, int T, const nvd_opts& o,
                     const double* P, const double* Q, double* d_out, double* X,
                     nvd_pair_info* info_host, hipStream_t s) {
  const bool mixed = o.precision == NVD_MIXED;
#define NVD_ST(TT)                                                                   \
  case TT:                                                                           \
    return mixed ? sweep_t<TT, float>(b, ks, o, P, Q, d_out, X, info_host, s)        \
                 : sweep_t<TT, double>(b, ks, o, P, Q, d_out, X, info_host, s);
  switch (T) {
    NVD_ST(1) NVD_ST(2) NVD_ST(4) NVD_ST(8) NVD_ST(16) NVD_ST(32) NVD_ST(64)
    default: break;
  }
#undef NVD_ST
  set_error("batched sweep: unsupported tile");
  return NVD_E_UNSUPPORTED;
}

}  // namespace nvd
