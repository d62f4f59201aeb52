// Laplacian apply of one right-hand-side column (T = 1) on large graphs, by
// column slices pinned to XCDs.  Same operator as k_spmm (the paper's
// section 3.1 L = D - A):
//   (L x)_v = sum_u w_vu (x_v - x_u).
//
// On a large random graph a one-column apply is bound by its neighbour
// gathers: each reads 4 or 8 bytes of x and brings a 128-byte line, and the
// lines of x do not stay in an XCD's 4 MB L2.  Here the columns (nodes) are
// cut into S = 8m slices of at most kSlNodes nodes, so that one slice of x
// fits in one XCD's L2, and the rows into chunks of kSlRows rows:
//  * slice pass: block b works on slice s = 8r + (b mod 8) of a group of
//    consecutive chunks, with the blocks of round r first.  The hardware
//    deals consecutive blocks to the 8 XCDs round-robin, so every gather of a
//    block hits the slice its XCD holds.  For every row of a chunk with
//    neighbours in the slice (an
//    "item") it writes one partial sum: in FP64, sum_{u in slice} w_vu (x_v - x_u)
//    (the edge-difference form); in FP32, sum_{u in slice} w_vu x_u
//    accumulated in FP64 (x_v is then not read by every slice: at 32 slices
//    those reads were three quarters of the pass's traffic).  Items of at
//    most kSlLongItem neighbours take one lane each (4 items per thread,
//    their neighbour lists contiguous, offsets from a block scan); longer
//    items take one wave each.
//  * combine: block per chunk; the partials of each slice are added into an
//    LDS row accumulator, slice after slice (a row has at most one item per
//    slice), then (FP32) y_v = d_v x_v - sum in FP64, d_v the FP64 sum of
//    the row's FP32 weights, rounded once to FP32 -- at least as accurate
//    as the FP32 edge-difference sum -- and the epilogue of the apply
//    (store, CG dot p^T q, or the FP64 residual r = b - L x and its dots) as
//    in k_spmm.
// Every sum is taken in a fixed order, so results repeat bit for bit.  The
// slice structure is built on the host from the graph's CSR the first time
// it is needed and kept with the graph.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

#include "device_common.hpp"
#include "prof.hpp"

namespace nvd {

constexpr int kSlRows = 2048;        // rows per chunk (LDS accumulator)
constexpr int kSlLongItem = 32;      // neighbours above which an item takes a wave
// Chunks of one slice per block of the slice pass: 8 for the FP32 pass; the
// FP64 pass (which also reads each row's own x) measured faster with one.
constexpr int slice_group(bool diff) { return diff ? 1 : 8; }
constexpr int kSlNodes = 327680;     // nodes per slice: 2.5 MB of FP64 x
constexpr int kSlMinN = 1 << 20;     // graphs this large try the slices by default

struct SliceGraph {
  int S = 0, nch = 0, sn = 0;
  long n_items = 0, n_long = 0;
  // short items, per (slice, chunk) k = s*nch + c: [it_off[k], it_off[k+1]),
  // a multiple of 4 (padding items: lrow = kSlRows, cnt = 0); their
  // neighbours [es_off[k], es_off[k+1]) in item order
  long* it_off = nullptr;
  long* es_off = nullptr;
  uint16_t* it_lrow = nullptr;
  uint8_t* it_cnt = nullptr;
  int* col_s = nullptr;
  float* w32_s = nullptr;
  double* w64_s = nullptr;
  // long items [lg_off[k], lg_off[k+1]), neighbours at lg_ent
  long* lg_off = nullptr;
  uint16_t* lg_lrow = nullptr;
  int* lg_cnt = nullptr;
  long* lg_ent = nullptr;
  int* col_l = nullptr;
  float* w32_l = nullptr;
  double* w64_l = nullptr;
  double* part_s = nullptr;   // one FP64 partial per item
  double* part_l = nullptr;
  double* dw32 = nullptr;     // weighted graphs: FP64 sum of each row's FP32 weights
  int64_t bytes = 0;
};

struct SliceArgs {
  int n, S, nch;
  const long* it_off;
  const long* es_off;
  const uint16_t* it_lrow;
  const uint8_t* it_cnt;
  const int* col_s;
  const void* w_s;
  const long* lg_off;
  const uint16_t* lg_lrow;
  const int* lg_cnt;
  const long* lg_ent;
  const int* col_l;
  const void* w_l;
  double* part_s;
  double* part_l;
  const double* dw;  // FP32 apply: d_v (sum of the row's FP32 weights, in FP64)
  const int* gate;   // EPI_CG: the tile's active count; nothing to do when 0
};

template <typename V>
struct SliceOut {
  const V* x;
  long ldx;
  V* y;
  long ldy;
  const double* b;
  long ldb;
  ColState* cs;
};

// DIFF: the edge-difference partial (FP64); else sum w x_u in FP64 (FP32).
template <typename V, bool UNIT, bool DIFF>
__global__ __launch_bounds__(kBS) void k_slice_pass(SliceArgs a, const V* __restrict__ x, long ldx) {
  using A = typename std::conditional<DIFF, V, double>::type;
  __shared__ int wsum[kBS / 64];
  constexpr int G = slice_group(DIFF);
  __shared__ long bnd[G + 1];
  __shared__ long bndl[G + 1];
  if (a.gate && *a.gate == 0) return;
  // block -> (slice s, chunks c0 .. c0+cn-1); consecutive blocks go to the
  // 8 XCDs in turn, and the blocks of one round cover slices 8r .. 8r+7
  const int ngrp = (a.nch + G - 1) / G;
  const int per_round = 8 * ngrp;
  const int r = (int)blockIdx.x / per_round;
  const int idx = (int)blockIdx.x - r * per_round;
  const int s = r * 8 + (idx & 7);
  const int c0 = (idx >> 3) * G;
  const int cn = min(G, a.nch - c0);
  const long k = (long)s * a.nch + c0;
  // the items (and neighbours) of consecutive chunks of one slice are
  // contiguous: the block walks them as one range
  if ((int)threadIdx.x <= cn) {
    bnd[threadIdx.x] = a.it_off[k + threadIdx.x];
    bndl[threadIdx.x] = a.lg_off[k + threadIdx.x];
  }
  __syncthreads();
  const V* ws = static_cast<const V*>(a.w_s);
  const V* wl = static_cast<const V*>(a.w_l);
  A* part_s = reinterpret_cast<A*>(a.part_s);
  A* part_l = reinterpret_cast<A*>(a.part_l);
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const long i0 = bnd[0], i1 = bnd[cn];
  long ebase = a.es_off[k];
  for (long tile = i0; tile < i1; tile += 4 * kBS) {
    const long my = tile + 4 * t;
    const bool has = my < i1;
    // a thread's 4 items lie in one chunk (every chunk's range is a
    // multiple of 4 items)
    long base_row = 0;
    if constexpr (DIFF) {
      int g = 0;
      while (g + 1 < cn && bnd[g + 1] <= my) ++g;
      base_row = (long)(c0 + g) * kSlRows;
    }
    // 4 items per thread: lrow and count as one 8- and one 4-byte load
    const uint32_t cw = has ? *reinterpret_cast<const uint32_t*>(a.it_cnt + my) : 0u;
    const uint2 lw = has ? *reinterpret_cast<const uint2*>(a.it_lrow + my) : make_uint2(0u, 0u);
    const int cnt[4] = {(int)(cw & 255u), (int)((cw >> 8) & 255u), (int)((cw >> 16) & 255u),
                        (int)(cw >> 24)};
    const int lr[4] = {(int)(lw.x & 0xffffu), (int)(lw.x >> 16), (int)(lw.y & 0xffffu), (int)(lw.y >> 16)};
    const int tot = cnt[0] + cnt[1] + cnt[2] + cnt[3];
    // offset of this thread's neighbours: exclusive scan of tot over the block
    int incl = tot;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int v = __shfl_up(incl, off, 64);
      if (lane >= off) incl += v;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int wpre = 0, btot = 0;
#pragma unroll
    for (int w = 0; w < kBS / 64; ++w) {
      if (w < wave) wpre += wsum[w];
      btot += wsum[w];
    }
    __syncthreads();
    const long e0 = ebase + wpre + incl - tot;
    ebase += btot;
    V xi[4] = {(V)0, (V)0, (V)0, (V)0};
    if constexpr (DIFF) {
#pragma unroll
      for (int j = 0; j < 4; ++j) xi[j] = cnt[j] > 0 ? x[(base_row + lr[j]) * ldx] : (V)0;
    }
    const int c1 = cnt[0], c2 = c1 + cnt[1], c3 = c2 + cnt[2];
    A acc[4] = {(A)0, (A)0, (A)0, (A)0};
    // neighbours in flight per thread (FP64 keeps 4: its registers bound occupancy)
    constexpr int EU = sizeof(V) == 8 ? 4 : 8;
    for (int q0 = 0; q0 < tot; q0 += EU) {
      int cc[EU];
      V wt[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        cc[u] = 0;
        wt[u] = (V)1;
        if (q0 + u < tot) {
          cc[u] = a.col_s[e0 + q0 + u];
          if constexpr (!UNIT) wt[u] = ws[e0 + q0 + u];
        }
      }
      V xv[EU];
#pragma unroll
      for (int u = 0; u < EU; ++u) xv[u] = q0 + u < tot ? x[(long)cc[u] * ldx] : (V)0;
#pragma unroll
      for (int u = 0; u < EU; ++u) {
        const int q = q0 + u;
        if (q < tot) {
          // item j of neighbour q: the counts' running sums c1 <= c2 <= c3
          const int j = q < c1 ? 0 : (q < c2 ? 1 : (q < c3 ? 2 : 3));
          A d;
          if constexpr (DIFF) {
            const V xo = j == 0 ? xi[0] : (j == 1 ? xi[1] : (j == 2 ? xi[2] : xi[3]));
            d = wt[u] * (xo - xv[u]);
          } else {
            d = (A)wt[u] * (A)xv[u];
          }
          if (j == 0)
            acc[0] += d;
          else if (j == 1)
            acc[1] += d;
          else if (j == 2)
            acc[2] += d;
          else
            acc[3] += d;
        }
      }
    }
    if (has) {
#pragma unroll
      for (int j = 0; j < 4; ++j) part_s[my + j] = acc[j];
    }
  }
  // long items: one wave each, lanes over the neighbours, fixed-order sum
  const long l0 = bndl[0], l1 = bndl[cn];
  for (long q = l0 + wave; q < l1; q += kBS / 64) {
    long row = 0;
    if constexpr (DIFF) {
      int g = 0;
      while (g + 1 < cn && bndl[g + 1] <= q) ++g;
      row = (long)(c0 + g) * kSlRows + a.lg_lrow[q];
    }
    const int cnt = a.lg_cnt[q];
    const long e = a.lg_ent[q];
    const V xr = DIFF ? x[row * ldx] : (V)0;
    A sum = (A)0;
    for (int j = lane; j < cnt; j += 64) {
      const V wt = UNIT ? (V)1 : wl[e + j];
      const V xu = x[(long)a.col_l[e + j] * ldx];
      if constexpr (DIFF)
        sum += wt * (xr - xu);
      else
        sum += (A)wt * (A)xu;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
    if (lane == 0) part_l[q] = sum;
  }
}

template <typename V, int EPI, bool DIFF>
__global__ __launch_bounds__(kBS) void k_slice_combine(SliceArgs a, SliceOut<V> o, GridRed red) {
  using A = typename std::conditional<DIFF, V, double>::type;
  constexpr int ND = EPI == EPI_CG ? 1 : (EPI == EPI_RESID ? 5 : 0);
  constexpr int NDA = ND > 0 ? ND : 1;
  __shared__ A acc[kSlRows + 1];
  __shared__ double sh_red[ND > 0 ? ND * kBS : 1];
  __shared__ double vals[NDA];
  if constexpr (EPI == EPI_CG) {
    if (o.cs->n_active == 0) return;
  }
  const int t = threadIdx.x;
  const A* part_s = reinterpret_cast<const A*>(a.part_s);
  const A* part_l = reinterpret_cast<const A*>(a.part_l);
  double dacc[NDA][1];
#pragma unroll
  for (int d = 0; d < NDA; ++d) dacc[d][0] = 0.0;
  for (int c = blockIdx.x; c < a.nch; c += gridDim.x) {
    for (int i = t; i <= kSlRows; i += kBS) acc[i] = (A)0;
    __syncthreads();
    for (int s = 0; s < a.S; ++s) {
      const long k = (long)s * a.nch + c;
      const long i0 = a.it_off[k], i1 = a.it_off[k + 1];
      for (long it = i0 + 4 * t; it < i1; it += 4 * kBS) {
        const uint2 lw = *reinterpret_cast<const uint2*>(a.it_lrow + it);
        // padding items add 0 into the spare slot kSlRows
        acc[lw.x & 0xffffu] += part_s[it];
        acc[lw.x >> 16] += part_s[it + 1];
        acc[lw.y & 0xffffu] += part_s[it + 2];
        acc[lw.y >> 16] += part_s[it + 3];
      }
      const long l0 = a.lg_off[k], l1 = a.lg_off[k + 1];
      for (long q = l0 + t; q < l1; q += kBS) acc[a.lg_lrow[q]] += part_l[q];
      __syncthreads();
    }
    for (int i = t; i < kSlRows; i += kBS) {
      const long row = (long)c * kSlRows + i;
      if (row >= a.n) break;
      V yv;
      if constexpr (DIFF)
        yv = acc[i];
      else
        yv = (V)((double)o.x[row * o.ldx] * a.dw[row] - acc[i]);
      if constexpr (EPI == EPI_PLAIN) {
        o.y[row * o.ldy] = yv;
      } else if constexpr (EPI == EPI_CG) {
        o.y[row * o.ldy] = yv;
        dacc[0][0] += (double)o.x[row * o.ldx] * (double)yv;
      } else {
        const double own = (double)o.x[row * o.ldx];
        const double bb = o.b[row * o.ldb];
        const double rr = bb - (double)yv;
        o.y[row * o.ldy] = (V)rr;
        dacc[0][0] += bb * own;
        dacc[1][0] += own * rr;
        dacc[2][0] += rr * rr;
        dacc[3][0] += rr;
        dacc[4][0] += own;
      }
    }
    __syncthreads();
  }
  if constexpr (ND > 0) {
    block_reduce_cols<kBS, ND, 1>(dacc, 1, sh_red);
    if (t == 0) {
#pragma unroll
      for (int d = 0; d < ND; ++d) vals[d] = sh_red[d * kBS];
    }
    __syncthreads();
    if (!grid_reduce<kBS>(vals, ND, red)) return;
    if (t == 0) {
      ColState* cs = o.cs;
      if constexpr (EPI == EPI_CG) {
        const double sg = vals[0];
        double al = 0.0;
        if (cs->active[0]) {
          if (!(sg > 0.0) || !isfinite(sg)) {
            cs->status[0] = kStBreak;
            cs->active[0] = 0;
            cs->oactive[0] = 0;
          } else {
            al = cs->rho[0] / sg;
          }
        }
        cs->alpha[0] = al;
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) cs->dots[d][0] = vals[d];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// host: build, use, free
// ---------------------------------------------------------------------------
void free_slices(DevGraph* g) {
  SliceGraph* sg = g->slices;
  if (!sg) return;
  (void)hipDeviceSynchronize();
  void* ps[] = {sg->it_off, sg->es_off, sg->it_lrow, sg->it_cnt, sg->col_s, sg->w32_s, sg->w64_s,
                sg->lg_off, sg->lg_lrow, sg->lg_cnt, sg->lg_ent, sg->col_l, sg->w32_l, sg->w64_l,
                sg->part_s, sg->part_l, sg->dw32};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  g->bytes -= sg->bytes;
  delete sg;
  g->slices = nullptr;
  g->slice_state = 0;
}

// NVD_SLICE: "0" never, "1" for every graph, otherwise graphs of at least
// kSlMinN nodes.  NVD_SLICE_NODES: nodes per slice (default kSlNodes).
static int slice_mode() {
  const char* e = std::getenv("NVD_SLICE");
  if (e && e[0] == '0') return 0;
  if (e && e[0] == '1') return 1;
  return 2;
}

template <typename T>
static bool up(T** dst, const std::vector<T>& v, int64_t& bytes) {
  const size_t nb = std::max<size_t>(1, v.size()) * sizeof(T);
  if (hipMalloc(reinterpret_cast<void**>(dst), nb) != hipSuccess) {
    *dst = nullptr;
    return false;
  }
  bytes += (int64_t)nb;
  if (!v.empty() && hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return false;
  return true;
}

static nvd_status build_slices(DevGraph* g) {
  const long n = g->n;
  long sn = kSlNodes;
  if (const char* e = std::getenv("NVD_SLICE_NODES")) {
    const long v = std::atol(e);
    if (v >= 1) sn = v;
  }
  if (sn > n) sn = n;
  const std::vector<int>& rp = g->h_rp;
  // Slice boundaries: consecutive node ranges with about the same number of
  // CSR entries (column j holds deg(j) of them: the graph is symmetric), so
  // that the 8 XCDs of a round get about the same work even where degree
  // follows the node id (preferential attachment puts the hubs first), and
  // at most sn nodes each (one slice of x in an XCD's L2).  A multiple of 8.
  const int S0 = (int)(((n + sn - 1) / sn + 7) / 8 * 8);
  std::vector<int> slice_of(n);
  int S = 0;
  {
    const double per = (double)g->nnz / S0;
    long first = 0;
    double acc = 0.0;
    for (long j = 0; j < n; ++j) {
      const double dj = (double)(rp[j + 1] - rp[j]);
      if (j > first && (j - first >= sn || acc + 0.5 * dj > per * (S + 1))) {
        ++S;
        first = j;
      }
      slice_of[j] = S;
      acc += dj;
    }
    S = (S + 1 + 7) / 8 * 8;
  }
  const int nch = (int)((n + kSlRows - 1) / kSlRows);
  const long K = (long)S * nch;
  if (K > (1L << 31) / 8 || (long)8 * nch > (1L << 30)) {
    set_error("slices: graph too large for the sliced apply");
    return NVD_E_UNSUPPORTED;
  }
  const std::vector<int>& ci = g->h_ci;
  const bool wtd = g->weighted;
  const std::vector<double>& hw = g->h_w;
  const int nthr = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  // pass 1: items and neighbours per (slice, chunk); rows are sorted by
  // column, so a row's neighbours in one slice are one run
  std::vector<long> ns(K + 1, 0), nl(K + 1, 0), es(K + 1, 0), el(K + 1, 0);
  std::vector<char> bad(nthr, 0);
  auto runs = [&](long i, auto&& f) {
    long e = rp[i];
    const long end = rp[i + 1];
    int prev = -1;
    while (e < end) {
      const int s = slice_of[ci[e]];
      if (s < prev) return false;
      long f2 = e + 1;
      while (f2 < end && slice_of[ci[f2]] == s) ++f2;
      f(s, e, (int)(f2 - e));
      prev = s;
      e = f2;
    }
    return true;
  };
  {
    std::vector<std::thread> th;
    for (int tt = 0; tt < nthr; ++tt)
      th.emplace_back([&, tt] {
        for (int c = tt; c < nch; c += nthr)
          for (long i = (long)c * kSlRows; i < std::min(n, (long)(c + 1) * kSlRows); ++i) {
            const bool ok = runs(i, [&](int s, long, int len) {
              const long k = (long)s * nch + c;
              if (len > kSlLongItem) {
                nl[k + 1]++;
                el[k + 1] += len;
              } else {
                ns[k + 1]++;
                es[k + 1] += len;
              }
            });
            if (!ok) bad[tt] = 1;
          }
      });
    for (auto& x : th) x.join();
  }
  if (std::any_of(bad.begin(), bad.end(), [](char b) { return b != 0; })) {
    set_error("slices: rows are not sorted by column");
    return NVD_E_UNSUPPORTED;
  }
  std::vector<long> it_off(K + 1, 0), lg_off(K + 1, 0);
  for (long k = 0; k < K; ++k) {
    it_off[k + 1] = it_off[k] + (ns[k + 1] + 3) / 4 * 4;
    lg_off[k + 1] = lg_off[k] + nl[k + 1];
    es[k + 1] += es[k];
    el[k + 1] += el[k];
  }
  const long NI = it_off[K], NL = lg_off[K];
  std::vector<uint16_t> it_lrow(NI, (uint16_t)kSlRows), lg_lrow(NL);
  std::vector<uint8_t> it_cnt(NI, 0);
  std::vector<int> col_s(es[K]), col_l(el[K]), lg_cnt(NL);
  std::vector<long> lg_ent(NL);
  std::vector<double> w_s(wtd ? es[K] : 0), w_l(wtd ? el[K] : 0);
  {
    std::vector<std::thread> th;
    for (int tt = 0; tt < nthr; ++tt)
      th.emplace_back([&, tt] {
        std::vector<long> pi(S), pe(S), pl(S), pq(S);
        for (int c = tt; c < nch; c += nthr) {
          for (int s = 0; s < S; ++s) {
            const long k = (long)s * nch + c;
            pi[s] = it_off[k];
            pe[s] = es[k];
            pl[s] = lg_off[k];
            pq[s] = el[k];
          }
          for (long i = (long)c * kSlRows; i < std::min(n, (long)(c + 1) * kSlRows); ++i) {
            const uint16_t lrow = (uint16_t)(i - (long)c * kSlRows);
            runs(i, [&](int s, long e, int len) {
              if (len > kSlLongItem) {
                const long q = pl[s]++;
                lg_lrow[q] = lrow;
                lg_cnt[q] = len;
                lg_ent[q] = pq[s];
                for (int j = 0; j < len; ++j) {
                  col_l[pq[s] + j] = ci[e + j];
                  if (wtd) w_l[pq[s] + j] = hw[e + j];
                }
                pq[s] += len;
              } else {
                const long q = pi[s]++;
                it_lrow[q] = lrow;
                it_cnt[q] = (uint8_t)len;
                for (int j = 0; j < len; ++j) {
                  col_s[pe[s] + j] = ci[e + j];
                  if (wtd) w_s[pe[s] + j] = hw[e + j];
                }
                pe[s] += len;
              }
            });
          }
        }
      });
    for (auto& x : th) x.join();
  }
  SliceGraph* sg = new SliceGraph();
  sg->S = S;
  sg->nch = nch;
  sg->sn = (int)sn;
  sg->n_items = NI;
  sg->n_long = NL;
  bool ok = up(&sg->it_off, it_off, sg->bytes) && up(&sg->es_off, es, sg->bytes) &&
            up(&sg->it_lrow, it_lrow, sg->bytes) && up(&sg->it_cnt, it_cnt, sg->bytes) &&
            up(&sg->col_s, col_s, sg->bytes) && up(&sg->lg_off, lg_off, sg->bytes) &&
            up(&sg->lg_lrow, lg_lrow, sg->bytes) && up(&sg->lg_cnt, lg_cnt, sg->bytes) &&
            up(&sg->lg_ent, lg_ent, sg->bytes) && up(&sg->col_l, col_l, sg->bytes);
  if (ok && wtd) {
    std::vector<double> dw(n, 0.0);
    for (long i = 0; i < n; ++i)
      for (long e = rp[i]; e < rp[i + 1]; ++e) dw[i] += (double)(float)hw[e];
    ok = up(&sg->dw32, dw, sg->bytes);
  }
  if (ok && wtd) {
    std::vector<float> f_s(w_s.size()), f_l(w_l.size());
    for (size_t j = 0; j < w_s.size(); ++j) f_s[j] = (float)w_s[j];
    for (size_t j = 0; j < w_l.size(); ++j) f_l[j] = (float)w_l[j];
    ok = up(&sg->w64_s, w_s, sg->bytes) && up(&sg->w64_l, w_l, sg->bytes) && up(&sg->w32_s, f_s, sg->bytes) &&
         up(&sg->w32_l, f_l, sg->bytes);
  }
  if (ok) {
    ok = hipMalloc(&sg->part_s, std::max<long>(4, NI) * sizeof(double)) == hipSuccess;
    if (ok) sg->bytes += std::max<long>(4, NI) * sizeof(double);
    else sg->part_s = nullptr;
  }
  if (ok) {
    ok = hipMalloc(&sg->part_l, std::max<long>(1, NL) * sizeof(double)) == hipSuccess;
    if (ok) sg->bytes += std::max<long>(1, NL) * sizeof(double);
    else sg->part_l = nullptr;
  }
  g->slices = sg;
  g->bytes += sg->bytes;
  if (!ok) {
    (void)hipGetLastError();
    free_slices(g);
    set_error("slices: device allocation failed");
    return NVD_E_NOMEM;
  }
  return NVD_OK;
}

template <typename V>
static nvd_status launch_sliced(const SpmmCall& c, const GridRed& red, hipStream_t s) {
  const DevGraph* g = c.g;
  const SliceGraph* sg = g->slices;
  const bool unit = !g->weighted;
  SliceArgs a{};
  a.n = g->n;
  a.S = sg->S;
  a.nch = sg->nch;
  a.it_off = sg->it_off;
  a.es_off = sg->es_off;
  a.it_lrow = sg->it_lrow;
  a.it_cnt = sg->it_cnt;
  a.col_s = sg->col_s;
  a.lg_off = sg->lg_off;
  a.lg_lrow = sg->lg_lrow;
  a.lg_cnt = sg->lg_cnt;
  a.lg_ent = sg->lg_ent;
  a.col_l = sg->col_l;
  if constexpr (sizeof(V) == 8) {
    a.w_s = sg->w64_s;
    a.w_l = sg->w64_l;
  } else {
    a.w_s = sg->w32_s;
    a.w_l = sg->w32_l;
  }
  a.part_s = sg->part_s;
  a.part_l = sg->part_l;
  a.dw = unit ? g->deg64 : sg->dw32;
  a.gate = c.epi == EPI_CG ? &c.cs->n_active : nullptr;
  SliceOut<V> o{};
  o.x = static_cast<const V*>(c.x);
  o.ldx = c.ldx;
  o.y = static_cast<V*>(c.y);
  o.ldy = c.ldy;
  o.b = c.b;
  o.ldb = c.ldb;
  o.cs = c.cs;
  constexpr bool DIFF = sizeof(V) == 8;
  constexpr int G = slice_group(DIFF);
  const int pass_grid = sg->S * ((sg->nch + G - 1) / G);   // S/8 rounds x 8 slices x chunk groups
  const int comb_grid = std::min(sg->nch, kMaxBlocks);
  int pid = -1;
  if (prof_enabled()) {
    const double sv = (double)sizeof(V);
    const double sw = unit ? 0.0 : sv;
    const double n = g->n;
    const double csr = (4.0 + sw) * g->nnz + 4.0 * (n + 1);
    const double vecb = c.epi == EPI_RESID ? 3.0 * 8.0 * n : 2.0 * sv * n;
    pid = prof_begin(s, sizeof(V) == 8 ? PK_SPMM64 : PK_SPMM32, csr + vecb);
  }
  if (unit)
    k_slice_pass<V, true, DIFF><<<pass_grid, kBS, 0, s>>>(a, o.x, o.ldx);
  else
    k_slice_pass<V, false, DIFF><<<pass_grid, kBS, 0, s>>>(a, o.x, o.ldx);
  bool ok = true;
  switch (c.epi) {
    case EPI_PLAIN: k_slice_combine<V, EPI_PLAIN, DIFF><<<comb_grid, kBS, 0, s>>>(a, o, red); break;
    case EPI_CG: k_slice_combine<V, EPI_CG, DIFF><<<comb_grid, kBS, 0, s>>>(a, o, red); break;
    case EPI_RESID:
      if constexpr (sizeof(V) == 8)
        k_slice_combine<V, EPI_RESID, DIFF><<<comb_grid, kBS, 0, s>>>(a, o, red);
      else
        ok = false;
      break;
    default: ok = false;
  }
  prof_end(s, pid);
  if (!ok) {
    set_error("slices: unsupported epilogue");
    return NVD_E_UNSUPPORTED;
  }
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

// Time the row-wise and the sliced apply of this call's x (EPI_PLAIN into a
// scratch y, 3 launches each after a warm-up) and keep the faster per
// precision.
template <typename V>
static nvd_status time_forms(DevGraph* g, const SpmmCall& c, const GridRed& red, hipStream_t s, float* t_row,
                             float* t_sliced) {
  void* y = nullptr;
  NVD_HIP(hipMalloc(&y, sizeof(V) * (size_t)g->n));
  SpmmCall t = c;
  t.epi = EPI_PLAIN;
  t.y = y;
  t.ldy = 1;
  t.b = nullptr;
  t.cs = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  nvd_status st = hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
  for (int form = 0; form < 2 && st == NVD_OK; ++form) {
    auto run = [&]() { return form == 0 ? launch_spmm(t, red, s) : launch_sliced<V>(t, red, s); };
    st = run();
    if (st == NVD_OK) st = hipEventRecord(a, s) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
    for (int i = 0; i < 3 && st == NVD_OK; ++i) st = run();
    if (st == NVD_OK) st = hipEventRecord(b, s) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
    if (st == NVD_OK) st = hipEventSynchronize(b) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
    float ms = 0.0f;
    if (st == NVD_OK) st = hipEventElapsedTime(&ms, a, b) == hipSuccess ? NVD_OK : NVD_E_DEVICE;
    (form == 0 ? *t_row : *t_sliced) = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  (void)hipStreamSynchronize(s);
  (void)hipFree(y);
  return st;
}

// The sliced apply serves T = 1 on graphs of at least kSlMinN nodes where it
// is the faster form: the first eligible call of each precision builds the
// slices (state -1 after a failed build: the graph keeps the row-wise apply)
// and times both forms.  Calls with a bounded SpMM grid keep the row-wise
// apply.
static bool use_slices(DevGraph* g, const SpmmCall& c, const GridRed& red, hipStream_t s) {
  // a caller that bounds the grid (the no-allocation entry point) has sized
  // its reduction scratch for it, and building the slices would allocate
  if (c.T != 1 || g->n < 1 || c.grid > 0) return false;
  const int mode = slice_mode();
  if (mode == 0) return false;
  if (mode == 2 && g->n < kSlMinN) return false;
  if (g->slice_state < 0) return false;
  const int p = c.prec == 0 ? 0 : 1;
  if (mode == 2 && g->slice_pick[p] < 0) return false;
  if (!g->slices) {
    if (build_slices(g) != NVD_OK) {
      g->slice_state = -1;
      return false;
    }
    g->slice_state = 1;
  }
  if (mode == 2 && g->slice_pick[p] == 0) {
    float tr = 0.0f, ts = 0.0f;
    const nvd_status st = c.prec == 0 ? time_forms<double>(g, c, red, s, &tr, &ts)
                                      : time_forms<float>(g, c, red, s, &tr, &ts);
    g->slice_pick[p] = (st == NVD_OK && ts < tr) ? 1 : -1;
    if (g->slice_pick[0] < 0 && g->slice_pick[1] < 0) {
      free_slices(g);
      return false;
    }
  }
  return mode == 1 || g->slice_pick[p] > 0;
}

nvd_status launch_apply(const SpmmCall& c, const GridRed& red, hipStream_t s) {
  if (c.g->n == 0) return NVD_OK;
  DevGraph* g = const_cast<DevGraph*>(c.g);
  if (use_slices(g, c, red, s)) return c.prec == 0 ? launch_sliced<double>(c, red, s) : launch_sliced<float>(c, red, s);
  return launch_spmm(c, red, s);
}

}  // namespace nvd
