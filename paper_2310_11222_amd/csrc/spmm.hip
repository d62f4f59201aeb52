// Laplacian apply Y = L X = D X - A X on the CSR graph (the operator of the
// paper's section 3.1), for a tile of T right-hand-side columns stored
// row-major, in FP64 or FP32.
//
// Work split:
//  * short rows (<= kLongRow neighbours): a group of G = T*NL lanes per row;
//    lane (c, j) owns column c and takes neighbours j, j+NL, ...; neighbour
//    indices are loaded G at a time by the whole group and shuffled out, so
//    the gathers of x issue back to back; the NL partial sums meet by
//    cross-lane shuffles.  A wave holds 64/G rows.
//  * long rows: segments of at most kSeg neighbours, one 256-thread block per
//    segment (256/T lanes per column), partial sums reduced in LDS; rows with
//    several segments combine them in fixed order in the last segment block
//    to arrive (per-row arrival counter), so results do not depend on timing.
// The CSR and the output are touched once per pass: they are loaded and
// stored non-temporally so that they do not push the gathered vector out of
// the last-level cache.
// Epilogues fuse the consumer of L X:
//  * EPI_PLAIN: store Y.
//  * EPI_CG:    q = L p, store q and reduce sigma_c = p_c^T q_c; the grid's
//               last block turns it into alpha_c = rho_c / sigma_c.
//  * EPI_RESID: r = b - L x (FP64), store r and reduce b^T x, x^T r, r^T r,
//               sum r, sum x per column.
#include "device_common.hpp"
#include "prof.hpp"

namespace nvd {

template <typename V>
struct SpmmK {
  int n;
  const int* rp;
  const int* ci;
  const V* w;      // null for unit weights
  const V* deg;    // null for unit weights
  const V* x;
  long ldx;
  V* y;
  long ldy;
  const double* b;
  long ldb;
  ColState* cs;
  int nlong_blocks;
  int nshort_blocks;
};

template <typename V, bool UNIT, int EPI, int ND>
__device__ __forceinline__ void spmm_epilogue(const SpmmK<V>& a, int row, int c, V sum, V own,
                                              V dg, double bb, double (&acc)[ND][1]) {
  const V yv = dg * own - sum;
  if constexpr (EPI == EPI_PLAIN) {
    __builtin_nontemporal_store(yv, &a.y[(long)row * a.ldy + c]);
  } else if constexpr (EPI == EPI_CG) {
    __builtin_nontemporal_store(yv, &a.y[(long)row * a.ldy + c]);
    acc[0][0] += (double)own * (double)yv;
  } else {
    const double rr = bb - (double)yv;
    __builtin_nontemporal_store((V)rr, &a.y[(long)row * a.ldy + c]);
    acc[0][0] += bb * (double)own;
    acc[1][0] += (double)own * rr;
    acc[2][0] += rr * rr;
    acc[3][0] += rr;
    acc[4][0] += (double)own;
  }
}

template <typename V, bool UNIT, int EPI, int ND>
__device__ __forceinline__ void spmm_epilogue_load(const SpmmK<V>& a, int row, int c, V sum,
                                                   double (&acc)[ND][1]) {
  const V own = a.x[(long)row * a.ldx + c];
  V dg;
  if constexpr (UNIT)
    dg = (V)(a.rp[row + 1] - a.rp[row]);
  else
    dg = a.deg[row];
  double bb = 0.0;
  if constexpr (EPI == EPI_RESID) bb = a.b[(long)row * a.ldb + c];
  spmm_epilogue<V, UNIT, EPI, ND>(a, row, c, sum, own, dg, bb, acc);
}

// Rows carried at once by one lane group (short-row path).
template <typename V, int T>
struct SpmmRows {
  static constexpr int R = (sizeof(V) == 8 && T >= 32) ? 2 : 4;
};

template <typename V, int T, int NL, bool UNIT, int EPI>
__global__ __launch_bounds__(kBS) void k_spmm(SpmmK<V> a, GridRed red, LongRows lr) {
  constexpr int G = T * NL;
  static_assert(G <= 64 && (64 % G) == 0, "lane group must divide a wave");
  constexpr int RW = 64 / G;
  constexpr int ND = EPI == EPI_CG ? 1 : (EPI == EPI_RESID ? 5 : 0);
  constexpr int NDA = ND > 0 ? ND : 1;
  __shared__ double sh_long[kBS];
  __shared__ double sh_red[NDA * kBS];
  __shared__ double vals[NDA * kMaxTile];
  __shared__ int s_last;

  if constexpr (EPI == EPI_CG) {
    if (a.cs->n_active == 0) return;
  }
  double acc[NDA][1];
#pragma unroll
  for (int d = 0; d < NDA; ++d) acc[d][0] = 0.0;
  const int t = threadIdx.x;

  if ((int)blockIdx.x < a.nlong_blocks) {
    // ---- split-row path: one segment per block, blocks loop over segments
    constexpr int NJ = kBS / T;
    const int c = t % T;
    const int j = t / T;
    for (int s = blockIdx.x; s < lr.n_seg; s += a.nlong_blocks) {
      const int row = lr.seg_row[s];
      const int lo = lr.seg_lo[s];
      const int hi = lr.seg_hi[s];
      V sum = (V)0;
      for (int e = lo + j; e < hi; e += NJ) {
        const int col = a.ci[e];
        V wt;
        if constexpr (UNIT)
          wt = (V)1;
        else
          wt = a.w[e];
        sum += wt * a.x[(long)col * a.ldx + c];
      }
      double part[1][1] = {{(double)sum}};
      block_reduce_cols<kBS, 1, 1>(part, T, sh_long);
      const int first = lr.seg_first[s];
      const int cnt = lr.seg_cnt[s];
      if (cnt == 1) {
        if (t < T) spmm_epilogue_load<V, UNIT, EPI, NDA>(a, row, t, (V)sh_long[t], acc);
      } else {
        if (t < T) st_agent(&lr.seg_part[(long)s * kMaxTile + t], sh_long[t]);
        wait_stores();
        __syncthreads();
        if (t == 0) s_last = (ticket(&lr.row_tick[first]) == (unsigned)(cnt - 1));
        __syncthreads();
        if (s_last) {
          if (t < T) {
            double tot = 0.0;
            for (int i = 0; i < cnt; ++i) tot += ld_agent(&lr.seg_part[(long)(first + i) * kMaxTile + t]);
            spmm_epilogue_load<V, UNIT, EPI, NDA>(a, row, t, (V)tot, acc);
          }
          if (t == 0) lr.row_tick[first] = 0u;
        }
      }
      __syncthreads();
    }
  } else {
    // ---- short rows.  Blocks are renumbered so that each XCD (blocks are
    // dealt to the 8 XCDs round-robin) walks contiguous row ranges.  Each
    // lane group carries R rows at once: their row bounds, neighbour indices,
    // gathers and own values are all issued before any of them is waited on.
    const int nsb = a.nshort_blocks;
    int sb = (int)blockIdx.x - a.nlong_blocks;
    if ((nsb & 7) == 0) sb = (sb & 7) * (nsb >> 3) + (sb >> 3);
    const int lane = t & 63;
    const int wave = t >> 6;
    const int g = lane / G;
    const int li = lane % G;
    const int c = li % T;
    const int j = li / T;
    constexpr int R = SpmmRows<V, T>::R;
    constexpr int ROWS_PER_WAVE = RW * R;
    constexpr int ROWS_PER_STEP = (kBS / 64) * ROWS_PER_WAVE;
    constexpr int MM = G / NL;             // neighbours per lane per chunk (= T)
    constexpr int MB = MM < 8 ? MM : 8;
    for (int base = sb * ROWS_PER_STEP; base < a.n; base += nsb * ROWS_PER_STEP) {
      int row[R], rs[R], deg[R];
      bool mine[R];
      V own[R], dg[R];
      double bb[R];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        row[r] = base + wave * ROWS_PER_WAVE + r * RW + g;
        rs[r] = 0;
        deg[r] = -1;                        // -1: no row in this slot
        if (row[r] < a.n) {
          rs[r] = a.rp[row[r]];
          deg[r] = a.rp[row[r] + 1] - rs[r];
        }
      }
      int maxdeg = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        mine[r] = deg[r] >= 0 && deg[r] <= kLongRow;
        own[r] = mine[r] ? a.x[(long)row[r] * a.ldx + c] : (V)0;
        if constexpr (UNIT)
          dg[r] = (V)(deg[r] > 0 ? deg[r] : 0);
        else
          dg[r] = mine[r] ? a.deg[row[r]] : (V)0;
        bb[r] = 0.0;
        if constexpr (EPI == EPI_RESID) bb[r] = mine[r] ? a.b[(long)row[r] * a.ldb + c] : 0.0;
        if (!mine[r]) deg[r] = 0;
        maxdeg = deg[r] > maxdeg ? deg[r] : maxdeg;
      }
      V sum[R];
#pragma unroll
      for (int r = 0; r < R; ++r) sum[r] = (V)0;
      for (int off = 0; off < maxdeg; off += G) {          // uniform across the group
        int myc[R], cnt[R];
        V myw[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cnt[r] = deg[r] - off;
          cnt[r] = cnt[r] < 0 ? 0 : (cnt[r] > G ? G : cnt[r]);
          myc[r] = li < cnt[r] ? __builtin_nontemporal_load(&a.ci[rs[r] + off + li]) : 0;
          myw[r] = (V)1;
          if constexpr (!UNIT)
            myw[r] = li < cnt[r] ? __builtin_nontemporal_load(&a.w[rs[r] + off + li]) : (V)0;
        }
        int maxcnt = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) maxcnt = cnt[r] > maxcnt ? cnt[r] : maxcnt;
#pragma unroll
        for (int m0 = 0; m0 < MM; m0 += MB) {
          if (NL * m0 >= maxcnt) break;                    // uniform across the group
          V xv[R][MB];
          V wv[R][MB];
#pragma unroll
          for (int r = 0; r < R; ++r) {
#pragma unroll
            for (int m = 0; m < MB; ++m) {
              const int idx = j + NL * (m0 + m);
              const int col = __shfl(myc[r], idx, G);
              if constexpr (UNIT)
                wv[r][m] = (V)1;
              else
                wv[r][m] = __shfl(myw[r], idx, G);
              xv[r][m] = idx < cnt[r] ? a.x[(long)col * a.ldx + c] : (V)0;
            }
          }
#pragma unroll
          for (int r = 0; r < R; ++r)
#pragma unroll
            for (int m = 0; m < MB; ++m) sum[r] += wv[r][m] * xv[r][m];
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
#pragma unroll
        for (int off = T; off < G; off <<= 1) sum[r] += __shfl_xor(sum[r], off, 64);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (j == 0 && mine[r]) spmm_epilogue<V, UNIT, EPI, NDA>(a, row[r], c, sum[r], own[r], dg[r], bb[r], acc);
      }
    }
  }

  if constexpr (ND > 0) {
    block_reduce_cols<kBS, ND, 1>(acc, T, sh_red);
    if (t < T) {
#pragma unroll
      for (int d = 0; d < ND; ++d) vals[d * T + t] = sh_red[d * kBS + t];
    }
    __syncthreads();
    if (!grid_reduce<kBS>(vals, ND * T, red)) return;
    if (t < T) {
      ColState* cs = a.cs;
      if constexpr (EPI == EPI_CG) {
        const double sg = vals[t];
        double al = 0.0;
        if (cs->active[t]) {
          if (!(sg > 0.0) || !isfinite(sg)) {
            cs->status[t] = kStBreak;
            cs->active[t] = 0;
            cs->oactive[t] = 0;
          } else {
            al = cs->rho[t] / sg;
          }
        }
        cs->alpha[t] = al;
      } else {
#pragma unroll
        for (int d = 0; d < ND; ++d) cs->dots[d][t] = vals[d * T + t];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <typename V, int T, int NL, bool UNIT, int EPI>
static void launch_one(const SpmmK<V>& k, const GridRed& red, const LongRows& lr, int grid,
                       hipStream_t s) {
  k_spmm<V, T, NL, UNIT, EPI><<<grid, kBS, 0, s>>>(k, red, lr);
}

template <typename V, int T, int NL, int EPI>
static void launch_unit(bool unit, const SpmmK<V>& k, const GridRed& red, const LongRows& lr,
                        int grid, hipStream_t s) {
  if (unit)
    launch_one<V, T, NL, true, EPI>(k, red, lr, grid, s);
  else
    launch_one<V, T, NL, false, EPI>(k, red, lr, grid, s);
}

template <typename V, int T, int EPI>
static bool launch_nl(int nl, bool unit, const SpmmK<V>& k, const GridRed& red,
                      const LongRows& lr, int grid, hipStream_t s) {
  switch (nl) {
    case 1: launch_unit<V, T, 1, EPI>(unit, k, red, lr, grid, s); return true;
    case 2:
      if constexpr (T * 2 <= 64) { launch_unit<V, T, 2, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    case 4:
      if constexpr (T * 4 <= 64) { launch_unit<V, T, 4, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    case 8:
      if constexpr (T * 8 <= 64) { launch_unit<V, T, 8, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    default: break;
  }
  return false;
}

template <typename V, int EPI>
static bool launch_t(int T, int nl, bool unit, const SpmmK<V>& k, const GridRed& red,
                     const LongRows& lr, int grid, hipStream_t s) {
  switch (T) {
    case 1: return launch_nl<V, 1, EPI>(nl, unit, k, red, lr, grid, s);
    case 2: return launch_nl<V, 2, EPI>(nl, unit, k, red, lr, grid, s);
    case 4: return launch_nl<V, 4, EPI>(nl, unit, k, red, lr, grid, s);
    case 8: return launch_nl<V, 8, EPI>(nl, unit, k, red, lr, grid, s);
    case 16: return launch_nl<V, 16, EPI>(nl, unit, k, red, lr, grid, s);
    case 32: return launch_nl<V, 32, EPI>(nl, unit, k, red, lr, grid, s);
    case 64: return launch_nl<V, 64, EPI>(nl, unit, k, red, lr, grid, s);
    default: return false;
  }
}

// Default neighbour lanes per row: enough lanes to cover a typical short row
// while keeping G = T*NL <= 64.
int default_nl(int T) {
  if (T >= 16) return 1;
  if (T == 8) return 2;
  if (T == 4) return 4;
  return 8;
}

int default_short_grid(int n, int T, int nl) {
  const int rows_per_step = (kBS / 64) * (64 / (T * nl));
  long steps = ((long)n + rows_per_step - 1) / rows_per_step;
  long grid = steps < 2048 ? steps : 2048;
  if (grid >= 8) grid &= ~7L;
  if (grid < 1) grid = 1;
  return (int)grid;
}

template <typename V>
static nvd_status launch_typed(const SpmmCall& c, const GridRed& red, hipStream_t s) {
  const DevGraph* g = c.g;
  SpmmK<V> k{};
  k.n = g->n;
  k.rp = g->rp;
  k.ci = g->ci;
  const bool unit = !g->weighted;
  if constexpr (sizeof(V) == 8) {
    k.w = g->w64;
    k.deg = g->deg64;
  } else {
    k.w = g->w32;
    k.deg = g->deg32;
  }
  k.x = static_cast<const V*>(c.x);
  k.ldx = c.ldx;
  k.y = static_cast<V*>(c.y);
  k.ldy = c.ldy;
  k.b = c.b;
  k.ldb = c.ldb;
  k.cs = c.cs;
  const int nl = c.nl > 0 ? c.nl : default_nl(c.T);
  k.nlong_blocks = g->lr.n_seg < 1024 ? g->lr.n_seg : 1024;
  int sg = c.grid > 0 ? c.grid : default_short_grid(g->n, c.T, nl);
  const int cap = kMaxBlocks - k.nlong_blocks;
  if (sg > cap) sg = cap & ~7;
  k.nshort_blocks = sg;
  const int grid = k.nlong_blocks + sg;
  int pid = -1;
  if (prof_enabled()) {
    const double sv = (double)sizeof(V);
    const double sw = unit ? 0.0 : sv;
    const double n = g->n;
    const double csr = (4.0 + sw) * g->nnz + 4.0 * (n + 1) + sw * n;
    const double vec = c.epi == EPI_RESID ? 3.0 * c.T * 8.0 * n : 2.0 * c.T * sv * n;
    pid = prof_begin(s, sizeof(V) == 8 ? PK_SPMM64 : PK_SPMM32, csr + vec);
  }
  bool ok = false;
  switch (c.epi) {
    case EPI_PLAIN: ok = launch_t<V, EPI_PLAIN>(c.T, nl, unit, k, red, g->lr, grid, s); break;
    case EPI_CG: ok = launch_t<V, EPI_CG>(c.T, nl, unit, k, red, g->lr, grid, s); break;
    case EPI_RESID:
      if constexpr (sizeof(V) == 8) ok = launch_t<V, EPI_RESID>(c.T, nl, unit, k, red, g->lr, grid, s);
      break;
    default: break;
  }
  prof_end(s, pid);
  if (!ok) {
    set_error("spmm: unsupported tile/lane configuration T=" + std::to_string(c.T) +
              " nl=" + std::to_string(nl));
    return NVD_E_UNSUPPORTED;
  }
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

nvd_status launch_spmm(const SpmmCall& c, const GridRed& red, hipStream_t s) {
  if (c.g->n == 0) return NVD_OK;
  return c.prec == 0 ? launch_typed<double>(c, red, s) : launch_typed<float>(c, red, s);
}

}  // namespace nvd
