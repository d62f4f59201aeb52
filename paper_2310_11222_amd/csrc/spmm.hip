// Laplacian apply Y = L X = D X - A X on the CSR graph (the operator of the
// paper's section 3.1), for a tile of T right-hand-side columns stored
// row-major, in FP64 or FP32.
//
// Each row is accumulated as a sum of edge differences,
//   (L x)_v = sum_u w_vu (x_v - x_u),
// not as d_v x_v - sum_u w_vu x_u: the rounding error is then relative to
// the differences across edges rather than to |x|.  The two differ little
// for rough x, but a smooth x with a large spread (what a strong
// preconditioner such as a spanning tree produces on long paths, and any
// solution on an ill-conditioned graph) loses most of its FP32 digits in the
// second form.  The degree is not read at all.
//
// Work split:
//  * short rows (<= kLongRow neighbours): a group of G = L*NL lanes per row,
//    where L = T/VW lanes cover one row of X with 16-byte vectors (VW
//    elements per lane) and NL sub-groups take every NL-th neighbour.  Each
//    sub-group walks its own row's neighbour list, U neighbours at a time:
//    the U column indices are loaded first, then the U row gathers, so the
//    index -> gather dependency is paid once per U neighbours.  A lane group
//    carries R rows at once.  The NL partial sums meet by cross-lane
//    shuffles.
//  * long rows: segments of at most kSeg neighbours, one 256-thread block per
//    segment, partial sums reduced in LDS; rows with several segments combine
//    them in fixed order in the last segment block to arrive (per-row arrival
//    counter), so results do not depend on timing.  (One wave per segment
//    was measured slower: at T = 32 a wave has a quarter of a block's
//    neighbour slots, and the longest hub segment sets the kernel's time.)
// The output is stored non-temporally (touched once per pass).  The CSR is
// read with ordinary loads: non-temporal ones made each of a row's unrolled
// index loads fetch the same lines again (NVD_NT_CSR=1 builds them).
// Epilogues fuse the consumer of L X:
//  * EPI_PLAIN: store Y.
//  * EPI_CG:    q = L p, store q and reduce sigma_c = p_c^T q_c; the grid's
//               last block turns it into alpha_c = rho_c / sigma_c.
//  * EPI_RESID: r = b - L x (FP64), store r and reduce b^T x, x^T r, r^T r,
//               sum r, sum x per column.
#include "device_common.hpp"
#include "prof.hpp"

// Neighbours per unrolled step (U) and rows per lane group (R) of the
// short-row path; build-time knobs.
#ifndef NVD_SPMM_U
#define NVD_SPMM_U 8
#endif

namespace nvd {

template <typename V>
struct SpmmK {
  int n;
  const int* rp;
  const int* ci;
  const V* w;      // null for unit weights
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

// Elements per lane: 16 bytes when the tile is wide enough and the operands
// are aligned for it (VEC), else one.
template <typename V, int T, bool VEC>
struct SpmmGeom {
  static constexpr int W16 = 16 / (int)sizeof(V);
  static constexpr int VW = VEC ? (T < W16 ? T : W16) : 1;
  static constexpr int L = T / VW;       // lanes per row of X
};

#ifndef NVD_SPMM_R
#define NVD_SPMM_R 1
#endif
constexpr int kSpmmR = NVD_SPMM_R;
// Short-row blocks at most (the rest of kMaxBlocks is left to long rows).
// Small row chunks per block let the dispatcher balance the work; more
// blocks than this lengthen the grid reduction's tail.
constexpr int kSpmmMaxShortGrid = kMaxBlocks - 1024;

// Epilogue for VW columns c0 .. c0+VW-1 of one row; sum = (L x) entries.
template <typename V, int VW, bool UNIT, int EPI, int NDA>
__device__ __forceinline__ void spmm_epilogue(const SpmmK<V>& a, int row, int cv, const V (&sum)[VW],
                                              const V (&own)[VW], double (&acc)[NDA][VW]) {
  using VV = typename VecOf<V, VW>::type;
  V yv[VW];
#pragma unroll
  for (int v = 0; v < VW; ++v) yv[v] = sum[v];
  VV* yp = reinterpret_cast<VV*>(a.y + (long)row * a.ldy) + cv;
  if constexpr (EPI == EPI_PLAIN) {
    __builtin_nontemporal_store(pack<V, VW>(yv), yp);
  } else if constexpr (EPI == EPI_CG) {
    __builtin_nontemporal_store(pack<V, VW>(yv), yp);
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[0][v] += (double)own[v] * (double)yv[v];
  } else {
    using BV = typename VecOf<double, VW>::type;
    double bb[VW];
    unpack<double, VW>(reinterpret_cast<const BV*>(a.b + (long)row * a.ldb)[cv], bb);
    V rv[VW];
#pragma unroll
    for (int v = 0; v < VW; ++v) {
      const double rr = bb[v] - (double)yv[v];
      rv[v] = (V)rr;
      acc[0][v] += bb[v] * (double)own[v];
      acc[1][v] += (double)own[v] * rr;
      acc[2][v] += rr * rr;
      acc[3][v] += rr;
      acc[4][v] += (double)own[v];
    }
    __builtin_nontemporal_store(pack<V, VW>(rv), yp);
  }
}

template <typename V, int T, int NL, bool UNIT, int EPI, bool VEC>
__global__ __launch_bounds__(kBS) void k_spmm(SpmmK<V> a, GridRed red, LongRows lr) {
  using Geo = SpmmGeom<V, T, VEC>;
  constexpr int VW = Geo::VW;
  constexpr int L = Geo::L;
  constexpr int G = L * NL;
  static_assert(G <= 64 && (64 % G) == 0, "lane group must divide a wave");
  using VV = typename VecOf<V, VW>::type;
  constexpr int RW = 64 / G;
  constexpr int ND = EPI == EPI_CG ? 1 : (EPI == EPI_RESID ? 5 : 0);
  constexpr int NDA = ND > 0 ? ND : 1;
  __shared__ double sh_long[kBS * VW];
  __shared__ double sh_red[ND > 0 ? ND * kBS * VW : 1];
  __shared__ double vals[NDA * kMaxTile];
  __shared__ int s_last;

  if constexpr (EPI == EPI_CG) {
    if (a.cs->n_active == 0) return;
  }
  double acc[NDA][VW];
#pragma unroll
  for (int d = 0; d < NDA; ++d)
#pragma unroll
    for (int v = 0; v < VW; ++v) acc[d][v] = 0.0;
  const int t = threadIdx.x;
  const VV* X = reinterpret_cast<const VV*>(a.x);
  const long ldxv = a.ldx / VW;

  if ((int)blockIdx.x < a.nlong_blocks) {
    // ---- split-row path: one segment per block, blocks loop over segments
    constexpr int NJ = kBS / L;
    const int cv = t % L;
    const int j = t / L;
    for (int s = blockIdx.x; s < lr.n_seg; s += a.nlong_blocks) {
      const int row = lr.seg_row[s];
      const int lo = lr.seg_lo[s];
      const int hi = lr.seg_hi[s];
      V sum[VW], xr[VW];
      unpack<V, VW>(X[(long)row * ldxv + cv], xr);
#pragma unroll
      for (int v = 0; v < VW; ++v) sum[v] = (V)0;
      for (int e = lo + j; e < hi; e += NJ) {
        const int col = a.ci[e];
        V wt;
        if constexpr (UNIT)
          wt = (V)1;
        else
          wt = a.w[e];
        V xv[VW];
        unpack<V, VW>(X[(long)col * ldxv + cv], xv);
#pragma unroll
        for (int v = 0; v < VW; ++v) sum[v] += wt * (xr[v] - xv[v]);
      }
      double part[1][VW];
#pragma unroll
      for (int v = 0; v < VW; ++v) part[0][v] = (double)sum[v];
      block_reduce_cols<kBS, 1, VW>(part, T, sh_long);   // sh_long[c], c < T: segment sums
      const int first = lr.seg_first[s];
      const int cnt = lr.seg_cnt[s];
      if (cnt == 1) {
        if (t < L) {
          V tot[VW], own[VW];
#pragma unroll
          for (int v = 0; v < VW; ++v) tot[v] = (V)sh_long[t * VW + v];
          unpack<V, VW>(X[(long)row * ldxv + t], own);
          spmm_epilogue<V, VW, UNIT, EPI, NDA>(a, row, t, tot, own, acc);
        }
      } else {
        if (t < T) st_agent(&lr.seg_part[(long)s * kMaxTile + t], sh_long[t]);
        wait_stores();
        __syncthreads();
        if (t == 0) s_last = (ticket(&lr.row_tick[first]) == (unsigned)(cnt - 1));
        __syncthreads();
        if (s_last) {
          if (t < L) {
            V tot[VW], own[VW];
#pragma unroll
            for (int v = 0; v < VW; ++v) {
              double sacc = 0.0;
              for (int i = 0; i < cnt; ++i)
                sacc += ld_agent(&lr.seg_part[(long)(first + i) * kMaxTile + t * VW + v]);
              tot[v] = (V)sacc;
            }
            unpack<V, VW>(X[(long)row * ldxv + t], own);
            spmm_epilogue<V, VW, UNIT, EPI, NDA>(a, row, t, tot, own, acc);
          }
          if (t == 0) lr.row_tick[first] = 0u;
        }
      }
      __syncthreads();
    }
  } else {
    // ---- short rows.  Consecutive blocks take consecutive row chunks, so
    // the hardware's round-robin dealing of blocks to the 8 XCDs spreads
    // every region of the graph over all of them: with preferential
    // attachment the heavy rows sit together at low ids, and contiguous
    // per-XCD ranges would leave one XCD with most of the work.
    const int nsb = a.nshort_blocks;
    const int sb = (int)blockIdx.x - a.nlong_blocks;
    const int lane = t & 63;
    const int wave = t >> 6;
    const int g = lane / G;
    const int li = lane % G;
    const int cv = li % L;                 // vector index within the row
    const int j = li / L;                  // neighbour sub-group
    constexpr int R = kSpmmR;
    constexpr int U = NVD_SPMM_U;
    constexpr int ROWS_PER_WAVE = RW * R;
    constexpr int ROWS_PER_STEP = (kBS / 64) * ROWS_PER_WAVE;
    for (int base = sb * ROWS_PER_STEP; base < a.n; base += nsb * ROWS_PER_STEP) {
      int row[R], rs[R], deg[R];
      bool mine[R];
      V own[R][VW];
      int mx = 0;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        row[r] = base + wave * ROWS_PER_WAVE + r * RW + g;
        rs[r] = 0;
        deg[r] = 0;
        mine[r] = false;
        if (row[r] < a.n) {
          rs[r] = a.rp[row[r]];
          const int d = a.rp[row[r] + 1] - rs[r];
          mine[r] = d <= kLongRow;
          deg[r] = mine[r] ? d : 0;
        }
        mx = deg[r] > mx ? deg[r] : mx;
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int orow = mine[r] ? row[r] : 0;
        unpack<V, VW>(X[(long)orow * ldxv + cv], own[r]);
      }
      V sum[R][VW];
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < VW; ++v) sum[r][v] = (V)0;
      for (int e0 = j; e0 < mx; e0 += NL * U) {
        int col[R][U];
        V wt[R][U];
#pragma unroll
        for (int r = 0; r < R; ++r) {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            // lanes past the end of their row issue no loads
            const int e = e0 + NL * u;
            col[r][u] = 0;
            wt[r][u] = (V)0;
            if (e < deg[r]) {
              col[r][u] = NVD_CSR_LOAD(&a.ci[rs[r] + e]);
              if constexpr (UNIT)
                wt[r][u] = (V)1;
              else
                wt[r][u] = NVD_CSR_LOAD(&a.w[rs[r] + e]);
            }
          }
        }
        VV xv[R][U];
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            xv[r][u] = VV{};
            if (e0 + NL * u < deg[r]) xv[r][u] = X[(long)col[r][u] * ldxv + cv];
          }
#pragma unroll
        for (int r = 0; r < R; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            V xs[VW];
            unpack<V, VW>(xv[r][u], xs);
#pragma unroll
            for (int v = 0; v < VW; ++v) sum[r][v] += wt[r][u] * (own[r][v] - xs[v]);
          }
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int v = 0; v < VW; ++v)
#pragma unroll
          for (int off = L; off < G; off <<= 1) sum[r][v] += __shfl_xor(sum[r][v], off, 64);
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (j == 0 && mine[r])
          spmm_epilogue<V, VW, UNIT, EPI, NDA>(a, row[r], cv, sum[r], own[r], acc);
      }
    }
  }

  if constexpr (ND > 0) {
    block_reduce_cols<kBS, ND, VW>(acc, T, sh_red);
    if (t < T) {
#pragma unroll
      for (int d = 0; d < ND; ++d) vals[d * T + t] = sh_red[d * kBS * VW + t];
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
template <typename V, int T, int NL, bool VEC>
constexpr bool spmm_fits() {
  return SpmmGeom<V, T, VEC>::L * NL <= 64;
}

template <typename V, int T, int NL, bool VEC, int EPI>
static void launch_geo(bool unit, const SpmmK<V>& k, const GridRed& red, const LongRows& lr,
                       int grid, hipStream_t s) {
  if (unit)
    k_spmm<V, T, NL, true, EPI, VEC><<<grid, kBS, 0, s>>>(k, red, lr);
  else
    k_spmm<V, T, NL, false, EPI, VEC><<<grid, kBS, 0, s>>>(k, red, lr);
}

// Rows handled per block and step for (T, nl, vec); 0 if the configuration
// does not exist.
template <typename V>
static int rows_per_block(int T, int nl, bool vec) {
  const int W16 = 16 / (int)sizeof(V);
  const int VW = vec ? (T < W16 ? T : W16) : 1;
  const int G = (T / VW) * nl;
  if (G > 64 || 64 % G) return 0;
  return (kBS / 64) * (64 / G) * kSpmmR;
}

template <typename V, int T, int EPI, bool VEC>
static bool launch_nl(int nl, bool unit, const SpmmK<V>& k, const GridRed& red,
                      const LongRows& lr, int grid, hipStream_t s) {
  switch (nl) {
    case 1:
      if constexpr (spmm_fits<V, T, 1, VEC>()) { launch_geo<V, T, 1, VEC, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    case 2:
      if constexpr (spmm_fits<V, T, 2, VEC>()) { launch_geo<V, T, 2, VEC, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    case 4:
      if constexpr (spmm_fits<V, T, 4, VEC>()) { launch_geo<V, T, 4, VEC, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    case 8:
      if constexpr (spmm_fits<V, T, 8, VEC>()) { launch_geo<V, T, 8, VEC, EPI>(unit, k, red, lr, grid, s); return true; }
      break;
    default: break;
  }
  return false;
}

template <typename V, int EPI, bool VEC>
static bool launch_t(int T, int nl, bool unit, const SpmmK<V>& k, const GridRed& red,
                     const LongRows& lr, int grid, hipStream_t s) {
  switch (T) {
    case 1: return launch_nl<V, 1, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 2: return launch_nl<V, 2, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 4: return launch_nl<V, 4, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 8: return launch_nl<V, 8, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 16: return launch_nl<V, 16, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 32: return launch_nl<V, 32, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    case 64: return launch_nl<V, 64, EPI, VEC>(nl, unit, k, red, lr, grid, s);
    default: return false;
  }
}

int spmm_max_nl(int prec, int T) {
  const int elem = prec == 0 ? 8 : 4;
  const int W16 = 16 / elem;
  const int VW = T < W16 ? T : W16;
  int nl = 1;
  while (nl * 2 <= 8 && (T / VW) * nl * 2 <= 64) nl *= 2;
  return nl;
}

// Default neighbour sub-groups per row: one (a lane group walks the whole
// neighbour list of its row); build-time knob, capped by the lane budget.
#ifndef NVD_DEFAULT_NL
#define NVD_DEFAULT_NL 1
#endif
int default_nl(int T) {
  int nl = NVD_DEFAULT_NL;
  while (nl > 1 && nl > spmm_max_nl(1, T)) nl >>= 1;
  return nl;
}

static int short_grid(int n, int rows_per_step) {
  long steps = ((long)n + rows_per_step - 1) / rows_per_step;
  long grid = steps < kSpmmMaxShortGrid ? steps : kSpmmMaxShortGrid;
  if (grid >= 8) grid &= ~7L;
  if (grid < 1) grid = 1;
  return (int)grid;
}

int default_short_grid(int n, int T, int nl) {
  return short_grid(n, rows_per_block<float>(T, nl, true) > 0 ? rows_per_block<float>(T, nl, true) : kBS);
}

// Rows of vw elements can be accessed as one vector: aligned base and stride.
static bool vec_rows(const void* p, int64_t ld, int elem, int vw) {
  return vw == 1 || (((uintptr_t)p % (uintptr_t)(vw * elem)) == 0 && (ld % vw) == 0);
}

template <typename V>
static nvd_status launch_typed(const SpmmCall& c, const GridRed& red, hipStream_t s) {
  const DevGraph* g = c.g;
  SpmmK<V> k{};
  k.n = g->n;
  k.rp = g->rp;
  k.ci = g->ci;
  const bool unit = !g->weighted;
  if constexpr (sizeof(V) == 8)
    k.w = g->w64;
  else
    k.w = g->w32;
  k.x = static_cast<const V*>(c.x);
  k.ldx = c.ldx;
  k.y = static_cast<V*>(c.y);
  k.ldy = c.ldy;
  k.b = c.b;
  k.ldb = c.ldb;
  k.cs = c.cs;
  int nl = c.nl > 0 ? c.nl : default_nl(c.T);
  // vector accesses need aligned rows of X, Y (and B)
  const int W16 = 16 / (int)sizeof(V);
  const int vw = c.T < W16 ? c.T : W16;
  bool vec = vec_rows(c.x, c.ldx, sizeof(V), vw) && vec_rows(c.y, c.ldy, sizeof(V), vw);
  if (c.epi == EPI_RESID) vec = vec && vec_rows(c.b, c.ldb, sizeof(double), vw);
  // the neighbour sub-groups were tuned for one element type and alignment
  // (the mixed solver's FP64 residual pass reuses the FP32 choice): halve
  // them until a row's lane group fits in a wave
  while (nl > 1 && rows_per_block<V>(c.T, nl, vec) == 0) nl >>= 1;
  const int rpb = rows_per_block<V>(c.T, nl, vec);
  if (rpb == 0) {
    set_error("spmm: unsupported tile/lane configuration T=" + std::to_string(c.T) +
              " nl=" + std::to_string(nl));
    return NVD_E_UNSUPPORTED;
  }
  k.nlong_blocks = g->lr.n_seg < 1024 ? g->lr.n_seg : 1024;
  int sg = c.grid > 0 ? c.grid : short_grid(g->n, rpb);
  const int cap = kMaxBlocks - k.nlong_blocks;
  if (sg > cap) sg = cap & ~7;
  k.nshort_blocks = sg;
  const int grid = k.nlong_blocks + sg;
  int pid = -1;
  if (prof_enabled()) {
    const double sv = (double)sizeof(V);
    const double sw = unit ? 0.0 : sv;
    const double n = g->n;
    const double csr = (4.0 + sw) * g->nnz + 4.0 * (n + 1);
    const double vecb = c.epi == EPI_RESID ? 3.0 * c.T * 8.0 * n : 2.0 * c.T * sv * n;
    pid = prof_begin(s, sizeof(V) == 8 ? PK_SPMM64 : PK_SPMM32, csr + vecb);
  }
  bool ok = false;
  switch (c.epi) {
    case EPI_PLAIN:
      ok = vec ? launch_t<V, EPI_PLAIN, true>(c.T, nl, unit, k, red, g->lr, grid, s)
               : launch_t<V, EPI_PLAIN, false>(c.T, nl, unit, k, red, g->lr, grid, s);
      break;
    case EPI_CG:
      // solver vectors are always aligned
      ok = vec && launch_t<V, EPI_CG, true>(c.T, nl, unit, k, red, g->lr, grid, s);
      break;
    case EPI_RESID:
      if constexpr (sizeof(V) == 8) ok = vec && launch_t<V, EPI_RESID, true>(c.T, nl, unit, k, red, g->lr, grid, s);
      break;
    default: break;
  }
  prof_end(s, pid);
  if (!ok) {
    set_error("spmm: unsupported tile/lane/alignment configuration T=" + std::to_string(c.T) +
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
