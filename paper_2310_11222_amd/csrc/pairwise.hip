// All pairwise distances among m node vectors from one solve with m
// right-hand sides.
//
// Many vectors compared on one network is the common use (introduction;
// section 5.2 compares regions, airlines, countries, communities and
// categories).  The distance of section 3.1 for vectors v_i, v_j is the
// quadratic form of delta = v_i - v_j, and everything it needs is linear in
// the vectors: with x_i the solution for v_bar_i (the solve of section 3.2)
// and r_i = v_bar_i - L x_i its final FP64 residual,
//     x_delta = x_i - x_j,  r_delta = r_i - r_j,
//     J(delta) = delta_bar^T x_delta + x_delta^T r_delta
//              = Gt_ii + Gt_jj - Gt_ij - Gt_ji,   Gt = V_bar^T X + X^T R.
// So the m solves of the columns give all m(m-1)/2 distances, each with the
// same quadratic error in the residual as a pair solved on its own.
//
// Gt is an FP64 contraction over the n rows: 64 x 64 output tiles, split over
// row slices so that small m still fills the GPU; the slices' partial tiles
// are added in a fixed order (results repeat bit for bit).
#include <algorithm>
#include <cmath>
#include <vector>

#include "device_common.hpp"

namespace nvd {

constexpr int kGramTile = 64;   // output tile edge
constexpr int kGramRows = 16;   // rows staged in LDS per step
constexpr int kGramBlocks = 2048;
constexpr int kPairwiseMax = 4096;

// Columns c0 .. c0+T-1 of an n x m row-major matrix from an n x T tile.
__global__ void k_tile_put(int n, int T, const double* __restrict__ src, double* __restrict__ dst,
                           long ld) {
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x)
    dst[(e / T) * ld + e % T] = src[e];
}

// Partial Gt tile of rows [i0, i1): part[s][a][b] = sum_i Vb[i][a] X[i][b] + X[i][a] R[i][b]
// for a in [a0, a0+64), b in [b0, b0+64).  Thread t owns the 4 x 4 block
// a = a0 + (t/16)*4 + p, b = b0 + (t%16)*4 + q.
__global__ __launch_bounds__(256) void k_gram(int n, int m, const double* __restrict__ Vb,
                                              const double* __restrict__ X,
                                              const double* __restrict__ R, int rows_per_slice,
                                              int tiles_b, double* __restrict__ part) {
  __shared__ double sVa[kGramRows][kGramTile];
  __shared__ double sXa[kGramRows][kGramTile];
  __shared__ double sXb[kGramRows][kGramTile];
  __shared__ double sRb[kGramRows][kGramTile];
  const int t = threadIdx.x;
  const int tile = blockIdx.x;
  const int a0 = (tile / tiles_b) * kGramTile;
  const int b0 = (tile % tiles_b) * kGramTile;
  const int s = blockIdx.y;
  const long i0 = (long)s * rows_per_slice;
  const long i1 = std::min((long)n, i0 + rows_per_slice);
  const int tr = t / 16, tc = t % 16;
  double acc[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[p][q] = 0.0;
  // staging: thread t loads row lr = t/16 of the step, columns lc .. lc+3
  const int lr = t / 16, lc = (t % 16) * 4;
  for (long base = i0; base < i1; base += kGramRows) {
    const long i = base + lr;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ca = a0 + lc + v, cb = b0 + lc + v;
      const bool ri = i < i1;
      sVa[lr][lc + v] = (ri && ca < m) ? Vb[i * m + ca] : 0.0;
      sXa[lr][lc + v] = (ri && ca < m) ? X[i * m + ca] : 0.0;
      sXb[lr][lc + v] = (ri && cb < m) ? X[i * m + cb] : 0.0;
      sRb[lr][lc + v] = (ri && cb < m) ? R[i * m + cb] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int r = 0; r < kGramRows; ++r) {
      double va[4], xa[4], xb[4], rb[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        va[p] = sVa[r][tr * 4 + p];
        xa[p] = sXa[r][tr * 4 + p];
        xb[p] = sXb[r][tc * 4 + p];
        rb[p] = sRb[r][tc * 4 + p];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(va[p], xb[q], fma(xa[p], rb[q], acc[p][q]));
    }
    __syncthreads();
  }
  double* out = part + (size_t)s * m * m;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int a = a0 + tr * 4 + p;
    if (a >= m) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = b0 + tc * 4 + q;
      if (b < m) out[(size_t)a * m + b] = acc[p][q];
    }
  }
}

// Gt = sum of the S partial tiles in two fixed-order levels: group y of
// blockIdx.y adds slices [y*per, (y+1)*per) into part2[y], then k_gram_sum2
// adds the groups in order.  Consecutive threads take consecutive entries,
// so every load is coalesced.
constexpr int kSumGroups = 64;
__global__ void k_gram_sum1(int m, int S, const double* __restrict__ part, double* __restrict__ part2) {
  const long mm = (long)m * m;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mm) return;
  const int per = (S + kSumGroups - 1) / kSumGroups;
  const int s0 = blockIdx.y * per;
  const int s1 = min(S, s0 + per);
  double acc = 0.0;
  for (int s = s0; s < s1; ++s) acc += part[(size_t)s * mm + e];
  part2[(size_t)blockIdx.y * mm + e] = acc;
}

__global__ void k_gram_sum2(int m, const double* __restrict__ part2, double* __restrict__ Gt) {
  const long mm = (long)m * m;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= mm) return;
  double acc = 0.0;
  for (int y = 0; y < kSumGroups; ++y) acc += part2[(size_t)y * mm + e];
  Gt[e] = acc;
}

// A pair whose Gram-form d^2 is below this fraction of Gt_ii + Gt_jj has
// lost that many digits to cancellation: it is evaluated again from the
// column differences (k_pair_exact).  Rounding of the Gram entries is a few
// eps of |Gt_ii| + |Gt_jj|, so the pairs kept lose at most ~1e-10 of d^2.
constexpr double kCloseRel = 1e-5;

// D_ij = sqrt(max(Gt_ii + Gt_jj - Gt_ij - Gt_ji, 0)), D_ii = 0; optionally the
// symmetrised Gram matrix (Gt + Gt^T) / 2.  Pairs i < j with heavy
// cancellation are appended to close[] (count in *nclose).
__global__ void k_pdist(int m, const double* __restrict__ Gt, double* __restrict__ D, long ldd,
                        double* __restrict__ G, long ldg, int2* __restrict__ close,
                        unsigned* __restrict__ nclose) {
  const long mm = (long)m * m;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < mm; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / m), j = (int)(e % m);
    const double gij = Gt[(long)i * m + j], gji = Gt[(long)j * m + i];
    double d = 0.0;
    if (i != j) {
      // (a + b) - (c + d): only commutative additions, so D_ij == D_ji exactly
      const double gii = Gt[(long)i * m + i], gjj = Gt[(long)j * m + j];
      const double dsq = (gii + gjj) - (gij + gji);
      d = sqrt(dsq > 0.0 ? dsq : 0.0);
      if (i < j && dsq < kCloseRel * (fabs(gii) + fabs(gjj))) {
        const unsigned slot = atomicAdd(nclose, 1u);
        close[slot] = make_int2(i, j);
      }
    }
    D[(long)i * ldd + j] = d;
    if (G) G[(long)i * ldg + j] = 0.5 * (gij + gji);
  }
}

// The quadratic form of a close pair from its column differences, with no
// cancellation between large Gram entries:
//   J = sum_r (vb_ri - vb_rj)(x_ri - x_rj) + (x_ri - x_rj)(r_ri - r_rj).
// Block (p, s) sums rows [s*rows, (s+1)*rows) of pair p into part[p][s].
constexpr int kExactSlices = 64;
__global__ __launch_bounds__(256) void k_pair_exact(int n, int m, const double* __restrict__ Vb,
                                                    const double* __restrict__ X,
                                                    const double* __restrict__ R,
                                                    const int2* __restrict__ close, int rows,
                                                    double* __restrict__ part) {
  __shared__ double sh[256];
  const int2 pr = close[blockIdx.x];
  const long r0 = (long)blockIdx.y * rows;
  const long r1 = min((long)n, r0 + rows);
  double acc = 0.0;
  for (long r = r0 + threadIdx.x; r < r1; r += 256) {
    const long o = r * m;
    const double dv = Vb[o + pr.x] - Vb[o + pr.y];
    const double dx = X[o + pr.x] - X[o + pr.y];
    const double dr = R[o + pr.x] - R[o + pr.y];
    acc += dv * dx + dx * dr;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[(long)blockIdx.x * kExactSlices + blockIdx.y] = sh[0];
}

// D_ij = D_ji = sqrt(max(J, 0)) from the slices' sums, added in slice order.
__global__ void k_pair_fix(int nclose, const int2* __restrict__ close, const double* __restrict__ part,
                           int slices, double* __restrict__ D, long ldd) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nclose) return;
  double j = 0.0;
  for (int s = 0; s < slices; ++s) j += part[(long)p * kExactSlices + s];
  const double d = sqrt(j > 0.0 ? j : 0.0);
  const int2 pr = close[p];
  D[(long)pr.x * ldd + pr.y] = d;
  D[(long)pr.y * ldd + pr.x] = d;
}

}  // namespace nvd

using namespace nvd;

extern "C" nvd_status nvd_pairwise(nvd_graph* h, int32_t m, const double* V, int64_t ld,
                                   const nvd_opts* opts, double* D, int64_t ldd, double* G,
                                   int64_t ldg, nvd_pair_info* info, void* stream) {
  set_error("");
  if (!h || !V || !D || m < 1 || ld < m || ldd < m || (G && ldg < m)) {
    set_error("nvd_pairwise: bad argument (NULL pointer, m < 1 or a leading dimension < m)");
    return NVD_E_ARG;
  }
  if (m > kPairwiseMax) {
    set_error("nvd_pairwise: at most 4096 vectors per call");
    return NVD_E_UNSUPPORTED;
  }
  nvd_opts o;
  nvd_opts_default(&o);
  if (opts) o = *opts;
  NVD_TRY(check_solve_opts(&o));
  if (o.flags & NVD_WARM_START) {
    set_error("nvd_pairwise: NVD_WARM_START is not supported");
    return NVD_E_ARG;
  }
  DevGraph* g = h->g;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const int n = g->n;
  const size_t nm = (size_t)n * m;
  // split of the rows for the contraction
  const int tiles_1d = (m + kGramTile - 1) / kGramTile;
  const int ntiles = tiles_1d * tiles_1d;
  int S = std::max(1, kGramBlocks / ntiles);
  S = std::min(S, std::max(1, (n + 255) / 256));
  int rows_per_slice = (n + S - 1) / S;
  rows_per_slice = (rows_per_slice + kGramRows - 1) / kGramRows * kGramRows;
  S = (n + rows_per_slice - 1) / rows_per_slice;
  if (S < 1) S = 1;
  // device scratch, freed on return
  double* buf = nullptr;
  // (+ the close-pair list: m(m-1)/2 int2, a counter, and their partial sums
  // in the space of part[], which is free again by then)
  const size_t npairs = (size_t)m * (m - 1) / 2;
  const size_t nbuf = 3 * nm + (size_t)(S + kSumGroups + 1) * m * m + kMaxTile + npairs + 1;
  NVD_HIP(hipMalloc((void**)&buf, nbuf * sizeof(double)));
  double* Vb = buf;
  double* X = Vb + nm;
  double* R = X + nm;
  double* part = R + nm;
  double* part2 = part + (size_t)S * m * m;
  double* Gt = part2 + (size_t)kSumGroups * m * m;
  double* dscratch = Gt + (size_t)m * m;
  int2* close = reinterpret_cast<int2*>(dscratch + kMaxTile);
  unsigned* nclose = reinterpret_cast<unsigned*>(close + npairs);
  SolveParams sp{};
  sp.precision = o.precision;
  sp.rtol = o.rtol;
  sp.inner_rtol = o.inner_rtol;
  sp.max_iter = o.max_iter;
  sp.max_refine = o.max_refine;
  sp.warm = false;
  sp.achol = (o.flags & NVD_PRECOND_ACHOL) != 0;
  sp.tree = sp.achol || use_tree(g, o.flags);
  int tile = o.tile_k;
  if (tile == 0) tile = choose_tile(g, m, o.precision, s);
  std::vector<nvd_pair_info> hinfo(m);
  nvd_status st = NVD_OK;
  for (int c0 = 0; c0 < m && st == NVD_OK;) {
    int T = tile;
    while (T > m - c0) T >>= 1;
    sp.nl = tuned_nl(g, o.precision, T);
    st = ensure_workspace(g, T, o.precision == NVD_MIXED);
    // x of the tile's columns into X; delta_bar and the final residual stay
    // in the workspace and are copied out
    if (st == NVD_OK)
      st = solve_tile(g, T, V + c0, nullptr, ld, sp, dscratch, X + c0, m, g->ws->info, s);
    if (st == NVD_OK) {
      const int grid = (int)std::min<long>(2048, ((long)n * T + 255) / 256);
      k_tile_put<<<std::max(grid, 1), 256, 0, s>>>(n, T, g->ws->b64, Vb + c0, m);
      k_tile_put<<<std::max(grid, 1), 256, 0, s>>>(n, T, g->ws->r64, R + c0, m);
      hipError_t e = hipGetLastError();
      if (e == hipSuccess)
        e = hipMemcpyAsync(hinfo.data() + c0, g->ws->info, sizeof(nvd_pair_info) * T,
                           hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        set_error(std::string("nvd_pairwise: ") + hipGetErrorString(e));
        st = NVD_E_DEVICE;
      }
    }
    c0 += T;
  }
  if (st == NVD_OK) {
    k_gram<<<dim3(ntiles, S), 256, 0, s>>>(n, m, Vb, X, R, rows_per_slice, tiles_1d, part);
    const int g2 = (int)std::min<long>(1024, ((long)m * m + 255) / 256);
    const int ge = (int)(((long)m * m + 255) / 256);
    k_gram_sum1<<<dim3(ge, kSumGroups), 256, 0, s>>>(m, S, part, part2);
    k_gram_sum2<<<ge, 256, 0, s>>>(m, part2, Gt);
    hipError_t e = hipMemsetAsync(nclose, 0, sizeof(unsigned), s);
    if (e == hipSuccess) {
      k_pdist<<<std::max(g2, 1), 256, 0, s>>>(m, Gt, D, ldd, G, ldg, close, nclose);
      e = hipGetLastError();
    }
    unsigned hclose = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&hclose, nclose, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && hclose > 0) {
      // close pairs again from their column differences; their partial sums
      // (64 per pair) go to part2[], free once Gt is formed: it holds
      // 64 m^2 > 64 m (m-1) / 2 doubles
      const int slices = std::min(kExactSlices, std::max(1, (n + 4095) / 4096));
      const int rows = (n + slices - 1) / slices;
      const int cnt = (int)hclose;
      k_pair_exact<<<dim3(cnt, slices), 256, 0, s>>>(n, m, Vb, X, R, close, rows, part2);
      k_pair_fix<<<(cnt + 255) / 256, 256, 0, s>>>(cnt, close, part2, slices, D, ldd);
      e = hipGetLastError();
      if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (e != hipSuccess) {
      set_error(std::string("nvd_pairwise: ") + hipGetErrorString(e));
      st = NVD_E_DEVICE;
    }
  }
  (void)hipFree(buf);
  if (st != NVD_OK) return st;
  nvd_status agg = NVD_OK;
  for (int j = 0; j < m; ++j) {
    if (hinfo[j].status == NVD_E_BREAKDOWN) agg = NVD_E_BREAKDOWN;
    else if (hinfo[j].status == NVD_E_NOCONV && agg == NVD_OK) agg = NVD_E_NOCONV;
  }
  if (info) std::copy(hinfo.begin(), hinfo.end(), info);
  if (agg != NVD_OK) set_error("nvd_pairwise: some columns did not converge (see info)");
  return agg;
}
