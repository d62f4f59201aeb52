// Approximate-Cholesky preconditioner: sparse approximate Gaussian
// elimination of the Laplacian (section 3.2: Cholesky elimination made sparse
// by sampling the cliques it would create; the solver behind Table 2),
// applied as the preconditioner of CG.
//
// Factorization (host, once per graph and weights).  Eliminating a vertex v
// with neighbours u_i (weights w_i, W = sum w_i) writes the factor column
// c_i = w_i / W and the pivot W, and exact elimination would join every pair
// of neighbours with weight w_i w_j / W (a clique).  Instead the neighbours
// are taken in ascending weight order and each u_i except the last is joined
// to ONE later neighbour u_j, drawn with probability w_j / S_i (S_i the sum
// of the later weights), with weight w_i S_i / W.  The expected weight of
// each pair is the clique's w_i w_j / W, at most deg - 1 edges are added for
// the deg removed, and degree-1 and degree-2 eliminations are exact (a leaf
// adds nothing; a degree-2 vertex joins its two neighbours with the series
// weight w_1 w_2 / W).  Draws come from a counter-based hash of (vertex,
// neighbour rank), so a graph always gets the same factor.
//
// Order, for the GPU.  Vertices are eliminated in rounds: each round takes a
// maximal set of live vertices no two of which are adjacent, greedily in
// ascending current degree, among those of degree at most max(2, 2 d_min)
// (d_min the smallest current degree), so that low degrees go first -- and a
// graph that can be taken apart by degree-1 and degree-2 eliminations (a
// tree, a cycle) is factored exactly.  Eliminations within a round commute
// (none touches another's neighbourhood), so the triangular solves process
// a round in parallel: the depth of each solve is the number of rounds.
// Elimination preserves connectivity, and the last vertex of each component
// ends with no neighbours: its pivot is 0 (the Laplacian's null space) and it
// grounds its component.  After kAcholMaxRounds rounds the vertices still
// live (if any) keep the diagonal of their current Schur complement (Jacobi
// on the remainder).
//
// Application z = M^-1 r, M = F D F^T (F unit lower triangular by
// elimination order), per column of the tile:
//   r <- r - mean_C(r)  (per component; see below)
//   forward, rounds in order:  y_u = r_u + sum over eliminated v with u in
//                              v's column: c_vu y_v
//   backward, remainder first, then rounds in reverse:
//                              z_v = y_v / W_v + sum_{u in v's column} c_vu z_u
// (y is kept in z.)  The map with ground pivots 0 is a grounded inverse, whose
// image of a constant vector is large on long, thin graphs; the rounding-level
// component mean that the solver's residual carries would then swamp z, so
// it is removed first.  z then differs from the exact pseudoinverse image
// by a constant per component, which does not change r^T z and which the
// solver's projections remove.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <numeric>
#include <thread>
#include <vector>

#include "device_common.hpp"

namespace nvd {

constexpr int kAcholMaxRounds = 256;   // default cap on elimination rounds
constexpr uint64_t kAcholSeed = 0x2310112200000001ull;

namespace {

uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

// Uniform [0, 1) from (vertex, neighbour rank): a counter-based hash.
double draw(uint64_t v, uint64_t i) {
  const uint64_t h = mix64(kAcholSeed ^ mix64(v * 0x9e3779b97f4a7c15ull + i));
  return (double)(h >> 11) * 0x1.0p-53;
}

struct Nb {
  int u;
  double w;
};

struct HostFactor {
  std::vector<int> order;          // vertices by position (rounds, then remainder)
  std::vector<int> round_off;      // positions: round r is [round_off[r], round_off[r+1]); last range: remainder
  std::vector<int> col_off;        // [n+1] by position: the factor column of order[p]
  std::vector<int> col_idx;        // later vertex
  std::vector<double> col_c;       // coefficient w / W
  std::vector<double> inv_pivot;   // by position: 1 / W (0: ground), remainder: 1 / Schur diagonal
  int rounds = 0;
  int grounds = 0;
  int remainder = 0;
};

// Merge repeated neighbours (sum of weights) and drop dead ones.  The first
// `clean` entries are already merged and sorted by neighbour (a previous
// compaction); only the entries appended since (fill) are sorted, then
// merged in: O(d + t log t) for t new entries instead of O(d log d), which
// matters for hubs, whose lists are compacted in almost every round.
void compact(std::vector<Nb>& a, int& clean, const std::vector<char>& alive) {
  size_t k = 0, kept = 0;
  for (size_t i = 0; i < a.size(); ++i) {
    if (!alive[a[i].u]) continue;
    if (i < (size_t)clean) ++kept;
    a[k++] = a[i];
  }
  a.resize(k);
  auto by_u = [](const Nb& x, const Nb& y) { return x.u < y.u; };
  std::stable_sort(a.begin() + kept, a.end(), by_u);
  std::inplace_merge(a.begin(), a.begin() + kept, a.end(), by_u);
  if (k >= 2) {
    size_t o = 0;
    for (size_t i = 1; i < a.size(); ++i) {
      if (a[i].u == a[o].u)
        a[o].w += a[i].w;
      else
        a[++o] = a[i];
    }
    a.resize(o + 1);
  }
  clean = (int)a.size();
}

// Host threads for the factorization (one for small graphs), and f(lo, hi)
// on contiguous ranges of [0, n) in parallel.
int factor_threads(int n) {
  if (n < (1 << 16)) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  return std::max(1, std::min(hw ? (int)hw : 4, 16));
}
template <class F>
void par_ranges(int n, int nt, F&& f) {
  if (nt <= 1 || n < 4 * nt) {
    f(0, n);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&f, lo, hi]() { f(lo, hi); });
  }
  for (auto& x : th) x.join();
}

// One fill edge of an elimination (a sampled clique edge).
struct Fill {
  int a, b;
  double w;
};

HostFactor factor_graph(const DevGraph* g, int max_rounds) {
  const int n = g->n;
  const std::vector<int>& rp = g->h_rp;
  const std::vector<int>& ci = g->h_ci;
  const bool weighted = !g->h_w.empty();
  std::vector<std::vector<Nb>> adj(n);
  for (int v = 0; v < n; ++v) {
    adj[v].reserve(rp[v + 1] - rp[v]);
    for (int e = rp[v]; e < rp[v + 1]; ++e) adj[v].push_back(Nb{ci[e], weighted ? g->h_w[e] : 1.0});
  }
  std::vector<char> alive(n, 1), blocked(n, 0);
  // lists that may hold dead or repeated neighbours (every list at first;
  // then those of eliminated vertices' neighbours and of fill endpoints):
  // only they are compacted again, the others are already merged and sorted
  std::vector<char> dirty(n, 1);
  std::vector<int> clean(n, 0);   // sorted, merged prefix of each list
  std::vector<int> live(n);
  std::iota(live.begin(), live.end(), 0);
  HostFactor f;
  f.order.reserve(n);
  f.col_off.reserve(n + 1);
  f.col_off.push_back(0);
  f.inv_pivot.reserve(n);
  f.round_off.push_back(0);
  std::vector<int> cand, next_live, bucket_cnt, todo;
  std::vector<std::vector<Nb>> cols;
  std::vector<std::vector<Fill>> fills;
  std::vector<double> pivots;
  const int nt = factor_threads(n);
  for (int r = 0; r < max_rounds && !live.empty(); ++r) {
    // current degrees (merged, live neighbours only), candidates in
    // ascending degree, ties in increasing vertex id
    todo.clear();
    for (int v : live)
      if (dirty[v]) todo.push_back(v);
    par_ranges((int)todo.size(), nt, [&](int lo, int hi) {   // independent lists
      for (int i = lo; i < hi; ++i) compact(adj[todo[i]], clean[todo[i]], alive);
    });
    for (int v : todo) dirty[v] = 0;
    int dmax = 0;
    for (int v : live) dmax = std::max(dmax, (int)adj[v].size());
    bucket_cnt.assign(dmax + 2, 0);
    for (int v : live) ++bucket_cnt[adj[v].size() + 1];
    for (int d = 0; d <= dmax; ++d) bucket_cnt[d + 1] += bucket_cnt[d];
    cand.resize(live.size());
    for (int v : live) cand[bucket_cnt[adj[v].size()]++] = v;
    // greedy maximal independent set among the low-degree candidates
    next_live.clear();
    const int round_begin = (int)f.order.size();
    const int dcap = std::max(2, 2 * (int)adj[cand[0]].size());
    for (int v : cand) {
      if ((int)adj[v].size() > dcap) break;   // candidates ascend in degree
      if (blocked[v]) continue;
      f.order.push_back(v);
      blocked[v] = 1;
      for (const Nb& nb : adj[v]) blocked[nb.u] = 1;
    }
    const int round_end = (int)f.order.size();
    // eliminate the round's vertices: each one's factor column and sampled
    // fill edges in parallel (their lists are disjoint: no two are
    // adjacent), then recorded and applied in round order
    const int nr = round_end - round_begin;
    cols.resize(std::max(nr, 1));
    fills.resize(std::max(nr, 1));
    pivots.resize(std::max(nr, 1));
    par_ranges(nr, nt, [&](int lo, int hi) {
      std::vector<double> pre;
      for (int q = lo; q < hi; ++q) {
        const int v = f.order[round_begin + q];
        std::vector<Nb>& a = adj[v];
        const int d = (int)a.size();
        double W = 0.0;
        for (const Nb& nb : a) W += nb.w;
        pivots[q] = (d == 0 || !(W > 0.0)) ? 0.0 : W;
        cols[q].assign(a.begin(), a.end());   // the column, by neighbour
        fills[q].clear();
        if (d >= 2) {
          std::stable_sort(a.begin(), a.end(), [](const Nb& x, const Nb& y) { return x.w < y.w; });
          pre.assign(d + 1, 0.0);
          for (int i = 0; i < d; ++i) pre[i + 1] = pre[i] + a[i].w;
          for (int i = 0; i + 1 < d; ++i) {
            const double S = pre[d] - pre[i + 1];            // weights after i
            const double t = pre[i + 1] + draw((uint64_t)v, (uint64_t)i) * S;
            // the later neighbour j whose cumulative range holds t
            int j = (int)(std::upper_bound(pre.begin() + i + 2, pre.begin() + d + 1, t) - pre.begin()) - 1;
            if (j <= i) j = i + 1;
            if (j >= d) j = d - 1;
            fills[q].push_back(Fill{a[i].u, a[j].u, a[i].w * S / W});
          }
        }
      }
    });
    for (int q = 0; q < nr; ++q) {
      const int v = f.order[round_begin + q];
      const double W = pivots[q];
      if (W == 0.0) {
        f.inv_pivot.push_back(0.0);   // last vertex of its component: the ground
        ++f.grounds;
      } else {
        f.inv_pivot.push_back(1.0 / W);
      }
      for (const Nb& nb : cols[q]) {
        f.col_idx.push_back(nb.u);
        f.col_c.push_back(W == 0.0 ? nb.w : nb.w / W);
        dirty[nb.u] = 1;   // v dies in their lists; fill lands in some
      }
      f.col_off.push_back((int)f.col_idx.size());
      for (const Fill& e : fills[q]) {
        adj[e.a].push_back(Nb{e.b, e.w});
        adj[e.b].push_back(Nb{e.a, e.w});
      }
      alive[v] = 0;
      std::vector<Nb>().swap(adj[v]);
    }
    for (int p = round_begin; p < round_end; ++p) blocked[f.order[p]] = 0;
    for (int v : live) {
      if (alive[v]) {
        blocked[v] = 0;
        next_live.push_back(v);
      }
    }
    live.swap(next_live);
    f.round_off.push_back((int)f.order.size());
    f.rounds = r + 1;
  }
  // remainder: the diagonal of the current Schur complement
  for (int v : live) {
    compact(adj[v], clean[v], alive);
    double s = 0.0;
    for (const Nb& nb : adj[v]) s += nb.w;
    f.order.push_back(v);
    f.inv_pivot.push_back(s > 0.0 ? 1.0 / s : 0.0);
    f.col_off.push_back((int)f.col_idx.size());
    ++f.remainder;
  }
  f.round_off.push_back((int)f.order.size());
  return f;
}

}  // namespace

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// Per-component column means of r.  One component: block partial sums over
// fixed row ranges, then one block adds them in order (k_am_total).  Several
// components: one block per component over its node list.
constexpr int kAmBlocks = 256;

template <typename V>
__global__ __launch_bounds__(256) void k_am_part(int n, int T, const V* __restrict__ r,
                                                 double* __restrict__ part) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int c = t % T;
  const int rpb = 256 / T;
  const long rows = ((long)n + gridDim.x - 1) / gridDim.x;
  const long lo = (long)blockIdx.x * rows;
  const long hi = min((long)n, lo + rows);
  // eight rows in flight per thread, summed in a fixed order
  double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  long i = lo + t / T;
  for (; i + 7L * rpb < hi; i += 8L * rpb) {
#pragma unroll
    for (int u = 0; u < 8; ++u) a[u] += (double)r[(i + (long)u * rpb) * T + c];
  }
  for (int u = 0; i < hi; i += rpb, ++u) a[u & 7] += (double)r[i * T + c];
  const double acc = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
  sh[t] = acc;
  __syncthreads();
  for (int h = 128; h >= T; h >>= 1) {
    if (t < h) sh[t] += sh[t + h];
    __syncthreads();
  }
  if (t < T) part[(long)blockIdx.x * kMaxTile + t] = sh[t];
}

__global__ void k_am_total(int n, int T, int nb, const double* __restrict__ part, double* __restrict__ mean) {
  const int t = threadIdx.x;
  if (t >= T) return;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += part[(long)b * kMaxTile + t];
  mean[t] = s / (double)n;
}

template <typename V>
__global__ __launch_bounds__(256) void k_am_comp(int ncomp, int T, const int* __restrict__ perm,
                                                 const int* __restrict__ off, const V* __restrict__ r,
                                                 double* __restrict__ mean) {
  __shared__ double sh[256];
  const int t = threadIdx.x;
  const int c = t % T;
  const int rpb = 256 / T;
  for (int k = blockIdx.x; k < ncomp; k += gridDim.x) {
    const int lo = off[k], hi = off[k + 1];
    double acc = 0.0;
    for (int p = lo + t / T; p < hi; p += rpb) acc += (double)r[(long)perm[p] * T + c];
    sh[t] = acc;
    __syncthreads();
    for (int h = 128; h >= T; h >>= 1) {
      if (t < h) sh[t] += sh[t + h];
      __syncthreads();
    }
    if (t < T) mean[(long)k * kMaxTile + t] = sh[t] / (double)(hi - lo);
    __syncthreads();
  }
}

// Pull of one vertex's list: sum over entries e in [lo, hi) taken by this
// lane's sub-group (every NL-th, starting at j) of c_e * z[idx_e][col], four
// entries' loads issued before their use.
template <typename V, typename C, int T>
__device__ __forceinline__ double pull(int lo, int hi, int j, int NL, int col,
                                       const int* __restrict__ idx, const C* __restrict__ cf,
                                       const V* __restrict__ z) {
  double acc = 0.0;
  int e = lo + j;
  for (; e + 3 * NL < hi; e += 4 * NL) {
    int ix[4];
    double cv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      ix[q] = idx[e + q * NL];
      cv[q] = (double)cf[e + q * NL];
    }
    double zv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) zv[q] = (double)z[(long)ix[q] * T + col];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc += cv[q] * zv[q];
  }
  for (; e < hi; e += NL) acc += (double)cf[e] * (double)z[(long)idx[e] * T + col];
  return acc;
}

// Forward round, positions [p0, p1): y_u (kept in z) = r_u - mean + pulls
// from earlier vertices.  WAVE: one wave per vertex, its 64 / T lane
// sub-groups splitting the list and meeting by shuffles (fixed order);
// otherwise one 1024-thread block per vertex (rounds with long lists), its
// BS / T sub-groups meeting in LDS.
template <typename V, typename C, int T, bool WAVE, int BS = 256>
__global__ __launch_bounds__(BS) void k_am_fwd(int p0, int p1, const int* __restrict__ order,
                                               const int* __restrict__ in_off,
                                               const int* __restrict__ in_idx,
                                               const C* __restrict__ in_c, const V* __restrict__ r,
                                               const int* __restrict__ comp,
                                               const double* __restrict__ mean, V* __restrict__ z) {
  constexpr int NL = (WAVE ? 64 : BS) / T;
  __shared__ double sh[WAVE ? 1 : BS];
  const int t = threadIdx.x;
  const int lt = WAVE ? (t & 63) : t;
  const int p = WAVE ? p0 + blockIdx.x * 4 + (t >> 6) : p0 + blockIdx.x;
  if (p >= p1) return;                 // per wave (WAVE) or per block: no partial exits
  const int c = lt % T, j = lt / T;
  double acc = pull<V, C, T>(in_off[p], in_off[p + 1], j, NL, c, in_idx, in_c, z);
  if constexpr (WAVE) {
#pragma unroll
    for (int off = T; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  } else {
    sh[t] = acc;
    __syncthreads();
    for (int h = BS / 2; h >= T; h >>= 1) {
      if (t < h) sh[t] += sh[t + h];
      __syncthreads();
    }
    acc = sh[t];
  }
  if (j == 0) {
    const int u = order[p];
    z[(long)u * T + c] = (V)(((double)r[(long)u * T + c] - mean[(long)comp[u] * kMaxTile + c]) + acc);
  }
}

// Backward round, positions [p0, p1): z_v = y_v / W_v + pulls from later
// vertices (already final); split as in the forward round.
template <typename V, typename C, int T, bool WAVE, int BS = 256>
__global__ __launch_bounds__(BS) void k_am_bwd(int p0, int p1, const int* __restrict__ order,
                                               const int* __restrict__ out_off,
                                               const int* __restrict__ out_idx,
                                               const C* __restrict__ out_c,
                                               const C* __restrict__ inv_pivot, V* __restrict__ z) {
  constexpr int NL = (WAVE ? 64 : BS) / T;
  __shared__ double sh[WAVE ? 1 : BS];
  const int t = threadIdx.x;
  const int lt = WAVE ? (t & 63) : t;
  const int p = WAVE ? p0 + blockIdx.x * 4 + (t >> 6) : p0 + blockIdx.x;
  if (p >= p1) return;
  const int c = lt % T, j = lt / T;
  double acc = pull<V, C, T>(out_off[p], out_off[p + 1], j, NL, c, out_idx, out_c, z);
  if constexpr (WAVE) {
#pragma unroll
    for (int off = T; off < 64; off <<= 1) acc += __shfl_xor(acc, off, 64);
  } else {
    sh[t] = acc;
    __syncthreads();
    for (int h = BS / 2; h >= T; h >>= 1) {
      if (t < h) sh[t] += sh[t + h];
      __syncthreads();
    }
    acc = sh[t];
  }
  if (j == 0) {
    const int v = order[p];
    z[(long)v * T + c] = (V)((double)z[(long)v * T + c] * (double)inv_pivot[p] + acc);
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
void free_achol(AcholPre* ap) {
  if (!ap) return;
  void* ptrs[] = {ap->order,  ap->out_off, ap->out_idx, ap->out_c64, ap->out_c32, ap->in_off,
                  ap->in_idx, ap->in_c64,  ap->in_c32,  ap->ip64,    ap->ip32,    ap->mean,
                  ap->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete ap;
}

static int achol_max_rounds() {
  if (const char* e = std::getenv("NVD_ACHOL_ROUNDS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 0 && v <= 1000000) return (int)v;
  }
  return kAcholMaxRounds;
}

nvd_status ensure_achol(DevGraph* g) {
  if (g->achol) return NVD_OK;
  const int n = g->n;
  HostFactor f = factor_graph(g, achol_max_rounds());
  // forward pull lists: for position q (vertex order[q]) the entries (v, c)
  // of the earlier columns that name it
  std::vector<int> pos_of(n);
  for (int p = 0; p < n; ++p) pos_of[f.order[p]] = p;
  const size_t nf = f.col_idx.size();
  if (nf >= (size_t)INT32_MAX) {
    set_error("approximate Cholesky: factor beyond 2^31 entries");
    return NVD_E_UNSUPPORTED;
  }
  std::vector<int> in_off(n + 1, 0);
  for (size_t e = 0; e < nf; ++e) ++in_off[pos_of[f.col_idx[e]] + 1];
  for (int p = 0; p < n; ++p) in_off[p + 1] += in_off[p];
  std::vector<int> in_idx(nf), fill(in_off.begin(), in_off.end() - 1);
  std::vector<double> in_c(nf);
  for (int p = 0; p < n; ++p) {
    const int v = f.order[p];
    for (int e = f.col_off[p]; e < f.col_off[p + 1]; ++e) {
      const int q = pos_of[f.col_idx[e]];
      in_idx[fill[q]] = v;
      in_c[fill[q]] = f.col_c[e];
      ++fill[q];
    }
  }
  std::vector<float> col_c32(f.col_c.begin(), f.col_c.end()), in_c32(in_c.begin(), in_c.end());
  std::vector<float> ip32(f.inv_pivot.begin(), f.inv_pivot.end());
  AcholPre* ap = new AcholPre();
  ap->rounds = f.rounds;
  ap->grounds = f.grounds;
  ap->remainder = f.remainder;
  ap->nnz = (int64_t)nf;
  ap->round_off = f.round_off;
  const int nr = (int)f.round_off.size() - 1;
  ap->fwd_max.assign(nr, 0);
  ap->bwd_max.assign(nr, 0);
  for (int k = 0; k < nr; ++k) {
    for (int p = f.round_off[k]; p < f.round_off[k + 1]; ++p) {
      ap->fwd_max[k] = std::max(ap->fwd_max[k], in_off[p + 1] - in_off[p]);
      ap->bwd_max[k] = std::max(ap->bwd_max[k], f.col_off[p + 1] - f.col_off[p]);
    }
  }
  nvd_status st = NVD_OK;
  auto alloc = [&](void** p, size_t bytes) {
    if (st != NVD_OK) return;
    if (hipMalloc(p, std::max<size_t>(bytes, 4)) != hipSuccess) {
      set_error("approximate Cholesky: device allocation failed");
      st = NVD_E_NOMEM;
    } else {
      ap->bytes += (int64_t)bytes;
    }
  };
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (st != NVD_OK || bytes == 0) return;
    if (hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) != hipSuccess) {
      set_error("approximate Cholesky: upload failed");
      st = NVD_E_DEVICE;
    }
  };
  alloc((void**)&ap->order, sizeof(int) * n);
  alloc((void**)&ap->out_off, sizeof(int) * (n + 1));
  alloc((void**)&ap->out_idx, sizeof(int) * nf);
  alloc((void**)&ap->out_c64, sizeof(double) * nf);
  alloc((void**)&ap->out_c32, sizeof(float) * nf);
  alloc((void**)&ap->in_off, sizeof(int) * (n + 1));
  alloc((void**)&ap->in_idx, sizeof(int) * nf);
  alloc((void**)&ap->in_c64, sizeof(double) * nf);
  alloc((void**)&ap->in_c32, sizeof(float) * nf);
  alloc((void**)&ap->ip64, sizeof(double) * n);
  alloc((void**)&ap->ip32, sizeof(float) * n);
  alloc((void**)&ap->mean, sizeof(double) * (size_t)std::max(g->n_comp, 1) * kMaxTile);
  alloc((void**)&ap->part, sizeof(double) * kAmBlocks * kMaxTile);
  up(ap->order, f.order.data(), sizeof(int) * n);
  up(ap->out_off, f.col_off.data(), sizeof(int) * (n + 1));
  up(ap->out_idx, f.col_idx.data(), sizeof(int) * nf);
  up(ap->out_c64, f.col_c.data(), sizeof(double) * nf);
  up(ap->out_c32, col_c32.data(), sizeof(float) * nf);
  up(ap->in_off, in_off.data(), sizeof(int) * (n + 1));
  up(ap->in_idx, in_idx.data(), sizeof(int) * nf);
  up(ap->in_c64, in_c.data(), sizeof(double) * nf);
  up(ap->in_c32, in_c32.data(), sizeof(float) * nf);
  up(ap->ip64, f.inv_pivot.data(), sizeof(double) * n);
  up(ap->ip32, ip32.data(), sizeof(float) * n);
  if (st != NVD_OK) {
    free_achol(ap);
    return st;
  }
  g->achol = ap;
  g->bytes += ap->bytes;
  return NVD_OK;
}

// Rounds whose longest pull list reaches this take a 1024-thread block per
// vertex, so that a hub's list, which grows with every neighbour eliminated
// before it, is read 16 rows at a time (and the round's time is that of its
// longest list).
constexpr int kAmLongList = 256;

template <typename V, int T>
static void achol_rounds(const DevGraph* g, const V* r, V* z, hipStream_t s) {
  const AcholPre* ap = g->achol;
  const int nr = (int)ap->round_off.size() - 1;   // rounds, then the remainder
  using C = V;
  const C* in_c = sizeof(V) == 8 ? (const C*)ap->in_c64 : (const C*)ap->in_c32;
  const C* out_c = sizeof(V) == 8 ? (const C*)ap->out_c64 : (const C*)ap->out_c32;
  const C* ip = sizeof(V) == 8 ? (const C*)ap->ip64 : (const C*)ap->ip32;
  for (int k = 0; k < nr; ++k) {
    const int p0 = ap->round_off[k], p1 = ap->round_off[k + 1];
    if (p1 <= p0) continue;
    if (ap->fwd_max[k] >= kAmLongList)
      k_am_fwd<V, C, T, false, 1024><<<p1 - p0, 1024, 0, s>>>(p0, p1, ap->order, ap->in_off, ap->in_idx,
                                                               in_c, r, g->comp, ap->mean, z);
    else
      k_am_fwd<V, C, T, true><<<(p1 - p0 + 3) / 4, 256, 0, s>>>(p0, p1, ap->order, ap->in_off,
                                                                ap->in_idx, in_c, r, g->comp, ap->mean, z);
  }
  for (int k = nr - 1; k >= 0; --k) {
    const int p0 = ap->round_off[k], p1 = ap->round_off[k + 1];
    if (p1 <= p0) continue;
    if (ap->bwd_max[k] >= kAmLongList)
      k_am_bwd<V, C, T, false, 1024><<<p1 - p0, 1024, 0, s>>>(p0, p1, ap->order, ap->out_off,
                                                               ap->out_idx, out_c, ip, z);
    else
      k_am_bwd<V, C, T, true><<<(p1 - p0 + 3) / 4, 256, 0, s>>>(p0, p1, ap->order, ap->out_off,
                                                                ap->out_idx, out_c, ip, z);
  }
}

template <typename V>
static nvd_status achol_solve_t(DevGraph* g, int T, const V* r, V* z, hipStream_t s) {
  AcholPre* ap = g->achol;
  const int n = g->n;
  // component means of r
  if (g->n_comp == 1) {
    k_am_part<V><<<kAmBlocks, 256, 0, s>>>(n, T, r, ap->part);
    k_am_total<<<1, 64, 0, s>>>(n, T, kAmBlocks, ap->part, ap->mean);
  } else {
    k_am_comp<V><<<std::min(g->n_comp, 4096), 256, 0, s>>>(g->n_comp, T, g->comp_perm, g->comp_off, r,
                                                           ap->mean);
  }
  switch (T) {
    case 1: achol_rounds<V, 1>(g, r, z, s); break;
    case 2: achol_rounds<V, 2>(g, r, z, s); break;
    case 4: achol_rounds<V, 4>(g, r, z, s); break;
    case 8: achol_rounds<V, 8>(g, r, z, s); break;
    case 16: achol_rounds<V, 16>(g, r, z, s); break;
    case 32: achol_rounds<V, 32>(g, r, z, s); break;
    default: achol_rounds<V, 64>(g, r, z, s); break;
  }
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

nvd_status achol_solve(DevGraph* g, int prec, int T, const void* r, void* z, hipStream_t s) {
  if (!g->achol) {
    set_error("approximate Cholesky preconditioner: not set up");
    return NVD_E_DEVICE;
  }
  if (T < 1 || T > kMaxTile || (T & (T - 1))) {
    set_error("approximate Cholesky preconditioner: tile must be a power of two up to 64");
    return NVD_E_ARG;
  }
  return prec == 0 ? achol_solve_t<double>(g, T, static_cast<const double*>(r), static_cast<double*>(z), s)
                   : achol_solve_t<float>(g, T, static_cast<const float*>(r), static_cast<float*>(z), s);
}

}  // namespace nvd
