// Augmented spanning-tree preconditioner (Table 1's "Aug Tree"): z = L_H^+ r
// for H = a spanning forest T of the graph plus the k off-forest edges of
// largest stretch.  T is, on unit weights, the breadth-first forest from
// each component's smallest node; on weighted graphs, of that forest and the
// maximum-weight spanning forest, the one whose off-forest edges have the
// smaller total stretch.  The k edges are solved with the forest exactly by
// the Woodbury identity: with U their signed incidence columns and W their
// weights, L_H^+ = L_T^+ - Y C^-1 Y^T, Y = L_T^+ U (k forest solves at
// set-up), C = W^-1 + U^T Y (k x k, inverted on the host); one application is
// a forest solve, s = U^T z, t = C^-1 s and z -= Y t.
//
// On a tree, L_T x = r has a closed solution (the flow formula): the flow on
// the edge from v to its parent is the sum f_v of r over v's subtree, the
// potential drops by f_v / w_v across that edge, and the root is held at 0.
// Both sums are prefix sums over an Euler tour of the forest (every node
// entered at tin[v] and left at tout[v], 2n events; a component is the
// contiguous tour range of its root, each node counted twice):
//   f_v = S1[tout_v] - S1[tin_v] + r_v - mu_c size_v,
//         S1 = prefix of (r_v at tin_v, 0 at tout_v), mu_c = mean of r over
//         v's component c, size_v = (tout_v - tin_v + 1) / 2
//   x_v = S2[tin_v],  S2 = prefix of (+f_v/w_v at tin_v, -f_v/w_v at tout_v)
// so one solve is two scans over 2n x T values, O(n) work in O(log n)
// depth whatever the depth of the tree.  The scans run in FP64 (prefix sums
// cancel) with a chunk and segment split that depend only on the tour
// length and the tile, so results repeat bit for bit.  The second scan
// writes x_v from its running sum at tin_v (tnode: the node entered at each
// tour position) instead of storing S2 for a separate gather.
//
// Subtracting mu_c makes the map the pseudoinverse on r's component means
// too (constants go to zero).  Without it the solve would be the grounded
// inverse, whose image of a constant grows like n times the tree depth: the
// small mean that rounding leaves in the solver's residual (FP32 above all)
// would swamp z.  Roots get potential 0, so z is L_T^+ r plus a constant
// per component, which does not change r^T z for r orthogonal to the
// constants and which the solver's projections remove.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <queue>
#include <vector>

#include "device_common.hpp"

namespace nvd {

// Tour rows per scan block: 2048 on large forests, down to 256 on small
// ones so that a short tour still spreads over many blocks (each lane walks
// chunk / (256 / T) rows in sequence).
constexpr int kScanChunkMax = 2048;
constexpr int kScanChunkMin = 256;
static int scan_chunk(long rows) {
  int c = kScanChunkMin;
  while (c < kScanChunkMax && (long)c * 1024 < rows) c <<= 1;
  return c;
}

// ---------------------------------------------------------------------------
// host: spanning forests, their stretch, the Euler tour
// ---------------------------------------------------------------------------
// Breadth-first forest, a root per component: its smallest node.
static int forest_bfs(const DevGraph* g, std::vector<int>& parent, std::vector<double>& pw) {
  const int n = g->n;
  const std::vector<int>& rp = g->h_rp;
  const std::vector<int>& ci = g->h_ci;
  const bool weighted = !g->h_w.empty();
  std::vector<char> seen(n, 0);
  std::vector<int> queue;
  queue.reserve(n);
  int tree_edges = 0;
  for (int s = 0; s < n; ++s) {
    if (seen[s]) continue;
    seen[s] = 1;
    size_t head = queue.size();
    queue.push_back(s);
    for (; head < queue.size(); ++head) {
      const int v = queue[head];
      for (int e = rp[v]; e < rp[v + 1]; ++e) {
        const int u = ci[e];
        if (seen[u]) continue;
        seen[u] = 1;
        parent[u] = v;
        pw[u] = weighted ? g->h_w[e] : 1.0;
        queue.push_back(u);
        ++tree_edges;
      }
    }
  }
  return tree_edges;
}

// Maximum-weight spanning forest: Prim from each component's smallest node,
// the heaviest edge leaving the tree first; among equal weights the earliest
// discovered edge (so equal weights give the breadth-first forest).
static int forest_max_weight(const DevGraph* g, std::vector<int>& parent, std::vector<double>& pw) {
  const int n = g->n;
  const std::vector<int>& rp = g->h_rp;
  const std::vector<int>& ci = g->h_ci;
  struct Cand {
    double w;
    long seq;
    int v, u;
  };
  auto lower = [](const Cand& a, const Cand& b) {
    return a.w < b.w || (a.w == b.w && a.seq > b.seq);
  };
  std::priority_queue<Cand, std::vector<Cand>, decltype(lower)> heap(lower);
  std::vector<char> seen(n, 0);
  long seq = 0;
  int tree_edges = 0;
  auto reach = [&](int v) {
    for (int e = rp[v]; e < rp[v + 1]; ++e)
      if (!seen[ci[e]]) heap.push(Cand{g->h_w[e], seq++, v, ci[e]});
  };
  for (int s = 0; s < n; ++s) {
    if (seen[s]) continue;
    seen[s] = 1;
    reach(s);
    while (!heap.empty()) {
      const Cand c = heap.top();
      heap.pop();
      if (seen[c.u]) continue;
      seen[c.u] = 1;
      parent[c.u] = c.v;
      pw[c.u] = c.w;
      ++tree_edges;
      reach(c.u);
    }
  }
  return tree_edges;
}

// Children of every node in a forest (CSR by parent).
static void forest_children(int n, const std::vector<int>& parent, std::vector<int>& coff,
                            std::vector<int>& kids) {
  coff.assign(n + 1, 0);
  for (int v = 0; v < n; ++v)
    if (parent[v] >= 0) ++coff[parent[v] + 1];
  for (int v = 0; v < n; ++v) coff[v + 1] += coff[v];
  kids.assign(std::max(coff[n], 1), 0);
  std::vector<int> fill(coff.begin(), coff.end() - 1);
  for (int v = 0; v < n; ++v)
    if (parent[v] >= 0) kids[fill[parent[v]]++] = v;
}

// One edge off the forest and its stretch.
struct OffEdge {
  double stretch;
  int u, v;
  double w;
};

// Total stretch of the edges off a forest: the sum over them of w_e times
// the resistance of the forest path between their ends, which bounds the
// condition number of the forest-preconditioned Laplacian.  Forest paths
// through lowest common ancestors, found offline (Tarjan: a depth-first
// walk that merges each finished subtree into its parent's set).  With
// `edges`, every off-forest edge is also listed once with its stretch.
static double forest_stretch(const DevGraph* g, const std::vector<int>& parent,
                             const std::vector<double>& pw, std::vector<OffEdge>* edges = nullptr) {
  const int n = g->n;
  const std::vector<int>& rp = g->h_rp;
  const std::vector<int>& ci = g->h_ci;
  const bool weighted = !g->h_w.empty();
  std::vector<int> coff, kids;
  forest_children(n, parent, coff, kids);
  std::vector<int> uf(n), anc(n);
  std::vector<char> done(n, 0);
  std::vector<double> dist(n, 0.0);
  auto find = [&](int v) {
    while (uf[v] != v) {
      uf[v] = uf[uf[v]];
      v = uf[v];
    }
    return v;
  };
  double stretch = 0.0;
  std::vector<std::pair<int, int>> stack;
  for (int root = 0; root < n; ++root) {
    if (parent[root] >= 0) continue;
    uf[root] = root;
    anc[root] = root;
    stack.emplace_back(root, coff[root]);
    while (!stack.empty()) {
      auto& top = stack.back();
      const int v = top.first;
      if (top.second < coff[v + 1]) {
        const int c = kids[top.second++];
        dist[c] = dist[v] + 1.0 / pw[c];
        uf[c] = c;
        anc[c] = c;
        stack.emplace_back(c, coff[c]);
        continue;
      }
      done[v] = 1;
      for (int e = rp[v]; e < rp[v + 1]; ++e) {
        const int u = ci[e];
        if (!done[u] || u == v || parent[u] == v || parent[v] == u) continue;
        const int l = anc[find(u)];
        const double w = weighted ? g->h_w[e] : 1.0;
        const double se = w * (dist[u] + dist[v] - 2.0 * dist[l]);
        stretch += se;
        if (edges) edges->push_back(OffEdge{se, u, v, w});
      }
      stack.pop_back();
      if (parent[v] >= 0) {
        uf[find(v)] = find(parent[v]);
        anc[find(parent[v])] = parent[v];
      }
    }
  }
  return stretch;
}

// Off-forest edges added back to the forest (the augmentation): the
// kAugMax of largest stretch, fewer where n x k doubles would pass 512 MB;
// NVD_TREE_AUG sets the count (0: none).
constexpr int kAugMax = 256;
static int aug_count(const DevGraph* g, long n_off) {
  long k = kAugMax;
  if (const char* e = std::getenv("NVD_TREE_AUG")) k = std::max(0L, std::strtol(e, nullptr, 10));
  k = std::min(k, n_off);
  k = std::min(k, (1L << 26) / std::max(1, g->n));
  return (int)k;
}

// host: spanning forest (the breadth-first one on unit weights; on weighted
// graphs, of the breadth-first and the maximum-weight forest the one of
// smaller total stretch) and its Euler tour
static nvd_status build_tree(DevGraph* g) {
  const int n = g->n;
  const bool weighted = !g->h_w.empty();
  std::vector<int> parent(n, -1);
  std::vector<double> pw(n, 0.0);
  int tree_edges = forest_bfs(g, parent, pw);
  if (weighted) {
    std::vector<int> parent2(n, -1);
    std::vector<double> pw2(n, 0.0);
    const int e2 = forest_max_weight(g, parent2, pw2);
    if (forest_stretch(g, parent2, pw2) < forest_stretch(g, parent, pw)) {
      parent.swap(parent2);
      pw.swap(pw2);
      tree_edges = e2;
    }
  }
  // the augmentation: the off-forest edges of largest stretch
  std::vector<OffEdge> aug;
  const long n_off = (long)g->nnz / 2 - tree_edges;
  const int k_aug = aug_count(g, n_off);
  if (k_aug > 0) {
    forest_stretch(g, parent, pw, &aug);
    auto larger = [](const OffEdge& a, const OffEdge& b) {
      if (a.stretch != b.stretch) return a.stretch > b.stretch;
      return a.u != b.u ? a.u < b.u : a.v < b.v;
    };
    if ((long)aug.size() > k_aug) {
      std::nth_element(aug.begin(), aug.begin() + k_aug, aug.end(), larger);
      aug.resize(k_aug);
    }
    std::sort(aug.begin(), aug.end(), larger);
  }
  // children lists (CSR), then an iterative depth-first Euler tour
  std::vector<int> coff, kids;
  forest_children(n, parent, coff, kids);
  std::vector<int> tin(n), tout(n), root_of(n);
  std::vector<std::pair<int, int>> stack;
  int t = 0;
  for (int root = 0; root < n; ++root) {
    if (parent[root] >= 0) continue;
    root_of[root] = root;
    tin[root] = t++;
    stack.emplace_back(root, coff[root]);
    while (!stack.empty()) {
      auto& top = stack.back();
      const int v = top.first;
      if (top.second < coff[v + 1]) {
        const int c = kids[top.second++];
        root_of[c] = root_of[v];
        tin[c] = t++;
        stack.emplace_back(c, coff[c]);
      } else {
        tout[v] = t++;
        stack.pop_back();
      }
    }
  }
  std::vector<double> winv(n);
  std::vector<int> rbeg(n), rend(n), tnode(2 * (size_t)n, -1);
  for (int v = 0; v < n; ++v) {
    winv[v] = parent[v] >= 0 ? 1.0 / pw[v] : 0.0;
    rbeg[v] = tin[root_of[v]];
    rend[v] = tout[root_of[v]];
    tnode[tin[v]] = v;
  }
  TreePre* tp = new TreePre();
  tp->n_tree_edges = tree_edges;
  tp->k_aug = (int)aug.size();
  for (const OffEdge& a : aug) {
    tp->aug_u.push_back(a.u);
    tp->aug_v.push_back(a.v);
    tp->aug_w.push_back(a.w);
  }
  nvd_status st = NVD_OK;
  auto al = [&](void** p, size_t bytes) {
    if (st == NVD_OK && hipMalloc(p, std::max<size_t>(bytes, 8)) != hipSuccess) {
      set_error("tree preconditioner: out of device memory");
      st = NVD_E_NOMEM;
    }
  };
  al((void**)&tp->tin, sizeof(int) * n);
  al((void**)&tp->tout, sizeof(int) * n);
  al((void**)&tp->winv, sizeof(double) * n);
  al((void**)&tp->rbeg, sizeof(int) * n);
  al((void**)&tp->rend, sizeof(int) * n);
  al((void**)&tp->tnode, sizeof(int) * 2 * (size_t)n);
  if (tp->k_aug > 0) {
    al((void**)&tp->aug_uv, sizeof(int) * 2 * (size_t)tp->k_aug);
    al((void**)&tp->aug_st, sizeof(double) * 2 * (size_t)tp->k_aug * kMaxTile);
  }
  if (st == NVD_OK &&
      (hipMemcpy(tp->tin, tin.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(tp->tout, tout.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(tp->rbeg, rbeg.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(tp->rend, rend.data(), sizeof(int) * n, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(tp->tnode, tnode.data(), sizeof(int) * 2 * (size_t)n, hipMemcpyHostToDevice) != hipSuccess ||
       hipMemcpy(tp->winv, winv.data(), sizeof(double) * n, hipMemcpyHostToDevice) != hipSuccess)) {
    set_error("tree preconditioner: upload failed");
    st = NVD_E_DEVICE;
  }
  if (st == NVD_OK && tp->k_aug > 0) {
    std::vector<int> uv(tp->aug_u);
    uv.insert(uv.end(), tp->aug_v.begin(), tp->aug_v.end());
    if (hipMemcpy(tp->aug_uv, uv.data(), sizeof(int) * uv.size(), hipMemcpyHostToDevice) != hipSuccess) {
      set_error("tree preconditioner: upload failed");
      st = NVD_E_DEVICE;
    }
  }
  if (st != NVD_OK) {
    free_tree(tp);
    return st;
  }
  g->tree = tp;
  return NVD_OK;
}

void free_tree(TreePre* tp) {
  if (!tp) return;
  void* ptrs[] = {tp->tin,  tp->tout, tp->winv, tp->rbeg,   tp->rend,   tp->tnode,
                  tp->E,    tp->S,    tp->part, tp->aug_uv, tp->aug_st, tp->aug_Y,
                  tp->aug_Cinv};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete tp;
}

bool use_tree(const DevGraph* g, uint32_t flags) {
  if (flags & NVD_PRECOND_TREE) return true;
  if (!(flags & NVD_PRECOND_AUTO)) return false;
  // edges off a spanning forest: m - (n - c); each adds at most one PCG
  // iteration to the tree's exact solve, and none if the augmentation
  // takes them all
  const long off = (long)g->nnz / 2 - g->n + g->n_comp;
  return off * 100 <= (long)g->n || off <= aug_count(g, off);
}

static nvd_status build_aug(DevGraph* g);

nvd_status ensure_tree(DevGraph* g, int T) {
  if (!g->tree) NVD_TRY(build_tree(g));
  TreePre* tp = g->tree;
  if (tp->cap_tile >= T) {
    if (tp->k_aug > 0 && !tp->aug_Y) NVD_TRY(build_aug(g));
    return NVD_OK;
  }
  void* ptrs[] = {tp->E, tp->S, tp->part};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  tp->E = tp->S = tp->part = nullptr;
  const size_t rows = 2 * (size_t)g->n;
  const size_t nchunk = (rows + kScanChunkMin - 1) / kScanChunkMin;   // the most any chunk size needs
  NVD_HIP(hipMalloc((void**)&tp->E, sizeof(double) * rows * T));
  NVD_HIP(hipMalloc((void**)&tp->S, sizeof(double) * rows * T));
  NVD_HIP(hipMalloc((void**)&tp->part, sizeof(double) * nchunk * T));
  tp->cap_tile = T;
  if (tp->k_aug > 0 && !tp->aug_Y) NVD_TRY(build_aug(g));
  return NVD_OK;
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------
// E[tin_v] = r_v, E[tout_v] = 0
template <typename V>
__global__ void k_tour_put(int n, int T, const V* __restrict__ r, const int* __restrict__ tin,
                           const int* __restrict__ tout, double* __restrict__ E) {
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long v = e / T;
    const int c = (int)(e % T);
    E[(long)tin[v] * T + c] = (double)r[e];
    E[(long)tout[v] * T + c] = 0.0;
  }
}

// f_v = S[tout_v] - S[tin_v] + r_v - mu size_v; y = f_v / w_v;
// E[tin_v] = y, E[tout_v] = -y
template <typename V>
__global__ void k_tour_flow(int n, int T, const V* __restrict__ r, const int* __restrict__ tin,
                            const int* __restrict__ tout, const int* __restrict__ rbeg,
                            const int* __restrict__ rend, const double* __restrict__ winv,
                            const double* __restrict__ S, double* __restrict__ E) {
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long v = e / T;
    const int c = (int)(e % T);
    const int ti = tin[v], to = tout[v], rb = rbeg[v], re = rend[v];
    const long a = (long)ti * T + c, b = (long)to * T + c;
    // component sum: the inclusive prefix over the root's tour range
    const double csum = S[(long)re * T + c] - (rb > 0 ? S[(long)(rb - 1) * T + c] : 0.0);
    const double mu = csum / (double)((re - rb + 1) / 2);
    const double f = S[b] - S[a] + (double)r[e] - mu * (double)((to - ti + 1) / 2);
    const double y = f * winv[v];
    E[a] = y;
    E[b] = -y;
  }
}

// Scan of a rows x T row-major array along the rows, per column.  Block b
// owns rows [b*chunk, (b+1)*chunk); inside it lane j of a column (NJ = 256/T
// lanes) owns a contiguous segment.  Phase 1: chunk sums; phase 2: exclusive
// scan of the chunk sums per column; phase 3: segment prefixes plus the
// chunk offset.  The split is the same in phases 1 and 3.
__device__ __forceinline__ void seg_of(int T, long rows, int chunk, int b, long* lo, long* hi, int* c) {
  const int t = threadIdx.x;
  const int NJ = 256 / T;
  const int j = t / T;
  *c = t % T;
  const long seg = (chunk + NJ - 1) / NJ;
  const long base = (long)b * chunk;
  const long end = min(rows, base + chunk);
  *lo = min(end, base + j * seg);
  *hi = min(end, *lo + seg);
}

// Sum of E[i][c] over i in [lo, hi), loads issued 8 rows at a time (one
// load in flight per lane left the scans latency-bound), added in row order.
__device__ __forceinline__ double seg_sum(const double* __restrict__ E, long lo, long hi, int T, int c) {
  constexpr int B = 8;
  double s = 0.0;
  long i = lo;
  for (; i + B <= hi; i += B) {
    double e[B];
#pragma unroll
    for (int k = 0; k < B; ++k) e[k] = E[(i + k) * T + c];
#pragma unroll
    for (int k = 0; k < B; ++k) s += e[k];
  }
  for (; i < hi; ++i) s += E[i * T + c];
  return s;
}

__global__ __launch_bounds__(256) void k_scan_sums(long rows, int T, int chunk,
                                                   const double* __restrict__ E,
                                                   double* __restrict__ part) {
  __shared__ double sh[256];
  long lo, hi;
  int c;
  seg_of(T, rows, chunk, blockIdx.x, &lo, &hi, &c);
  sh[threadIdx.x] = seg_sum(E, lo, hi, T, c);
  __syncthreads();
  if ((int)threadIdx.x < T) {
    double tot = 0.0;
    for (int j = 0; j < 256 / T; ++j) tot += sh[j * T + threadIdx.x];
    part[(long)blockIdx.x * T + threadIdx.x] = tot;
  }
}

// one block per column: exclusive scan of part[b][c] over b, in place
__global__ __launch_bounds__(256) void k_scan_offsets(int nchunk, int T, double* __restrict__ part) {
  __shared__ double sh[256];
  const int c = blockIdx.x;
  const int t = threadIdx.x;
  const int per = (nchunk + 255) / 256;
  const int b0 = min(nchunk, t * per), b1 = min(nchunk, b0 + per);
  double s = 0.0;
  for (int b = b0; b < b1; ++b) s += part[(long)b * T + c];
  sh[t] = s;
  __syncthreads();
  if (t == 0) {
    double run = 0.0;
    for (int i = 0; i < 256; ++i) {
      const double v = sh[i];
      sh[i] = run;
      run += v;
    }
  }
  __syncthreads();
  double run = sh[t];
  for (int b = b0; b < b1; ++b) {
    const double v = part[(long)b * T + c];
    part[(long)b * T + c] = run;
    run += v;
  }
}

// TO_Z: instead of S, write the running sum at the position where node v is
// entered to z_v (the second scan, whose prefix is only read there).
template <typename V, bool TO_Z>
__global__ __launch_bounds__(256) void k_scan_apply(long rows, int T, int chunk,
                                                    const double* __restrict__ E,
                                                    const double* __restrict__ part,
                                                    double* __restrict__ S,
                                                    const int* __restrict__ tnode,
                                                    V* __restrict__ z) {
  __shared__ double sh[256];
  long lo, hi;
  int c;
  seg_of(T, rows, chunk, blockIdx.x, &lo, &hi, &c);
  sh[threadIdx.x] = seg_sum(E, lo, hi, T, c);
  __syncthreads();
  const int j = threadIdx.x / T;
  double run = part[(long)blockIdx.x * T + c];
  for (int q = 0; q < j; ++q) run += sh[q * T + c];
  constexpr int B = 8;
  long i = lo;
  for (; i + B <= hi; i += B) {
    double e[B];
    int tv[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      e[k] = E[(i + k) * T + c];
      if constexpr (TO_Z) tv[k] = tnode[i + k];
    }
#pragma unroll
    for (int k = 0; k < B; ++k) {
      run += e[k];
      if constexpr (TO_Z) {
        if (tv[k] >= 0) z[(long)tv[k] * T + c] = (V)run;
      } else {
        S[(i + k) * T + c] = run;
      }
    }
  }
  for (; i < hi; ++i) {
    run += E[i * T + c];
    if constexpr (TO_Z) {
      const int v = tnode[i];
      if (v >= 0) z[(long)v * T + c] = (V)run;
    } else {
      S[i * T + c] = run;
    }
  }
}

template <typename V, bool TO_Z>
static void scan_rows(long rows, int T, const double* E, double* part, double* S, const int* tnode,
                      V* z, hipStream_t s) {
  const int chunk = scan_chunk(rows);
  const int nchunk = (int)((rows + chunk - 1) / chunk);
  k_scan_sums<<<nchunk, 256, 0, s>>>(rows, T, chunk, E, part);
  k_scan_offsets<<<T, 256, 0, s>>>(nchunk, T, part);
  k_scan_apply<V, TO_Z><<<nchunk, 256, 0, s>>>(rows, T, chunk, E, part, S, tnode, z);
}

// ---------------------------------------------------------------------------
// augmentation (Woodbury): z -= Y C^-1 U^T z, with U the signed incidence
// columns of the k added edges, Y = L_T^+ U and C = W^-1 + U^T Y
// ---------------------------------------------------------------------------
// s[f][c] = z[u_f][c] - z[v_f][c]
template <typename V>
__global__ void k_aug_s(int T, int k, const int* __restrict__ uv, const V* __restrict__ z,
                        double* __restrict__ sv) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * T) return;
  const int f = i / T, c = i % T;
  sv[(size_t)f * kMaxTile + c] = (double)z[(long)uv[f] * T + c] - (double)z[(long)uv[k + f] * T + c];
}

// out[i][c] = sum_f A[i][f] B[f][c] for rows i < rows, columns c < T (A
// row-major with k columns, B with row stride kMaxTile), in a fixed order:
// B staged in LDS 64 rows at a time, four partial sums per thread.  SUB:
// out -= (V), else out = (double).  One thread per (row, column).
template <typename O, bool SUB>
__global__ __launch_bounds__(256) void k_aug_gemm(long rows, int T, int k, const double* __restrict__ A,
                                                  const double* __restrict__ B, O* __restrict__ out) {
  constexpr int FC = 64;
  __shared__ double bl[FC * kMaxTile];
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  const long i = e / T;
  const int c = (int)(e % T);
  const bool live = i < rows;
  const double* a = A + (live ? i : 0) * (long)k;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int f0 = 0; f0 < k; f0 += FC) {
    const int fc = min(FC, k - f0);
    __syncthreads();
    for (int q = threadIdx.x; q < fc * T; q += 256) bl[(q / T) * kMaxTile + q % T] = B[(size_t)(f0 + q / T) * kMaxTile + q % T];
    __syncthreads();
    if (live) {
      int j = 0;
      for (; j + 3 < fc; j += 4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += a[f0 + j + u] * bl[(j + u) * kMaxTile + c];
      }
      for (; j < fc; ++j) acc[0] += a[f0 + j] * bl[j * kMaxTile + c];
    }
  }
  if (!live) return;
  const double v = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  if constexpr (SUB)
    out[e] = (O)((double)out[e] - v);
  else
    out[i * kMaxTile + c] = v;
}

// Set-up helpers: a tile of U's columns f0 .. f0 + T - 1 (zero beyond k),
// the solved tile into Y's columns, and U^T Y.
__global__ void k_aug_zero(long len, double* __restrict__ a) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (long)gridDim.x * blockDim.x)
    a[i] = 0.0;
}
__global__ void k_aug_rhs(int T, int f0, int k, const int* __restrict__ uv, double* __restrict__ ut) {
  const int c = threadIdx.x;
  if (c >= T || f0 + c >= k) return;
  ut[(long)uv[f0 + c] * T + c] = 1.0;
  ut[(long)uv[k + f0 + c] * T + c] = -1.0;
}
__global__ void k_aug_store(int n, int T, int f0, int k, const double* __restrict__ yt,
                            double* __restrict__ Y) {
  const long tot = (long)n * T;
  for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < tot; e += (long)gridDim.x * blockDim.x) {
    const long v = e / T;
    const int c = (int)(e % T);
    if (f0 + c < k) Y[v * k + f0 + c] = yt[e];
  }
}
__global__ void k_aug_gram(int k, const int* __restrict__ uv, const double* __restrict__ Y,
                           double* __restrict__ G) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k * k) return;
  const int e = i / k, f = i % k;
  G[i] = Y[(long)uv[e] * k + f] - Y[(long)uv[k + e] * k + f];
}

template <typename V>
static nvd_status tree_solve_t(DevGraph* g, int T, const V* r, V* z, hipStream_t s) {
  TreePre* tp = g->tree;
  const int n = g->n;
  const long rows = 2L * n;
  const int grid = (int)std::min<long>(4096, ((long)n * T + 255) / 256);
  k_tour_put<V><<<std::max(grid, 1), 256, 0, s>>>(n, T, r, tp->tin, tp->tout, tp->E);
  scan_rows<V, false>(rows, T, tp->E, tp->part, tp->S, nullptr, (V*)nullptr, s);
  k_tour_flow<V><<<std::max(grid, 1), 256, 0, s>>>(n, T, r, tp->tin, tp->tout, tp->rbeg, tp->rend,
                                                   tp->winv, tp->S, tp->E);
  scan_rows<V, true>(rows, T, tp->E, tp->part, nullptr, tp->tnode, z, s);
  if (tp->aug_Y) {
    // the augmentation: z -= Y C^-1 U^T z (Woodbury)
    const int k = tp->k_aug;
    double* sv = tp->aug_st;
    double* tv = tp->aug_st + (size_t)k * kMaxTile;
    const int kt = (k * T + 255) / 256;
    k_aug_s<V><<<kt, 256, 0, s>>>(T, k, tp->aug_uv, z, sv);
    k_aug_gemm<double, false><<<kt, 256, 0, s>>>(k, T, k, tp->aug_Cinv, sv, tv);
    k_aug_gemm<V, true><<<(int)(((long)n * T + 255) / 256), 256, 0, s>>>(n, T, k, tp->aug_Y, tv, z);
  }
  NVD_HIP(hipGetLastError());
  return NVD_OK;
}

// Y = L_T^+ U by tree solves of U's columns, a tile at a time; C = W^-1 +
// U^T Y on the host, inverted by Cholesky.  If C is not numerically
// positive definite the augmentation is dropped (plain forest).
static nvd_status build_aug(DevGraph* g) {
  TreePre* tp = g->tree;
  const int n = g->n, k = tp->k_aug, T = tp->cap_tile;
  const hipStream_t s = nullptr;
  double *ut = nullptr, *yt = nullptr, *Y = nullptr, *G = nullptr;
  nvd_status st = NVD_OK;
  auto al = [&](double** p, size_t count) {
    if (st == NVD_OK && hipMalloc((void**)p, sizeof(double) * std::max<size_t>(count, 1)) != hipSuccess) {
      set_error("tree preconditioner: out of device memory (augmentation)");
      st = NVD_E_NOMEM;
    }
  };
  al(&ut, (size_t)n * T);
  al(&yt, (size_t)n * T);
  al(&Y, (size_t)n * k);
  al(&G, (size_t)k * k);
  const int grid = (int)std::min<long>(4096, ((long)n * T + 255) / 256);
  for (int f0 = 0; st == NVD_OK && f0 < k; f0 += T) {
    k_aug_zero<<<std::max(grid, 1), 256, 0, s>>>((long)n * T, ut);
    k_aug_rhs<<<1, 64, 0, s>>>(T, f0, k, tp->aug_uv, ut);
    st = tree_solve_t<double>(g, T, ut, yt, s);
    if (st == NVD_OK) k_aug_store<<<std::max(grid, 1), 256, 0, s>>>(n, T, f0, k, yt, Y);
  }
  std::vector<double> C((size_t)k * k);
  if (st == NVD_OK) {
    k_aug_gram<<<(k * k + 255) / 256, 256, 0, s>>>(k, tp->aug_uv, Y, G);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpy(C.data(), G, sizeof(double) * C.size(), hipMemcpyDeviceToHost) != hipSuccess) {
      set_error("tree preconditioner: augmentation set-up failed");
      st = NVD_E_DEVICE;
    }
  }
  (void)hipFree(ut);
  (void)hipFree(yt);
  (void)hipFree(G);
  if (st != NVD_OK) {
    (void)hipFree(Y);
    return st;
  }
  // C = W^-1 + U^T Y, symmetrised; Cholesky C = L L^T; C^-1 column by column
  for (int e = 0; e < k; ++e) C[(size_t)e * k + e] += 1.0 / tp->aug_w[e];
  for (int e = 0; e < k; ++e)
    for (int f = 0; f < e; ++f) {
      const double m = 0.5 * (C[(size_t)e * k + f] + C[(size_t)f * k + e]);
      C[(size_t)e * k + f] = C[(size_t)f * k + e] = m;
    }
  std::vector<double> L((size_t)k * k, 0.0);
  bool spd = true;
  for (int j = 0; j < k && spd; ++j) {
    double d = C[(size_t)j * k + j];
    for (int q = 0; q < j; ++q) d -= L[(size_t)j * k + q] * L[(size_t)j * k + q];
    if (!(d > 0.0) || !std::isfinite(d)) {
      spd = false;
      break;
    }
    const double ljj = std::sqrt(d);
    L[(size_t)j * k + j] = ljj;
    for (int i = j + 1; i < k; ++i) {
      double a = C[(size_t)i * k + j];
      for (int q = 0; q < j; ++q) a -= L[(size_t)i * k + q] * L[(size_t)j * k + q];
      L[(size_t)i * k + j] = a / ljj;
    }
  }
  if (!spd) {
    (void)hipFree(Y);
    tp->k_aug = 0;
    return NVD_OK;
  }
  std::vector<double> Cinv((size_t)k * k), col(k);
  for (int j = 0; j < k; ++j) {
    for (int i = 0; i < k; ++i) {   // L y = e_j
      double a = i == j ? 1.0 : 0.0;
      for (int q = 0; q < i; ++q) a -= L[(size_t)i * k + q] * col[q];
      col[i] = a / L[(size_t)i * k + i];
    }
    for (int i = k - 1; i >= 0; --i) {   // L^T x = y
      double a = col[i];
      for (int q = i + 1; q < k; ++q) a -= L[(size_t)q * k + i] * col[q];
      col[i] = a / L[(size_t)i * k + i];
    }
    for (int i = 0; i < k; ++i) Cinv[(size_t)i * k + j] = col[i];
  }
  if (hipMalloc((void**)&tp->aug_Cinv, sizeof(double) * Cinv.size()) != hipSuccess ||
      hipMemcpy(tp->aug_Cinv, Cinv.data(), sizeof(double) * Cinv.size(), hipMemcpyHostToDevice) !=
          hipSuccess) {
    (void)hipFree(Y);
    set_error("tree preconditioner: augmentation upload failed");
    return NVD_E_DEVICE;
  }
  tp->aug_Y = Y;
  return NVD_OK;
}

nvd_status tree_solve(DevGraph* g, int prec, int T, const void* r, void* z, hipStream_t s) {
  if (!g->tree || g->tree->cap_tile < T) {
    set_error("tree preconditioner: not set up for this tile");
    return NVD_E_DEVICE;
  }
  return prec == 0 ? tree_solve_t<double>(g, T, static_cast<const double*>(r), static_cast<double*>(z), s)
                   : tree_solve_t<float>(g, T, static_cast<const float*>(r), static_cast<float*>(z), s);
}

}  // namespace nvd
