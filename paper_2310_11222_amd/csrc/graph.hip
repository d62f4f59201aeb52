// Graph handle: host validation of the CSR, self-loop removal, upload,
// weighted degrees and inverse degrees (on the device), connected
// components (host union-find), the split-row work list, and the cached
// solver workspace.  The host passes run on row ranges in parallel.
//
// The paper builds L = D - A from the simplified (undirected, simple) graph
// and does not count this preprocessing in its timings (section 5.2).
#include <algorithm>
#include <cmath>
#include <climits>
#include <cstring>
#include <numeric>
#include <thread>

#include "device_common.hpp"

namespace nvd {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }
const char* get_error() { return g_err.c_str(); }

template <typename T>
static nvd_status dalloc(T** p, size_t count, int64_t* bytes) {
  *p = nullptr;
  if (count == 0) count = 1;
  NVD_HIP(hipMalloc((void**)p, count * sizeof(T)));
  if (bytes) *bytes += (int64_t)(count * sizeof(T));
  return NVD_OK;
}

__global__ void k_degree(int n, const int* rp, const double* w64, float* w32, double* deg64,
                         float* deg32, double* invd64, float* invd32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int lo = rp[i], hi = rp[i + 1];
  double d = 0.0;
  if (w64) {
    for (int e = lo; e < hi; ++e) {
      d += w64[e];
      w32[e] = (float)w64[e];
    }
  } else {
    d = (double)(hi - lo);
  }
  deg64[i] = d;
  deg32[i] = (float)d;
  const double inv = d > 0.0 ? 1.0 / d : 0.0;
  invd64[i] = inv;
  invd32[i] = (float)inv;
}

static void free_graph_arrays(DevGraph* g) {
  void* ptrs[] = {g->rp,     g->ci,     g->w64,  g->w32,      g->deg64,    g->deg32,
                  g->invd64, g->invd32, g->comp, g->comp_perm, g->comp_off, g->in_pos,
                  g->long_buf, g->lr.seg_part, g->lr.row_tick};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

nvd_status free_workspace(Workspace* ws) {
  if (!ws) return NVD_OK;
  void* ptrs[] = {ws->b64, ws->x64, ws->r64, ws->p64, ws->q64, ws->x32, ws->r32, ws->p32,
                  ws->q32, ws->comp_mean, ws->cs, ws->info, ws->red.part1, ws->red.part2,
                  ws->red.tick1, ws->red.tick2, ws->msync, ws->hq};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (ws->h_pinned) (void)hipHostFree(ws->h_pinned);
  delete ws;
  return NVD_OK;
}

// Vectors are n x tile, padded to a multiple of 16 elements so that the
// streaming kernels can use 16-byte accesses throughout.
static size_t padded(size_t n, int tile) { return ((n * (size_t)tile + 15) / 16) * 16; }

nvd_status ensure_workspace(DevGraph* g, int tile, bool need32) {
  Workspace* ws = g->ws;
  const size_t need = padded((size_t)g->n, tile);
  if (ws && ws->cap_rows >= need && (!need32 || ws->x32)) return NVD_OK;
  size_t cap = need;
  if (ws) {
    cap = std::max(cap, ws->cap_rows);
    need32 = need32 || ws->x32 != nullptr;
    g->bytes -= ws->bytes;
    free_workspace(ws);
    g->ws = nullptr;
  }
  ws = new Workspace();
  int64_t* by = &ws->bytes;
  nvd_status st = NVD_OK;
  auto chk = [&](nvd_status s) {
    if (st == NVD_OK) st = s;
  };
  chk(dalloc(&ws->b64, cap, by));
  chk(dalloc(&ws->x64, cap, by));
  chk(dalloc(&ws->r64, cap, by));
  chk(dalloc(&ws->p64, cap, by));
  chk(dalloc(&ws->q64, cap, by));
  if (need32) {
    chk(dalloc(&ws->x32, cap, by));
    chk(dalloc(&ws->r32, cap, by));
    chk(dalloc(&ws->p32, cap, by));
    chk(dalloc(&ws->q32, cap, by));
  }
  chk(dalloc(&ws->comp_mean, (size_t)std::max(g->n_comp, 1) * kMaxTile, by));
  chk(dalloc(&ws->cs, 1, by));
  chk(dalloc(&ws->info, kMaxTile, by));
  const size_t stride = kRedStride;
  chk(dalloc(&ws->red.part1, (size_t)kMaxBlocks * stride, by));
  chk(dalloc(&ws->red.part2, (size_t)(kMaxBlocks / kGrp) * stride, by));
  chk(dalloc(&ws->red.tick1, (size_t)(kMaxBlocks / kGrp), by));
  chk(dalloc(&ws->red.tick2, 1, by));
  chk(dalloc(&ws->msync, 64, by));
  if (st == NVD_OK) {
    hipError_t e = hipHostMalloc((void**)&ws->h_pinned, 64, hipHostMallocDefault);
    if (e != hipSuccess) {
      set_error(std::string("hipHostMalloc: ") + hipGetErrorString(e));
      st = NVD_E_NOMEM;
    }
  }
  if (st == NVD_OK) {
    // zero everything once: padding of vectors and the reduction counters
    // must start at zero
    double* v64[] = {ws->b64, ws->x64, ws->r64, ws->p64, ws->q64};
    for (double* p : v64) {
      if (hipMemset(p, 0, cap * sizeof(double)) != hipSuccess) st = NVD_E_DEVICE;
    }
    float* v32[] = {ws->x32, ws->r32, ws->p32, ws->q32};
    for (float* p : v32)
      if (p && hipMemset(p, 0, cap * sizeof(float)) != hipSuccess) st = NVD_E_DEVICE;
    if (hipMemset(ws->red.tick1, 0, (kMaxBlocks / kGrp) * sizeof(unsigned)) != hipSuccess ||
        hipMemset(ws->red.tick2, 0, sizeof(unsigned)) != hipSuccess ||
        hipMemset(ws->cs, 0, sizeof(ColState)) != hipSuccess)
      st = NVD_E_DEVICE;
    if (st == NVD_E_DEVICE) set_error("workspace initialisation failed");
  }
  if (st != NVD_OK) {
    free_workspace(ws);
    return st;
  }
  ws->cap_rows = cap;
  ws->cap_tile = tile;
  g->ws = ws;
  g->bytes += ws->bytes;
  return NVD_OK;
}

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------
// Host threads for the set-up passes (one for small graphs).
static int host_threads(size_t work) {
  if (work < ((size_t)1 << 18)) return 1;
  const unsigned hw = std::thread::hardware_concurrency();
  const int t = hw ? (int)hw : 4;
  return std::max(1, std::min(t, 16));
}

// f(lo, hi, tid) on nt contiguous row ranges of [0, n), in parallel.
template <class F>
static void parallel_rows(int n, int nt, F&& f) {
  if (nt <= 1 || n < 2 * nt) {
    f(0, n, 0);
    return;
  }
  std::vector<std::thread> th;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int lo = t * chunk, hi = std::min(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([&f, lo, hi, t]() { f(lo, hi, t); });
  }
  for (auto& x : th) x.join();
}

static nvd_status build_graph(int64_t n64, int64_t nnz64, const int64_t* row_ptr,
                              const int32_t* col_idx, const double* wts, hipStream_t stream,
                              DevGraph** out) {
  if (!out) {
    set_error("nvd_graph_create: out is NULL");
    return NVD_E_ARG;
  }
  *out = nullptr;
  if (n64 < 1 || nnz64 < 0) {
    set_error("nvd_graph_create: need n >= 1 and nnz >= 0");
    return NVD_E_ARG;
  }
  if (n64 >= INT32_MAX || nnz64 >= INT32_MAX) {
    set_error("nvd_graph_create: n and nnz must be below 2^31 (int32 indices)");
    return NVD_E_UNSUPPORTED;
  }
  if (!row_ptr || (nnz64 > 0 && !col_idx)) {
    set_error("nvd_graph_create: row_ptr/col_idx is NULL");
    return NVD_E_ARG;
  }
  const int n = (int)n64;
  const int nnz_in = (int)nnz64;
  if (row_ptr[0] != 0 || row_ptr[n] != nnz64) {
    set_error("nvd_graph_create: row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
    return NVD_E_GRAPH;
  }
  for (int i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) {
      set_error("nvd_graph_create: row_ptr not monotone at row " + std::to_string(i));
      return NVD_E_GRAPH;
    }
  }
  // drop self-loops, sort each row by column, check range / repeats /
  // weights, check symmetry, find the components: row ranges in parallel.
  // Errors name the lowest offending row, as a sequential scan would.
  const int nt = host_threads((size_t)nnz_in + (size_t)n);
  struct RowErr {
    int row = INT32_MAX;
    int kind = 0;        // 1 column range, 2 weight, 3 repeated entry, 4 no mirror, 5 weights differ
    int64_t e = 0;
    int a = 0, b = 0;
  };
  auto keep = [](RowErr& r, int row, int kind, int64_t e, int a, int b) {
    if (row < r.row) r = RowErr{row, kind, e, a, b};
  };
  auto report = [&](const RowErr& r) -> nvd_status {
    switch (r.kind) {
      case 1:
        set_error("nvd_graph_create: column " + std::to_string(r.a) + " out of range in row " +
                  std::to_string(r.row));
        break;
      case 2:
        set_error("nvd_graph_create: weight of entry " + std::to_string(r.e) +
                  " is not a finite positive number");
        break;
      case 3:
        set_error("nvd_graph_create: repeated entry (" + std::to_string(r.row) + ", " +
                  std::to_string(r.a) + ")");
        break;
      case 4:
        set_error("nvd_graph_create: entry (" + std::to_string(r.row) + ", " + std::to_string(r.a) +
                  ") has no mirror (" + std::to_string(r.a) + ", " + std::to_string(r.row) + ")");
        break;
      default:
        set_error("nvd_graph_create: weights of (" + std::to_string(r.row) + ", " +
                  std::to_string(r.a) + ") and its mirror differ");
        break;
    }
    return NVD_E_GRAPH;
  };
  // pass 1: entries kept per row, range and weight checks, sorted rows
  std::vector<int> rp(n + 1, 0);
  std::vector<char> sorted_row(n, 1);
  std::vector<RowErr> err1(nt);
  std::vector<int> loops_t(nt, 0);
  parallel_rows(n, nt, [&](int lo, int hi, int tid) {
    RowErr& er = err1[tid];
    int loops = 0;
    for (int i = lo; i < hi && i < er.row; ++i) {
      int kept = 0, prev = -1;
      bool srt = true;
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        const int c = col_idx[e];
        if (c < 0 || c >= n) {
          keep(er, i, 1, e, c, 0);
          break;
        }
        if (wts) {
          const double wv = wts[e];
          if (!(wv > 0.0) || !std::isfinite(wv)) {
            keep(er, i, 2, e, c, 0);
            break;
          }
        }
        if (c == i) {
          ++loops;
          continue;
        }
        if (c <= prev) srt = false;
        prev = c;
        ++kept;
      }
      rp[i + 1] = kept;
      sorted_row[i] = srt;
    }
    loops_t[tid] = loops;
  });
  RowErr first_err;
  for (const RowErr& r : err1)
    if (r.row < first_err.row) first_err = r;
  const int self_loops = std::accumulate(loops_t.begin(), loops_t.end(), 0);
  for (int i = 0; i < n; ++i) rp[i + 1] += rp[i];
  const int nnz = rp[n];
  // pass 2: kept entries in column order (rows before the first pass-1 error)
  std::vector<int> ci(nnz), in_pos(nnz);
  std::vector<double> w(wts ? nnz : 0);
  std::vector<RowErr> err2(nt);
  const int rows2 = first_err.row < n ? first_err.row : n;
  parallel_rows(rows2, nt, [&](int lo, int hi, int tid) {
    RowErr& er = err2[tid];
    std::vector<std::pair<int, int>> rowbuf;
    for (int i = lo; i < hi && i < er.row; ++i) {
      int o = rp[i];
      if (sorted_row[i]) {
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
          const int c = col_idx[e];
          if (c == i) continue;
          ci[o] = c;
          in_pos[o] = (int)e;
          if (wts) w[o] = wts[e];
          ++o;
        }
        continue;
      }
      rowbuf.clear();
      for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
        if (col_idx[e] != i) rowbuf.emplace_back(col_idx[e], (int)e);
      std::sort(rowbuf.begin(), rowbuf.end());
      for (size_t k = 0; k < rowbuf.size(); ++k) {
        if (k > 0 && rowbuf[k].first == rowbuf[k - 1].first) {
          keep(er, i, 3, 0, rowbuf[k].first, 0);
          break;
        }
        ci[o] = rowbuf[k].first;
        in_pos[o] = rowbuf[k].second;
        if (wts) w[o] = wts[rowbuf[k].second];
        ++o;
      }
    }
  });
  for (const RowErr& r : err2)
    if (r.row < first_err.row) first_err = r;
  if (first_err.row < n) return report(first_err);
  // pass 3: symmetry with equal weights: every (i, j) has a matching (j, i)
  std::vector<RowErr> err3(nt);
  parallel_rows(n, nt, [&](int lo, int hi, int tid) {
    RowErr& er = err3[tid];
    for (int i = lo; i < hi && i < er.row; ++i) {
      for (int e = rp[i]; e < rp[i + 1]; ++e) {
        const int j = ci[e];
        const int* b = ci.data() + rp[j];
        const int* en = ci.data() + rp[j + 1];
        const int* f = std::lower_bound(b, en, i);
        if (f == en || *f != i) {
          keep(er, i, 4, 0, j, 0);
          break;
        }
        if (wts && w[f - ci.data()] != w[e]) {
          keep(er, i, 5, 0, j, 0);
          break;
        }
      }
    }
  });
  for (const RowErr& r : err3)
    if (r.row < first_err.row) first_err = r;
  if (first_err.row < n) return report(first_err);
  // connected components: concurrent union-find that always hangs the larger
  // root under the smaller one, so every component's root is its smallest
  // node; components are numbered in order of that node
  std::vector<int> parent(n);
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int x) {
    for (;;) {
      const int p = __atomic_load_n(&parent[x], __ATOMIC_RELAXED);
      if (p == x) return x;
      const int gp = __atomic_load_n(&parent[p], __ATOMIC_RELAXED);
      if (gp != p) {
        int expect = p;
        __atomic_compare_exchange_n(&parent[x], &expect, gp, false, __ATOMIC_RELAXED, __ATOMIC_RELAXED);
      }
      x = p;
    }
  };
  parallel_rows(n, nt, [&](int lo, int hi, int) {
    for (int i = lo; i < hi; ++i) {
      for (int e = rp[i]; e < rp[i + 1]; ++e) {
        int u = i, v = ci[e];
        if (v < u) continue;     // each undirected edge once
        for (;;) {
          u = find(u);
          v = find(v);
          if (u == v) break;
          if (u < v) std::swap(u, v);   // u: the larger root
          int expect = u;
          if (__atomic_compare_exchange_n(&parent[u], &expect, v, false, __ATOMIC_ACQ_REL,
                                          __ATOMIC_RELAXED))
            break;
        }
      }
    }
  });
  std::vector<int> comp(n);
  parallel_rows(n, nt, [&](int lo, int hi, int) {
    for (int i = lo; i < hi; ++i) comp[i] = find(i);
  });
  int ncomp = 0, nisol = 0, maxdeg = 0;
  std::vector<int> comp_id(n, -1);
  for (int i = 0; i < n; ++i) {
    if (comp[i] == i) comp_id[i] = ncomp++;
    maxdeg = std::max(maxdeg, rp[i + 1] - rp[i]);
    if (rp[i + 1] == rp[i]) ++nisol;
  }
  std::vector<int> comp_off(ncomp + 1, 0);
  for (int i = 0; i < n; ++i) {
    comp[i] = comp_id[comp[i]];
    ++comp_off[comp[i] + 1];
  }
  for (int c = 0; c < ncomp; ++c) comp_off[c + 1] += comp_off[c];
  std::vector<int> perm(n), fill(comp_off.begin(), comp_off.end() - 1);
  for (int i = 0; i < n; ++i) perm[fill[comp[i]]++] = i;   // ascending ids within a component
  // split-row segments
  std::vector<int> seg_row, seg_lo, seg_hi, seg_first, seg_cnt;
  int nlong = 0;
  for (int i = 0; i < n; ++i) {
    const int d = rp[i + 1] - rp[i];
    if (d <= kLongRow) continue;
    ++nlong;
    const int cnt = (d + kSeg - 1) / kSeg;
    const int first = (int)seg_row.size();
    for (int k = 0; k < cnt; ++k) {
      seg_row.push_back(i);
      seg_lo.push_back(rp[i] + k * kSeg);
      seg_hi.push_back(std::min(rp[i] + (k + 1) * kSeg, rp[i + 1]));
      seg_first.push_back(first);
      seg_cnt.push_back(cnt);
    }
  }

  DevGraph* g = new DevGraph();
  g->n = n;
  g->nnz = nnz;
  g->nnz_in = nnz64;
  g->weighted = wts != nullptr;
  g->n_comp = ncomp;
  g->n_isolated = nisol;
  g->max_deg = maxdeg;
  g->self_loops = self_loops;
  g->n_long_rows = nlong;
  nvd_status st = NVD_OK;
  auto chk = [&](nvd_status s) {
    if (st == NVD_OK) st = s;
  };
  int64_t* by = &g->bytes;
  chk(dalloc(&g->rp, n + 1, by));
  chk(dalloc(&g->ci, nnz, by));
  if (wts) {
    chk(dalloc(&g->w64, nnz, by));
    chk(dalloc(&g->w32, nnz, by));
  }
  chk(dalloc(&g->deg64, n, by));
  chk(dalloc(&g->deg32, n, by));
  chk(dalloc(&g->invd64, n, by));
  chk(dalloc(&g->invd32, n, by));
  chk(dalloc(&g->comp, n, by));
  chk(dalloc(&g->comp_perm, n, by));
  chk(dalloc(&g->comp_off, ncomp + 1, by));
  // the map to input positions is needed whenever it is not the identity:
  // self-loops were dropped or some row was given unsorted
  const bool all_sorted = std::all_of(sorted_row.begin(), sorted_row.end(), [](char c) { return c != 0; });
  const bool need_pos = self_loops > 0 || !all_sorted;
  if (need_pos) chk(dalloc(&g->in_pos, nnz, by));
  const int nseg = (int)seg_row.size();
  if (nseg > 0) {
    chk(dalloc(&g->long_buf, (size_t)5 * nseg, by));
    chk(dalloc(&g->lr.seg_part, (size_t)nseg * kMaxTile, by));
    chk(dalloc(&g->lr.row_tick, (size_t)nseg, by));
  }
  auto up = [&](void* dst, const void* src, size_t bytes) {
    if (st != NVD_OK || bytes == 0) return;
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, stream);
    if (e != hipSuccess) {
      set_error(std::string("upload: ") + hipGetErrorString(e));
      st = NVD_E_DEVICE;
    }
  };
  up(g->rp, rp.data(), (n + 1) * sizeof(int));
  up(g->ci, ci.data(), nnz * sizeof(int));
  if (wts) up(g->w64, w.data(), nnz * sizeof(double));
  up(g->comp, comp.data(), n * sizeof(int));
  up(g->comp_perm, perm.data(), n * sizeof(int));
  up(g->comp_off, comp_off.data(), (ncomp + 1) * sizeof(int));
  if (need_pos) up(g->in_pos, in_pos.data(), nnz * sizeof(int));
  if (nseg > 0 && st == NVD_OK) {
    int* lb = g->long_buf;
    up(lb + 0 * nseg, seg_row.data(), nseg * sizeof(int));
    up(lb + 1 * nseg, seg_lo.data(), nseg * sizeof(int));
    up(lb + 2 * nseg, seg_hi.data(), nseg * sizeof(int));
    up(lb + 3 * nseg, seg_first.data(), nseg * sizeof(int));
    up(lb + 4 * nseg, seg_cnt.data(), nseg * sizeof(int));
    g->lr.n_seg = nseg;
    g->lr.seg_row = lb;
    g->lr.seg_lo = lb + nseg;
    g->lr.seg_hi = lb + 2 * nseg;
    g->lr.seg_first = lb + 3 * nseg;
    g->lr.seg_cnt = lb + 4 * nseg;
    if (st == NVD_OK && hipMemsetAsync(g->lr.row_tick, 0, nseg * sizeof(unsigned), stream) != hipSuccess)
      st = NVD_E_DEVICE;
  }
  if (st == NVD_OK) {
    k_degree<<<(n + 255) / 256, 256, 0, stream>>>(n, g->rp, g->w64, g->w32, g->deg64, g->deg32,
                                                  g->invd64, g->invd32);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) {
      set_error(std::string("graph setup: ") + hipGetErrorString(e));
      st = NVD_E_DEVICE;
    }
  }
  if (st != NVD_OK) {
    free_graph_arrays(g);
    delete g;
    return st;
  }
  g->h_rp = std::move(rp);
  g->h_ci = std::move(ci);
  g->h_comp = std::move(comp);
  g->h_w = std::move(w);
  *out = g;
  return NVD_OK;
}

nvd_status graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr, const int32_t* col_idx,
                        const double* w, hipStream_t s, DevGraph** out) {
  return build_graph(n, nnz, row_ptr, col_idx, w, s, out);
}

nvd_status graph_destroy(DevGraph* g) {
  if (!g) return NVD_OK;
  (void)hipDeviceSynchronize();
  if (g->ws) free_workspace(g->ws);
  free_tree(g->tree);
  free_achol(g->achol);
  free_slices(g);
  if (g->heavy) (void)hipFree(g->heavy);
  free_graph_arrays(g);
  delete g;
  return NVD_OK;
}

}  // namespace nvd
