// nvd_distances_noalloc: the distance solve of nvd_distances for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid allocation).  Every device buffer
// beyond the caller's inputs and outputs -- solver vectors, per-column
// state, reduction partials and counters, per-component means -- is carved
// from one file-scope device array of fixed size, `scratch`, which each GPU
// holds for the life of the process.  The kernels are those of
// nvd_distances; they take the carved pointers as they take the handle's
// cached workspace.
//
// The host never names `scratch` directly when it needs its memory: the
// name is a host-side stand-in, not a device address.  Once per device,
// with that device current, hipGetSymbolAddress gives the device address,
// which is kept per device and used for every kernel argument.
//
// Every call on one GPU shares that GPU's array and leaves its contents
// behind: the call clears what must start at zero (reduction counters,
// column state, vector padding) with a fill kernel, and two calls that
// overlap on one GPU (different streams, or threads) race on it.
#include <mutex>

#include "device_common.hpp"

namespace nvd {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;   // 64 MiB per GPU
constexpr int kNoAllocShortGrid = 1024;             // SpMM short-row blocks
// the largest grid of a reducing kernel in this mode: long-row blocks (at
// most 1024) plus the short-row blocks; the vector kernels use fewer
constexpr int kNoAllocRedBlocks = 1024 + kNoAllocShortGrid;

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char* g_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (looked up once per device).
nvd_status scratch_ptr(unsigned char** out) {
  int dev = 0;
  NVD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("nvd_distances_noalloc: device index beyond the library's table");
    return NVD_E_UNSUPPORTED;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("nvd_distances_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return NVD_E_DEVICE;
    }
    g_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_ptr[dev];
  return NVD_OK;
}

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// Host words the solver polls (pageable: the copies are followed by a stream
// synchronisation anyway).
thread_local int g_poll_words[16];

struct Carve {
  size_t off = 0;
  unsigned char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + off);
    off += up256(count * sizeof(T));
    return p;
  }
};
}  // namespace

// Zero a few byte ranges of the scratch array (counters, column state and
// the padding of every vector past n*T): each (dst, bytes) range is a
// multiple of 4 bytes.
struct ZeroList {
  unsigned* dst[12];
  int words[12];
  int count;
};

__global__ void k_zero_ranges(ZeroList z) {
  for (int r = 0; r < z.count; ++r)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < z.words[r]; i += gridDim.x * blockDim.x)
      z.dst[r][i] = 0u;
}

}  // namespace nvd

using namespace nvd;

extern "C" nvd_status nvd_distances_noalloc(nvd_graph* h, int32_t k, const double* P,
                                            const double* Q, int64_t ld, const nvd_opts* opts,
                                            double* d_out, double* X, int64_t ldx,
                                            nvd_pair_info* info, void* stream) {
  set_error("");
  if (!h || !P || !Q || !d_out || k < 1 || ld < k || (X && ldx < k)) {
    set_error("nvd_distances_noalloc: bad argument (NULL pointer, k < 1 or ld < k)");
    return NVD_E_ARG;
  }
  nvd_opts o;
  nvd_opts_default(&o);
  if (opts) o = *opts;
  NVD_TRY(check_solve_opts(&o));
  if ((o.flags & NVD_WARM_START) && !X) {
    set_error("nvd_distances_noalloc: NVD_WARM_START needs X_inout");
    return NVD_E_ARG;
  }
  if (o.flags & (NVD_PRECOND_TREE | NVD_PRECOND_AUTO | NVD_PRECOND_ACHOL | NVD_BATCH_PERSISTENT)) {
    set_error("nvd_distances_noalloc: only the Jacobi preconditioner (the spanning forest and "
              "the approximate-Cholesky factor allocate their data on first use)");
    return NVD_E_UNSUPPORTED;
  }
  DevGraph* g = h->g;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  const bool mixed = o.precision == NVD_MIXED;
  const int tile = o.tile_k ? o.tile_k : untimed_tile(g, k, o.precision);
  int T0 = tile;
  while (T0 > k) T0 >>= 1;   // the widest tile any pass of this call uses
  // layout for the widest tile: the narrower tail tiles fit in it
  const size_t cap = ((size_t)g->n * T0 + 15) / 16 * 16;
  const size_t red_stride = kRedStride;
  size_t need = 0;
  need += up256(sizeof(unsigned) * (kMaxBlocks / kGrp)) + up256(sizeof(unsigned));   // counters
  need += up256(sizeof(ColState)) + up256(sizeof(nvd_pair_info) * kMaxTile);
  need += up256(sizeof(double) * kNoAllocRedBlocks * red_stride);
  need += up256(sizeof(double) * (kNoAllocRedBlocks / kGrp + 1) * red_stride);
  need += g->n_comp > 1 ? up256(sizeof(double) * (size_t)g->n_comp * kMaxTile) : 0;
  need += 5 * up256(sizeof(double) * cap);
  if (mixed) need += 4 * up256(sizeof(float) * cap);
  if (need > kNoAllocBytes) {
    set_error("nvd_distances_noalloc: the solve needs " + std::to_string(need >> 20) +
              " MiB of scratch for n = " + std::to_string(g->n) + " and tile " +
              std::to_string(T0) + "; the limit is " + std::to_string(kNoAllocBytes >> 20) +
              " MiB (use nvd_distances, or fewer pairs per call)");
    return NVD_E_UNSUPPORTED;
  }
  unsigned char* base = nullptr;
  NVD_TRY(scratch_ptr(&base));
  Carve cv;
  cv.base = base;
  Workspace ws;
  ws.red.tick1 = cv.take<unsigned>(kMaxBlocks / kGrp);
  ws.red.tick2 = cv.take<unsigned>(1);
  ws.cs = cv.take<ColState>(1);
  ws.info = cv.take<nvd_pair_info>(kMaxTile);
  ws.red.part1 = cv.take<double>((size_t)kNoAllocRedBlocks * red_stride);
  ws.red.part2 = cv.take<double>((size_t)(kNoAllocRedBlocks / kGrp + 1) * red_stride);
  ws.comp_mean = g->n_comp > 1 ? cv.take<double>((size_t)g->n_comp * kMaxTile) : nullptr;
  ws.b64 = cv.take<double>(cap);
  ws.x64 = cv.take<double>(cap);
  ws.r64 = cv.take<double>(cap);
  ws.p64 = cv.take<double>(cap);
  ws.q64 = cv.take<double>(cap);
  if (mixed) {
    ws.x32 = cv.take<float>(cap);
    ws.r32 = cv.take<float>(cap);
    ws.p32 = cv.take<float>(cap);
    ws.q32 = cv.take<float>(cap);
  }
  ws.cap_rows = cap;
  ws.cap_tile = T0;
  ws.h_pinned = g_poll_words;

  SolveParams sp{};
  sp.precision = o.precision;
  sp.rtol = o.rtol;
  sp.inner_rtol = o.inner_rtol;
  sp.max_iter = o.max_iter;
  sp.max_refine = o.max_refine;
  sp.warm = (o.flags & NVD_WARM_START) != 0;
  sp.tree = false;
  sp.achol = false;
  sp.out_dsq = (o.flags & NVD_OUT_DSQ) != 0;
  sp.grid = kNoAllocShortGrid;
  nvd_status agg = NVD_OK;
  for (int c0 = 0; c0 < k;) {
    int T = tile;
    while (T > k - c0) T >>= 1;
    sp.nl = tuned_nl(g, o.precision, T);
    // clear what must start at zero: counters, column state and the padding
    // of every vector past n*T (a previous call may have used another layout)
    const size_t nT = (size_t)g->n * T;
    const size_t capT = (nT + 15) / 16 * 16;
    ZeroList z{};
    auto add = [&](void* p, size_t bytes) {
      z.dst[z.count] = static_cast<unsigned*>(p);
      z.words[z.count] = (int)(bytes / 4);
      ++z.count;
    };
    add(ws.red.tick1, sizeof(unsigned) * (kMaxBlocks / kGrp));
    add(ws.red.tick2, sizeof(unsigned));
    add(ws.cs, sizeof(ColState));
    double* v64[5] = {ws.b64, ws.x64, ws.r64, ws.p64, ws.q64};
    for (double* v : v64) add(v + nT, sizeof(double) * (capT - nT));
    if (mixed) {
      float* v32[4] = {ws.x32, ws.r32, ws.p32, ws.q32};
      for (float* v : v32) add(v + nT, sizeof(float) * (capT - nT));
    }
    k_zero_ranges<<<64, 256, 0, s>>>(z);
    NVD_HIP(hipGetLastError());
    NVD_TRY(solve_tile_ws(g, &ws, T, P + c0, Q + c0, ld, sp, d_out + c0, X ? X + c0 : nullptr, ldx,
                          ws.info, s));
    nvd_pair_info tile_info[kMaxTile];
    NVD_HIP(hipMemcpyAsync(tile_info, ws.info, sizeof(nvd_pair_info) * T, hipMemcpyDeviceToHost, s));
    NVD_HIP(hipStreamSynchronize(s));
    for (int j = 0; j < T; ++j) {
      if (tile_info[j].status == NVD_E_BREAKDOWN) agg = NVD_E_BREAKDOWN;
      else if (tile_info[j].status == NVD_E_NOCONV && agg == NVD_OK) agg = NVD_E_NOCONV;
      if (info) info[c0 + j] = tile_info[j];
    }
    c0 += T;
  }
  if (agg != NVD_OK) set_error("nvd_distances_noalloc: some pairs did not converge (see info)");
  return agg;
}
