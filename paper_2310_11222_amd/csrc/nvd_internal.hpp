// Internal declarations shared by the library's translation units: the
// graph handle, workspace, preconditioner state, entry points and error
// plumbing (host side); the device-side types are in device_types.hpp.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nvd.h"
#include "device_types.hpp"

namespace nvd {

// ---------------------------------------------------------------------------
// host-side handles
// ---------------------------------------------------------------------------
struct Workspace;

// Spanning forest for the tree preconditioner (built on first use): Euler
// tour positions, inverse edge weights to the parent, and scan buffers.
struct TreePre {
  int* tin = nullptr;          // [n] tour position where v is entered (0 .. 2n-1)
  int* tout = nullptr;         // [n] tour position where v is left
  double* winv = nullptr;      // [n] 1 / weight of the edge to the parent (0 at roots)
  int* rbeg = nullptr;         // [n] tin of v's root: v's component is the tour
  int* rend = nullptr;         // [n] range [rbeg, rend] (tout of the root)
  int* tnode = nullptr;        // [2n] node entered at each tour position, -1 where one is left
  double* E = nullptr;         // [2n][cap_tile] tour values
  double* S = nullptr;         // [2n][cap_tile] their prefix sums
  double* part = nullptr;      // [chunks][cap_tile] scan offsets
  int cap_tile = 0;
  int n_tree_edges = 0;
  // augmentation: k off-forest edges solved exactly with the forest
  // (Woodbury: M^+ = L_T^+ - Y C^-1 Y^T, Y = L_T^+ U, C = W^-1 + U^T Y)
  int k_aug = 0;
  std::vector<int> aug_u, aug_v;  // host: the edges' ends
  std::vector<double> aug_w;      // host: their weights
  int* aug_uv = nullptr;          // [2k] u then v
  double* aug_Y = nullptr;        // [n][k] L_T^+ U (built with the first tile)
  double* aug_Cinv = nullptr;     // [k][k] C^-1
  double* aug_st = nullptr;       // [2][k][kMaxTile] U^T z, then C^-1 U^T z
};

// Approximate-Cholesky factor for its preconditioner (built on first use):
// vertices by elimination position, the factor's columns (pull lists for the
// backward solve) and their transpose (pull lists for the forward solve),
// 1 / pivot by position, and scratch for the component means of r.
struct AcholPre {
  int* order = nullptr;        // [n] vertex at each position (rounds, then remainder)
  int* out_off = nullptr;      // [n+1] by position
  int* out_idx = nullptr;      // [nnz] later vertex
  double* out_c64 = nullptr;   // [nnz] coefficient w / W
  float* out_c32 = nullptr;
  int* in_off = nullptr;       // [n+1] by position
  int* in_idx = nullptr;       // [nnz] earlier vertex
  double* in_c64 = nullptr;
  float* in_c32 = nullptr;
  double* ip64 = nullptr;      // [n] by position: 1 / pivot (0: ground)
  float* ip32 = nullptr;
  double* mean = nullptr;      // [n_comp][kMaxTile]
  double* part = nullptr;      // [blocks][kMaxTile]
  std::vector<int> round_off;  // host: positions of each round, last range = remainder
  std::vector<int> fwd_max;    // host: longest forward pull list of each round
  std::vector<int> bwd_max;    // host: longest backward pull list of each round
  int rounds = 0;
  int grounds = 0;
  int remainder = 0;
  int64_t nnz = 0;
  int64_t bytes = 0;
};

struct SliceGraph;   // column slices of the one-column apply (slice.hip)

struct DevGraph {
  int n = 0;
  int nnz = 0;                 // internal nnz (self-loops removed)
  int64_t nnz_in = 0;          // nnz as passed in
  bool weighted = false;
  int n_comp = 0;
  int n_isolated = 0;
  int max_deg = 0;
  int self_loops = 0;
  // device arrays
  int* rp = nullptr;           // [n+1]
  int* ci = nullptr;           // [nnz]
  double* w64 = nullptr;       // [nnz] or null (unit)
  float* w32 = nullptr;
  double* deg64 = nullptr;     // [n]
  float* deg32 = nullptr;
  double* invd64 = nullptr;    // [n], 0 for isolated nodes
  float* invd32 = nullptr;
  int* comp = nullptr;         // [n] component label
  int* comp_perm = nullptr;    // nodes grouped by component
  int* comp_off = nullptr;     // [n_comp+1]
  int* in_pos = nullptr;       // [nnz] input position of each internal entry (null if identity)
  int* long_buf = nullptr;     // segment arrays
  LongRows lr;
  int n_long_rows = 0;
  // host copies kept for queries and batching
  std::vector<int> h_rp, h_ci, h_comp;
  std::vector<double> h_w;     // empty if unit
  int64_t bytes = 0;
  Workspace* ws = nullptr;
  int tuned_tile[2][8] = {};   // [precision][log2 k bucket] -> tile (0 = not tuned)
  int tuned_nl[2][8] = {};     // [precision][log2 tile] -> neighbour lanes (0 = default)
  TreePre* tree = nullptr;     // spanning forest, built when first needed
  AcholPre* achol = nullptr;   // approximate-Cholesky factor, built when first needed
  int* heavy = nullptr;        // rows walked by a whole wave in the single-launch solve
  int n_heavy = -1;            // (built when first needed, longest first; -1: not yet)
  int heavy_base = 0;          // degree threshold the list was built for
  std::vector<int> heavy_deg_desc;  // host: their degrees
  SliceGraph* slices = nullptr; // built when the sliced apply is first needed
  int slice_state = 0;          // -1: build failed, use the row-wise apply
  int slice_pick[2] = {0, 0};   // [FP64, FP32]: 1 sliced, -1 row-wise (timed), 0 not yet
};

struct Workspace {
  size_t cap_rows = 0;         // rows * tile capacity (elements per vector)
  int cap_tile = 0;
  // FP64 vectors (n x tile)
  double* b64 = nullptr;       // delta_bar
  double* x64 = nullptr;
  double* r64 = nullptr;
  double* p64 = nullptr;
  double* q64 = nullptr;
  // FP32 vectors for the inner solver
  float* x32 = nullptr;
  float* r32 = nullptr;
  float* p32 = nullptr;
  float* q32 = nullptr;
  double* comp_mean = nullptr; // [n_comp][kMaxTile]
  ColState* cs = nullptr;
  nvd_pair_info* info = nullptr;  // [kMaxTile] per-pair results of one tile
  GridRed red{};
  unsigned* msync = nullptr;   // [2] grid barrier of the multi-block small solve
  double* hq = nullptr;        // n x tile: q of heavy rows in the single-launch solve (lazy)
  int* h_pinned = nullptr;     // pinned host words for polling
  int64_t bytes = 0;
};

// ---------------------------------------------------------------------------
// error plumbing (host)
// ---------------------------------------------------------------------------
void set_error(const std::string& msg);
const char* get_error();

#define NVD_HIP(call)                                                     \
  do {                                                                    \
    hipError_t e_ = (call);                                               \
    if (e_ != hipSuccess) {                                               \
      ::nvd::set_error(std::string(#call) + ": " + hipGetErrorString(e_)); \
      return e_ == hipErrorOutOfMemory ? NVD_E_NOMEM : NVD_E_DEVICE;     \
    }                                                                     \
  } while (0)

#define NVD_TRY(expr)                  \
  do {                                 \
    nvd_status s_ = (expr);            \
    if (s_ != NVD_OK) return s_;       \
  } while (0)

// workspace management (graph.hip)
nvd_status ensure_workspace(DevGraph* g, int tile, bool need32);
nvd_status free_workspace(Workspace* ws);

// kernels' host launchers (spmm.hip, cg.hip)
enum Epi { EPI_PLAIN = 0, EPI_CG = 1, EPI_RESID = 2 };

struct SpmmCall {
  const DevGraph* g;
  int prec;                 // 0: FP64 weights/vectors, 1: FP32
  int T;                    // columns
  int nl;                   // lanes per row across neighbours (0 = auto)
  const void* x; int64_t ldx;
  void* y; int64_t ldy;
  const double* b; int64_t ldb;   // EPI_RESID right-hand side
  ColState* cs;
  int epi;
  int grid;                 // short-row blocks (0 = auto)
};
nvd_status launch_spmm(const SpmmCall& c, const GridRed& red, hipStream_t s);
// The apply the solvers and nvd_laplacian_apply use: one column (T = 1) on a
// large graph by XCD-pinned column slices (slice.hip), else launch_spmm.
nvd_status launch_apply(const SpmmCall& c, const GridRed& red, hipStream_t s);
void free_slices(DevGraph* g);

struct SolveParams {
  int precision;            // NVD_FP64 or NVD_MIXED
  double rtol, inner_rtol;
  int max_iter, max_refine;
  int nl;                   // SpMM lanes per row across neighbours (0 = default)
  int grid;                 // SpMM short-row grid (0 = default)
  bool warm;
  bool tree;                // an explicit preconditioner solve z = M^-1 r instead of
                            // Jacobi: the spanning forest, or (achol) the factor
  bool achol;               // the approximate-Cholesky factor
  bool out_dsq;             // d_out receives d^2 instead of d
};
nvd_status solve_tile(DevGraph* g, int T, const double* P, const double* Q, int64_t ld,
                      const SolveParams& sp, double* d_out, double* X, int64_t ldx,
                      nvd_pair_info* info_dev, hipStream_t s);
nvd_status solve_tile_ws(DevGraph* g, Workspace* ws, int T, const double* P, const double* Q,
                         int64_t ld, const SolveParams& sp, double* d_out, double* X,
                         int64_t ldx, nvd_pair_info* info_dev, hipStream_t s);
// One launch per tile for small and mid-size connected graphs (small.hip):
// small_blocks gives the launch's block count (1: one block; more: a
// cooperative launch with grid barriers) or 0 where the multi-kernel path
// runs.  NVD_SMALL=0 in the environment turns the path off.
int small_blocks(DevGraph* g, int T, const SolveParams& sp);
nvd_status solve_small(DevGraph* g, int T, int nb, const double* P, const double* Q, int64_t ld,
                       const SolveParams& sp, double* d_out, double* X, int64_t ldx,
                       nvd_pair_info* info_dev, hipStream_t s);
// Tile for k pairs without timing anything: the autotuner's cached choice,
// else the fixed heuristic.
int untimed_tile(const DevGraph* g, int k, int precision);
nvd_status project_tile(DevGraph* g, int T, const double* P, const double* Q, int64_t ld,
                        double* Dbar, int64_t ldd, double* norms, hipStream_t s);
// Tree preconditioner (tree.hip): set up for tiles up to T; z = L_T^+ r.
// NVD_PRECOND_TREE, or NVD_PRECOND_AUTO on a graph with few edges off its
// spanning forest.
bool use_tree(const DevGraph* g, uint32_t flags);
nvd_status ensure_tree(DevGraph* g, int T);
nvd_status tree_solve(DevGraph* g, int prec, int T, const void* r, void* z, hipStream_t s);
void free_tree(TreePre* tp);
// Approximate-Cholesky preconditioner (achol.hip): NVD_PRECOND_ACHOL.
nvd_status ensure_achol(DevGraph* g);
nvd_status achol_solve(DevGraph* g, int prec, int T, const void* r, void* z, hipStream_t s);
void free_achol(AcholPre* ap);

// Validation of solver options (NVD_E_ARG with a message).
nvd_status check_solve_opts(const nvd_opts* o);
int choose_tile(DevGraph* g, int k, int precision, hipStream_t s);
// One CG iteration (apply + update + direction) on the workspace vectors, timed.
nvd_status time_cg_iteration(DevGraph* g, int prec, int T, int nl, hipStream_t s, float* ms);
int tuned_nl(const DevGraph* g, int precision, int T);
int default_nl(int T);
// Largest neighbour sub-group count the apply supports for (precision, T).
int spmm_max_nl(int prec, int T);
int default_short_grid(int n, int T, int nl);

}  // namespace nvd

// The opaque handle behind nvd_graph*.
struct nvd_graph {
  nvd::DevGraph* g;
};
