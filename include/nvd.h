/*
 * nvd.h -- C ABI of the MI355X (gfx950) node-vector-distance library.
 *
 * The library computes the Generalized Euclidean (GE) distance between node
 * vectors a, b on an undirected graph G with positive edge weights
 * (Coscia & Devriendt, "Fast Node Vector Distance Computations using
 * Laplacian Solvers", section 3.1):
 *
 *     d(a, b) = sqrt( (a - b)^T L^+ (a - b) ),   L = D - A,
 *
 * where A holds the edge weights, D the weighted degrees and L^+ is the
 * Moore-Penrose pseudoinverse.  As in the paper's section 3.2, L^+ is never
 * formed: L x = delta_bar is solved with a Laplacian solver (here
 * Jacobi-preconditioned conjugate gradients on the GPU), where delta_bar is
 * delta = a - b with its mean removed on every connected component, and
 *
 *     d^2 = delta_bar^T x + x^T r,   r = delta_bar - L x,
 *
 * evaluated in FP64 (equal to delta_bar^T x for an exact or Galerkin x; the
 * x^T r term makes the error quadratic in the residual after refinement).
 *
 * Conventions (the paper fixes only the unit-weight case):
 *   - weights are conductances: L_ii = sum_j w_ij, L_ij = -w_ij;
 *   - self-loops are dropped on input (they cancel in D - A);
 *   - an isolated node is its own component and contributes nothing;
 *   - delta_bar = 0 gives d = 0 exactly, with no iterations.
 *
 * Layouts.  A graph is a symmetric CSR (host arrays, or device arrays with
 * nvd_graph_create_ex and NVD_PTR_DEVICE): row_ptr int64 [n+1],
 * col_idx int32 [nnz] (both directions of every edge present, equal weights,
 * no repeated (i, j) within a row), weights float64 [nnz] or NULL for unit
 * weights.  Node-vector blocks are row-major n x k float64 with a leading
 * dimension ld >= k (element (i, j) at P[i*ld + j]), column j being pair j.
 *
 * Ownership.  A graph or batch handle owns device copies of everything it
 * needs, plus its solver workspace (allocated on first use and cached); the
 * caller's input arrays may be freed after the create call returns.  Buffers
 * passed to solve calls stay owned by the caller.  A handle is not
 * thread-safe: one call in flight per handle.
 *
 * Streams.  Every `stream` argument is a hipStream_t passed as void*
 * (NULL = the default stream).  Solve calls (nvd_distances, nvd_pairwise,
 * nvd_batch_distances, nvd_graph_set_weights) enqueue their work on that
 * stream and return after it has completed, so outputs are ready on return:
 * the iteration count is data dependent, and the host reads a few words of
 * convergence state (a 24-byte copy and a stream synchronisation, ~10-20 us)
 * after each chunk of CG iterations.  The chunk is sized from the observed
 * decay of the worst residual, so a solve of I iterations polls about
 * 3 + I / 8 times.  nvd_laplacian_apply, nvd_project and the adjoint calls
 * only enqueue.
 *
 * Errors.  Every call returns an nvd_status.  Argument and graph errors are
 * found before anything is enqueued; nvd_last_error() then holds a message
 * (thread-local, valid until the next call on the same thread).  HIP failures
 * return NVD_E_DEVICE.  Per-pair numerical outcomes (no convergence,
 * breakdown) are reported in nvd_pair_info and, aggregated, in the return
 * value as NVD_E_NOCONV / NVD_E_BREAKDOWN while every output is still
 * written.  Nothing is printed and no call aborts the process.
 */
#ifndef NVD_H
#define NVD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define NVD_ABI_VERSION 1

typedef enum nvd_status {
  NVD_OK = 0,
  NVD_E_ARG = 1,         /* bad argument (NULL pointer, k < 1, ld < k, ...) */
  NVD_E_GRAPH = 2,       /* invalid CSR: not monotone, column out of range,
                            asymmetric, repeated entry, bad weight */
  NVD_E_VALUE = 3,       /* non-finite value in a node vector */
  NVD_E_NOCONV = 4,      /* at least one pair hit max_iter / max_refine */
  NVD_E_BREAKDOWN = 5,   /* at least one pair lost positivity (p^T L p <= 0) */
  NVD_E_DEVICE = 6,      /* a HIP call failed */
  NVD_E_NOMEM = 7,       /* device allocation failed */
  NVD_E_UNSUPPORTED = 8  /* valid request beyond the library's limits */
} nvd_status;

/* nvd_opts.precision */
enum { NVD_FP64 = 0, NVD_MIXED = 1 };
/* dtype of nvd_laplacian_apply */
enum { NVD_DT_F64 = 0, NVD_DT_F32 = 1 };
/* nvd_opts.flags */
enum {
  NVD_WARM_START = 1u,      /* X_inout holds a starting guess on entry */
  NVD_BATCH_PERSISTENT = 2u,/* nvd_batch_distances: the single persistent
                               launch instead of the sweep solver */
  NVD_PRECOND_TREE = 4u,    /* nvd_distances / nvd_pairwise: precondition CG
                               with an augmented spanning forest (Table 1's
                               "Aug Tree"): a breadth-first or maximum-weight
                               forest, whichever has the smaller stretch,
                               plus up to 256 off-forest edges of largest
                               stretch, solved exactly (forest solve and a
                               rank-k correction); instead of the Jacobi
                               diagonal, for sparse graphs, above all with
                               heavy-tailed weights.  Not for batches. */
  NVD_PRECOND_AUTO = 8u,    /* nvd_distances / nvd_pairwise: the spanning
                               forest when at most n/100 edges lie off it
                               (m - n + c <= n / 100 for m edges and c
                               components: tree PCG then needs at most that
                               many iterations plus one in exact arithmetic)
                               or when the augmentation takes all of them,
                               else the Jacobi diagonal.  Batches always use
                               the Jacobi diagonal under this flag. */
  NVD_OUT_DSQ = 16u,        /* nvd_distances: d_out receives d^2 (the
                               quadratic form, clamped at 0) instead of d */
  NVD_PRECOND_ACHOL = 32u   /* nvd_distances / nvd_pairwise: precondition CG
                               with an approximate Cholesky factor of L
                               (section 3.2: sparse approximate Gaussian
                               elimination, cliques replaced by sampled
                               edges; the solver of Table 2), built on the
                               host on first use and applied as two
                               triangular solves of one GPU step per
                               elimination round.  Excludes NVD_PRECOND_TREE
                               and NVD_PRECOND_AUTO.  Not for batches. */
};
/* nvd_pair_info.flags */
enum { NVD_INFO_FP64_FALLBACK = 1 };
/* nvd_graph_create_ex flags: where the CSR arrays live */
enum { NVD_PTR_HOST = 0u, NVD_PTR_DEVICE = 1u };

typedef struct nvd_graph nvd_graph;
typedef struct nvd_batch nvd_batch;

typedef struct nvd_opts {
  int32_t precision;   /* NVD_FP64: all CG arithmetic in FP64.  NVD_MIXED:
                          inner CG in FP32, outer residual delta_bar - L x,
                          its norm and the update of x in FP64 (iterative
                          refinement). */
  double rtol;         /* stop when ||delta_bar - L x|| <= rtol ||delta_bar||
                          (relative 2-norm per pair; default 1e-10) */
  double inner_rtol;   /* MIXED: relative residual of each inner FP32 solve
                          (default 1e-5) */
  int32_t max_iter;    /* CG iterations per pair (FP64) or per inner solve
                          (MIXED); default 20000 */
  int32_t max_refine;  /* MIXED: outer refinement steps; default 30 */
  int32_t tile_k;      /* columns per SpMM pass: 1,2,4,8,16,32,64; 0 = the
                          library's autotuned choice */
  uint32_t flags;      /* NVD_WARM_START, NVD_BATCH_PERSISTENT, NVD_PRECOND_TREE,
                          NVD_PRECOND_AUTO, NVD_OUT_DSQ, NVD_PRECOND_ACHOL */
} nvd_opts;

typedef struct nvd_pair_info {
  int32_t status;       /* NVD_OK, NVD_E_NOCONV or NVD_E_BREAKDOWN
                           (NVD_E_DEVICE: a persistent launch -- the batch's,
                           or the single-launch solve of a small graph -- gave
                           up at a barrier; its outputs are then meaningless) */
  int32_t iters;        /* CG iterations (all inner solves summed) */
  int32_t refine_steps; /* MIXED outer steps (0 for FP64) */
  int32_t flags;        /* NVD_INFO_FP64_FALLBACK: the mixed solve stalled
                           (FP32 could not reduce the FP64 residual by 2x in
                           two consecutive outer steps) and the pair was
                           finished by the FP64 solver from its current x */
  double rel_res;       /* final true ||delta_bar - L x|| / ||delta_bar|| */
  double dsq_plain;     /* delta_bar^T x */
  double dsq;           /* delta_bar^T x + x^T r (returned d = sqrt(max(dsq,0))) */
} nvd_pair_info;

typedef struct nvd_stats {
  int64_t n;            /* nodes */
  int64_t nnz;          /* stored off-diagonal entries (2 |E|) */
  int64_t n_comp;       /* connected components (isolated nodes included) */
  int64_t n_isolated;   /* nodes of degree 0 */
  int64_t max_deg;      /* largest number of neighbours */
  int64_t n_long_rows;  /* rows handled by the split-row path of the SpMM */
  int64_t device_bytes; /* device memory held by the handle (workspace incl.) */
  int32_t weighted;     /* 1 if explicit weights were given */
  int32_t self_loops_dropped; /* number of diagonal entries removed on input */
  int64_t achol_rounds; /* approximate-Cholesky factor (0s until built):
                           elimination rounds = steps of each triangular
                           solve */
  int64_t achol_factor_nnz;  /* off-diagonal entries of the factor */
  int64_t achol_remainder;   /* vertices left to the Schur diagonal after
                                the last round */
} nvd_stats;

/* ---- library ----------------------------------------------------------- */
int32_t nvd_abi_version(void);
const char* nvd_status_string(int32_t status);
/* Message of the last failing call on this thread ("" if none). */
const char* nvd_last_error(void);
/* Fills *o with the defaults listed in nvd_opts. */
nvd_status nvd_opts_default(nvd_opts* o);

/* ---- graph (operator setup; the paper excludes this preprocessing from its
 *      timings, section 5.2) ------------------------------------------------
 * Validates the host CSR (see Layouts), drops self-loops, uploads it,
 * computes weighted degrees and their inverses (0 for isolated nodes),
 * FP32 copies, connected-component labels (for the per-component mean
 * removal) and the list of long rows for the SpMM's split-row path.
 * Limits: n < 2^31, nnz < 2^31 (NVD_E_UNSUPPORTED otherwise). */
nvd_status nvd_graph_create(int64_t n, int64_t nnz, const int64_t* row_ptr,
                            const int32_t* col_idx, const double* weights,
                            void* stream, nvd_graph** out);
/* As nvd_graph_create; flags NVD_PTR_DEVICE: row_ptr, col_idx and weights
 * are device pointers (same layouts).  They are read after the work already
 * on `stream` has completed and copied to the host, where validation runs;
 * the caller keeps ownership.  Unknown flags: NVD_E_ARG. */
nvd_status nvd_graph_create_ex(int64_t n, int64_t nnz, const int64_t* row_ptr,
                               const int32_t* col_idx, const double* weights,
                               uint32_t flags, void* stream, nvd_graph** out);
nvd_status nvd_graph_destroy(nvd_graph* g);
nvd_status nvd_graph_stats(const nvd_graph* g, nvd_stats* s);
/* Host copies of the component label of every node (int32 [n], labels
 * 0..n_comp-1 numbered by each component's smallest node) and of the
 * weighted degree (float64 [n]).  Either pointer may be NULL. */
nvd_status nvd_graph_query(const nvd_graph* g, int32_t* labels_host,
                           double* degree_host);

/* ---- Laplacian apply: Y = L X (section 3.1's L = D - A) ----------------
 * X, Y: device, row-major n x k with leading dimensions ldx, ldy, element
 * type float64 (dtype NVD_DT_F64, FP64 weights) or float32 (NVD_DT_F32, the
 * graph's FP32 weight copy).  X and Y must not overlap.  Asynchronous:
 * returns once enqueued.
 * One column (k = 1, here and in the solvers' tiles of one pair) on a graph
 * of at least 2^20 nodes may be applied by column slices: the nodes are cut
 * into slices whose part of X fits one XCD's L2, each XCD gathers from its
 * own slice, and per-row partial sums are added slice by slice in a fixed
 * order.  The first such call of each precision builds the slice structure
 * on the host, times both forms of the apply on its X and keeps the faster
 * for the graph (that call waits for the device and then enqueues).  The
 * structure is kept with the graph while one precision uses it (device
 * memory: about 4 bytes per CSR entry, plus 11 bytes per row and slice with
 * neighbours there; weighted graphs 12 more per entry and 8 per row) and
 * dropped by nvd_graph_set_weights and nvd_graph_destroy.  nvd_distances_noalloc never
 * uses it.  Environment: NVD_SLICE=0 never uses it, NVD_SLICE=1 uses it at
 * any size without timing. */
nvd_status nvd_laplacian_apply(nvd_graph* g, int32_t dtype, int32_t k,
                               const void* X, int64_t ldx, void* Y,
                               int64_t ldy, void* stream);

/* ---- projection: delta_bar = (P - Q) minus its mean on every component --
 * P, Q: device float64 n x k (ld); Dbar: device float64 n x k (ldd);
 * norms: device float64 [k] receives ||delta_bar_j||_2 (may be NULL).
 * Asynchronous. */
nvd_status nvd_project(nvd_graph* g, int32_t k, const double* P,
                       const double* Q, int64_t ld, double* Dbar, int64_t ldd,
                       double* norms, void* stream);

/* ---- distances (the paper's GE computation, section 3.1 via 3.2) ---------
 * P, Q: device float64 n x k (ld) -- pair j is (P[:, j], Q[:, j]).
 * opts: NULL for defaults.
 * d_out: device float64 [k] receives d_j.
 * X_inout: device float64 n x k (ldx) or NULL; on return holds x_j = L^+
 *   delta_j (mean zero on every component).  With NVD_WARM_START it also
 *   supplies the starting guess.
 * info: host array of k nvd_pair_info or NULL.
 * Synchronous with respect to `stream` (see Streams).  On a connected graph
 * with the Jacobi preconditioner and no warm start, a tile of up to about
 * 1e6 vector elements (n times the tile) is solved by one kernel launch
 * (one block, or a cooperative launch of up to 256 blocks); NVD_E_DEVICE if
 * that launch gives up at a barrier. */
nvd_status nvd_distances(nvd_graph* g, int32_t k, const double* P,
                         const double* Q, int64_t ld, const nvd_opts* opts,
                         double* d_out, double* X_inout, int64_t ldx,
                         nvd_pair_info* info, void* stream);

/* ---- distances without device allocation ---------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the solve
 * of nvd_distances (same arguments, same kernels, same results up to the
 * order of floating-point sums), with every device buffer beyond the
 * caller's inputs and outputs taken from one fixed array of 64 MiB that the
 * library holds on each GPU it runs on until the process ends.  The call
 * allocates nothing, on the device or in pinned host memory.
 * Limits: the solve of the widest tile T must fit the array, about
 *   56 n T bytes (mixed; 40 n T in FP64) + 6.5 MiB + 512 n_comp bytes,
 * so n T up to about 1e6 (NVD_E_UNSUPPORTED beyond, with the size in the
 * message); only the Jacobi preconditioner (NVD_PRECOND_TREE, AUTO and ACHOL
 * give NVD_E_UNSUPPORTED); the tile is opts->tile_k, else the autotuner's cached
 * choice for this graph, else a fixed heuristic (nothing is timed).
 * The array keeps the last call's contents; each call clears what must
 * start at zero.  Calls that overlap on one GPU (two streams or threads)
 * race on the array: serialise them.  Synchronous, as nvd_distances. */
nvd_status nvd_distances_noalloc(nvd_graph* g, int32_t k, const double* P,
                                 const double* Q, int64_t ld, const nvd_opts* opts,
                                 double* d_out, double* X_inout, int64_t ldx,
                                 nvd_pair_info* info, void* stream);

/* ---- all pairwise distances among m node vectors --------------------------
 * D[i][j] = d(v_i, v_j) (section 3.1 distance) for the m columns of V, from
 * ONE solve with m right-hand sides: X = L^+ V_bar (section 3.2 solve, the
 * tiles and precision of nvd_distances), R = V_bar - L X its final FP64
 * residuals, and
 *     Gt = V_bar^T X + X^T R,   D_ij^2 = Gt_ii + Gt_jj - Gt_ij - Gt_ji,
 * which equals, by linearity, the quadratic form delta^T x + x^T r of the
 * pair delta = v_i - v_j: every distance has the accuracy of a pair solved
 * on its own.
 * V: device float64 n x m, row-major, leading dimension ld (>= m); 1 <= m
 *   <= 4096 (NVD_E_UNSUPPORTED above).
 * opts: as for nvd_distances (NULL: defaults); NVD_WARM_START is rejected.
 * D: device float64 m x m (ldd >= m): symmetric, zero diagonal.
 * G: NULL or device float64 m x m (ldg >= m): (Gt + Gt^T) / 2, the Gram
 *   matrix of the vectors in the L^+ inner product.
 * info: NULL or host [m]: per-column solve outcome (status as for
 *   nvd_distances; the return value aggregates NOCONV / BREAKDOWN).
 * Needs 3 n m + O(m^2) doubles of device scratch, allocated and freed by the
 * call.  Synchronous with respect to `stream`. */
nvd_status nvd_pairwise(nvd_graph* g, int32_t m, const double* V, int64_t ld,
                        const nvd_opts* opts, double* D, int64_t ldd, double* G,
                        int64_t ldg, nvd_pair_info* info, void* stream);

/* ---- tile autotuner --------------------------------------------------------
 * The tile (pairs per SpMM pass) and the number of lane sub-groups that
 * share each row's neighbours in the Laplacian apply (nl), which
 * nvd_distances uses for k pairs when opts->tile_k == 0.  Candidates are
 * timed on this graph on first use (whole CG iterations; device work on
 * `stream`) and cached in the handle.  Environment variable NVD_TUNE=0
 * selects a fixed heuristic. */
nvd_status nvd_tune_query(nvd_graph* g, int32_t k, int32_t precision,
                          int32_t* tile, int32_t* nl, void* stream);

/* ---- new edge weights for an existing graph -------------------------------
 * w: device float64 [nnz] in the order of the CSR given to nvd_graph_create
 * (self-loop entries ignored).  Replaces the weights (a graph created with
 * unit weights becomes weighted), recomputes degrees and their inverses, and
 * checks on the device, before anything is replaced, that every value is
 * finite and positive and equal to its mirror entry's (NVD_E_GRAPH
 * otherwise; the graph then keeps its previous weights).
 * Synchronous with respect to `stream`.  Batches made earlier keep their
 * own copy; a spanning forest built for the tree preconditioner is dropped
 * and rebuilt from the new weights when next needed. */
nvd_status nvd_graph_set_weights(nvd_graph* g, const double* w, void* stream);

/* ---- adjoint of d^2 with respect to the edge weights ---------------------
 * Given X (device float64 n x k, ldx; normally the X_inout of a previous
 * nvd_distances call) and gscale (device float64 [k], the upstream
 * dLoss/d(d_j^2)), writes for every entry e = (i, j) of the CSR passed to
 * nvd_graph_create (same order, self-loop entries get 0):
 *     grad_w[e] = -1/2 * sum_j gscale_j * (X[i, j] - X[c, j])^2,  c = col_idx[e],
 * so that the two stored directions of an edge sum to d(sum_j g_j d_j^2)/dw
 * of that undirected edge (section 3.1's L is linear in w: dL/dw_e is the
 * Laplacian of the single edge e, and d(delta^T L^+ delta)/dw_e =
 * -(x_i - x_j)^2 with x = L^+ delta).  grad_w: device float64 [nnz].
 * Asynchronous. */
nvd_status nvd_grad_weights(nvd_graph* g, int32_t k, const double* X,
                            int64_t ldx, const double* gscale, double* grad_w,
                            void* stream);

/* ---- adjoint of d^2 with respect to the node vectors ----------------------
 * d(sum_j g_j d_j^2)/dP = 2 X diag(gscale) and d/dQ = -2 X diag(gscale),
 * with X the saved solutions (x_j = L^+ delta_j; L^+ is symmetric, so no
 * second solve).  X: device float64 n x k (ldx); gscale: device [k];
 * GP, GQ: device float64 n x k (ldp, ldq), either may be NULL (not both).
 * Asynchronous. */
nvd_status nvd_grad_vectors(nvd_graph* g, int32_t k, const double* X,
                            int64_t ldx, const double* gscale, double* GP,
                            int64_t ldp, double* GQ, int64_t ldq, void* stream);

/* ---- upstream gradient on d to the scale on d^2 ---------------------------
 * gscale_j = g_d_j / (2 d_j) where d_j > 0, else 0 (d is not differentiable
 * at 0; zero is the minimum-norm subgradient).  Feeds nvd_grad_vectors and
 * nvd_grad_weights for gradients of d itself.  All device float64 [k].
 * Asynchronous. */
nvd_status nvd_grad_scale_from_d(int32_t k, const double* g_d, const double* d,
                                 double* gscale, void* stream);

/* ---- batches of graphs ----------------------------------------------------
 * nvd_batch_create packs G graphs into one device structure (the graphs may
 * be destroyed afterwards).  nvd_batch_distances solves k_g pairs on every
 * graph g: FP32 CG with FP64 iterative refinement (opts->precision
 * NVD_MIXED, the default for batches) or FP64 CG.  Two solvers:
 *  - sweep (default): the graphs form one block-diagonal operator; every
 *    phase is one kernel over the rows of all graphs still open, each graph
 *    and pair keeping its own CG scalars (a few launches per iteration).
 *  - persistent (opts->flags & NVD_BATCH_PERSISTENT): one cooperative
 *    launch in which blocks or teams of blocks take graphs from a work plan.
 * k_per_graph: host int32 [G] (each 1..64).
 * P, Q: device float64, graph-major packed: graph g's block is n_g x k_g
 *   row-major (leading dimension k_g) starting at element offset
 *   sum_{h<g} n_h k_h.
 * d_out: device float64 [sum k_g] (graph-major).  X_out: NULL or device
 *   float64 packed like P.  info: NULL or host [sum k_g].
 * Graphs must be connected (NVD_E_UNSUPPORTED at create time otherwise).
 * The persistent launch is captured in a hipGraph and replayed by later
 * calls with the same pointers, pair counts and options (NVD_BATCH_GRAPH=0
 * launches directly).  Synchronous with respect to `stream`. */
nvd_status nvd_batch_create(int32_t G, nvd_graph* const* graphs, void* stream,
                            nvd_batch** out);
nvd_status nvd_batch_destroy(nvd_batch* b);
/* Counts of how batched calls ran: launches captured into a hipGraph,
 * replays of a captured graph (calls whose arguments matched the previous
 * capture), and direct launches (capture off via NVD_BATCH_GRAPH=0, or
 * refused by the runtime). */
nvd_status nvd_batch_query(const nvd_batch* b, int64_t* captures,
                           int64_t* replays, int64_t* eager);
/* Per-graph timing of the last nvd_batch_distances call made with the
 * environment variable NVD_BATCH_TRACE=1: start_end (host int64 [2G])
 * receives device wall-clock ticks (100 MHz) at the start and end of each
 * graph's solve, team_size (host int32 [G]) the number of blocks that solved
 * it.  NVD_E_ARG if no trace was recorded. */
nvd_status nvd_batch_trace(const nvd_batch* b, int32_t G, int64_t* start_end,
                           int32_t* team_size);
nvd_status nvd_batch_distances(nvd_batch* b, const int32_t* k_per_graph,
                               const double* P, const double* Q,
                               const nvd_opts* opts, double* d_out,
                               double* X_out, nvd_pair_info* info,
                               void* stream);

/* ---- launch timing (instrumentation) -------------------------------------
 * When enabled, every launch of the solver's SpMM, CG-update and
 * CG-direction kernels is bracketed by HIP events on its stream.
 * nvd_prof_read (host arrays of NVD_PROF_KINDS entries) returns, per kind,
 * the summed kernel milliseconds, the launch count and the algorithmic
 * bytes those launches must move (CSR once, each vector stream once), then
 * clears the record.  Kinds: 0 SpMM FP64, 1 SpMM FP32, 2 update FP64,
 * 3 update FP32, 4 direction FP64, 5 direction FP32, 6 other. */
#define NVD_PROF_KINDS 7
nvd_status nvd_prof_enable(int32_t on);
nvd_status nvd_prof_read(double* ms, int64_t* launches, double* bytes);

#ifdef __cplusplus
}
#endif
#endif /* NVD_H */
