/*
 * kkt.h -- C ABI of the MI355X sparse KKT refactorization library.
 *
 * The library solves a sequence of linear systems K_k x_k = b_k, k = 1..M, whose matrices
 * share one sparsity pattern while their values change (the interior-point Newton systems
 * of Section II, eq. (12)).  It follows the refactorization strategy of Section III,
 * Algorithm 1: the first system is analysed and factored once on the host (ordering,
 * equilibration, pivot order and the pattern of L and U, as in the analysis stage of the
 * three-stage direct solver of Section II); every later system is refactored on the GPU
 * with that pattern and pivot order fixed, solved by forward/backward substitution and
 * refined iteratively.  The paper allows the permutations to come from any LU solver;
 * kkt_opts.fixed_p / fixed_q accept them.
 *
 * Conventions
 *  - Matrices are square, in CSR with int64 row pointers and int32 column indices, rows
 *    sorted ascending, no duplicates, every diagonal entry present, both triangles stored
 *    (no symmetry is assumed).  Values are FP64 in that CSR order.
 *  - "host" pointers are ordinary CPU memory; "device" pointers are GPU memory of the
 *    device that was current at kkt_bind.  Every buffer belongs to the caller; the library
 *    owns only the host handle.  The device workspace (kkt_workspace_bytes) is caller
 *    memory that the library carves up; it must stay allocated until kkt_destroy.
 *  - Calls that take a stream are enqueued on it and return without waiting unless stated.
 *  - Indices of the symbolic export are 0-based in the permuted index space: row k of
 *    P A Q is row P[k] of A and column k is column Q[k].
 *  - Return value: 0 = KKT_OK, > 0 = warning, < 0 = error.  A handle is not thread safe;
 *    distinct handles are independent.
 */
#ifndef KKT_H
#define KKT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *hipStream_t;   /* identical to HIP's own typedef */

#define KKT_OK 0
#define KKT_WARN_PIVOT_PERTURBED 1  /* a refactor replaced tiny pivots (kkt_info) */
#define KKT_WARN_NOT_CONVERGED 2    /* refinement stopped at max_iters above berr_tol */
#define KKT_ERR_ARG (-1)            /* null pointer, bad size, bad option, a size beyond the int32
                                     * indices of the device structures */
#define KKT_ERR_PATTERN (-2)        /* non-square, unsorted, duplicate, out of range, no diagonal */
#define KKT_ERR_SINGULAR (-3)       /* analyze found a pivot step with no nonzero candidate */
#define KKT_ERR_NONFINITE (-4)      /* NaN/Inf in values or factors */
#define KKT_ERR_STATE (-5)          /* call order: refactor before bind, solve before refactor */
#define KKT_ERR_NOMEM (-6)          /* host allocation failed or workspace too small */
#define KKT_ERR_DEVICE (-7)         /* a HIP call failed */
#define KKT_ERR_SCHEDULE (-8)       /* the analysed structure broke an internal invariant or limit of
                                     * the GPU schedule (a library fault, not a property of the input) */

typedef struct kkt_handle kkt_handle;

typedef struct {
    /* Pivot rule at analyze (Algorithm 1, first system): the diagonal candidate is kept
     * when it is nonzero and |x_diag| >= pivot_tau * max|candidates|; otherwise the largest
     * candidate (lowest row index on ties).  0 = static diagonal pivoting (default). */
    double pivot_tau;
    /* Refactor: |u_kk| < tiny_pivot * ||A~||_inf is replaced by +-tiny_pivot*||A~||_inf
     * (sign kept, zero counts as +) and counted.  Default 2^-40: on the grid KKT systems the
     * small pivots are genuine (the Schur complements of the -delta_c I block), and
     * replacing them at 2^-26 (the square root of the unit roundoff) cost refinement steps
     * that 2^-34 and below never needed. */
    double tiny_pivot;
    /* 1 = power-of-two row-then-column max equilibration, recomputed per refactor. */
    int32_t equilibrate;
    /* FGMRES restart length m (1..64), iteration cap, backward-error target. */
    int32_t gmres_restart;
    int32_t max_iters;
    double berr_tol;
    /* Maximum width of a structural supernode in the symbolic export (>= 1). */
    int32_t sn_max_width;
    /* Optional externally chosen permutations (host, int32[n]); fixed_p requires fixed_q.
     * With fixed_q the ordering step is skipped; with both, pivoting is skipped too. */
    const int32_t *fixed_p;
    const int32_t *fixed_q;
    /* 1 = dense supernodal update blocks (a wide source panel updating several target
     * columns) run on the FP64 matrix cores (default); 0 = vector FMAs. */
    int32_t dense_mfma;
    /* 1 = hybrid triangular solves (default): one launch per dependency level while levels
     * are wide, and one persistent launch for the narrow levels at the top of the tree, in
     * which blocks take work items in dependency order and wait, bounded, for the unknowns
     * they read; items are assigned to blocks in a fixed order, which needs every block of
     * the launch resident (a cooperative launch on a device the solve has to itself).
     * 2 = the same with items taken from a ticket counter by the running blocks: slightly
     * slower, but safe when other streams' work shares the device (the serving engine
     * uses it).  0 = one launch per dependency level throughout.  All three give bitwise
     * identical results. */
    int32_t persistent_solve;
    /* 1 = the refactorization's per-level launches (everything after the value update) are
     * recorded into a HIP graph at the first kkt_refactor after kkt_bind and replayed by
     * later calls on the caller's stream (default); they are launched one by one while the
     * launch profiler is on, when the caller's stream is itself being captured, or when
     * recording fails.  0 = always one by one.  Results are bitwise identical either way. */
    int32_t graph_refactor;
    /* 0 = every preconditioner application inside kkt_refine is an exact triangular solve
     * (default).  k in 1..1024 = the applications inside the FGMRES iterations are
     * approximate instead (Section V: the triangular solves approximated by Jacobi or
     * Gauss-Seidel iterations): k sweeps per triangle of the kind approx_kind, each triangle
     * from the zero vector; the first solve of kkt_refine and kkt_solve stay exact, and
     * FGMRES, being flexible, accepts the varying preconditioner.  kkt_solve_approx applies
     * the approximation alone. */
    int32_t approx_sweeps;
    /* Storage and arithmetic of the factors (the mixed-precision pattern of the refactor
     * path): KKT_FP64 (default) or KKT_FP32 = the value update rounds the scaled values to
     * FP32 once, the refactorization computes in FP32 (dense update blocks on the FP32 matrix
     * cores, FP32 accumulation) and stores FP32 factors; the triangular solves read the FP32
     * factors into FP64 sums; residuals, orthogonalisation and the solution update of the
     * refinement stay FP64, so kkt_refine still reaches berr_tol on the original A. */
    int32_t factor_precision;
    /* Tiny-pivot factor of the FP32 factors (in place of tiny_pivot): default 2^-26
     * (measured on the grid workloads: larger factors such as 2^-12 replace so many pivots
     * that refinement needs tens to hundreds of FGMRES steps, and smaller ones leave FP32
     * pivots so small that refinement stalls). */
    double tiny_pivot_fp32;
    /* Kind of the approximate sweeps: 0 = Jacobi (every row reads the previous iterate;
     * default), 1 = block Gauss-Seidel (rows cut into chunks of 32 consecutive rows of the
     * permuted order; inside its chunk a row uses the values already updated in the sweep,
     * ascending for L and descending for U, and the previous iterate elsewhere). */
    int32_t approx_kind;
} kkt_opts;

#define KKT_FP64 0
#define KKT_FP32 1

typedef struct {
    int32_t iters;              /* FGMRES (Arnoldi) steps after the first solve */
    int32_t status;             /* KKT_OK, KKT_WARN_NOT_CONVERGED or an error */
    double berr;                /* ||b - A x||_inf / (||A||_inf ||x||_inf + ||b||_inf) */
    int64_t perturbed_pivots;   /* pivots replaced by the last kkt_refactor */
} kkt_info;

typedef struct {
    int32_t n;                  /* order N */
    int32_t nsn;                /* structural supernodes */
    int64_t nnz_a;              /* entries of A */
    int64_t nnz_lu;             /* entries of the combined L+U (diagonal included) */
    int32_t levels_f;           /* refactor dependency levels (columns) */
    int32_t levels_l;           /* forward-solve levels (rows) */
    int32_t levels_u;           /* backward-solve levels (rows) */
    int32_t gpu_levels_f;       /* launches of one GPU refactorization */
    int32_t gpu_levels_l;       /* launches of one GPU forward solve */
    int32_t gpu_levels_u;       /* launches of one GPU backward solve */
    int32_t persistent_levels_l; /* forward levels run by the persistent launch */
    int32_t persistent_levels_u; /* backward levels run by the persistent launch */
    double flops_refactor;      /* sum_k 2 |L(:,k)| |U(k,:)| + |L(:,k)| */
    int64_t nnz_lu_wide;        /* L+U entries of the columns factored by the 512-thread launches
                                 * (their wide items and the narrow items that ride with them) */
    int64_t nnz_lu_medium;      /* L+U entries of the columns factored by the 256-thread launches
                                 * of panels up to 16 columns */
    int64_t copy_in_levels;     /* entries of the row-ordered factor copy done by the level
                                 * launches (the rest by a copy after the last level) */
    int64_t nnz_lu_w256;        /* L+U entries of the columns factored by the 256-thread launches
                                 * of panels up to 32 columns (kkt_tuning.wide256) */
} kkt_stats;

/* Fills *o with the defaults listed in kkt_opts. */
void kkt_default_opts(kkt_opts *o);

/* Analysis stage (Section II; Algorithm 1, factor the first system, extract the
 * permutations and the L/U pattern, convert the layout).  Host only, no device work.
 * rowptr int64[n+1], colind int32[nnz], values_k1 FP64[nnz] (all host, borrowed for the
 * call only); opts may be NULL for defaults.  On success *out owns a new handle.
 * Errors: ARG, PATTERN, SINGULAR, NONFINITE, NOMEM. */
int kkt_analyze(int32_t n, const int64_t *rowptr, const int32_t *colind,
                const double *values_k1, const kkt_opts *opts, kkt_handle **out);

/* A new, unbound handle with src's analysis, options and schedule (host copies; no
 * analysis is repeated): several resident replicas of one pattern, each with its own
 * workspace, can then serve requests at the same time.  Errors: ARG, NOMEM. */
int kkt_clone(const kkt_handle *src, kkt_handle **out);

/* Sizes and schedule statistics of an analysed handle. */
int kkt_get_stats(const kkt_handle *h, kkt_stats *out);

/* Canonical symbolic factorization (host copies; every pointer is caller memory of the
 * stated size, any may be NULL to skip it):
 *   P, Q int32[n]; colptr int64[n+1]; rowidx int32[nnz_lu] -- combined L+U in CSC, per
 *   column U rows ascending, the diagonal, then L rows ascending; parent int32[n] (first
 *   L row below the diagonal, -1 if none); lev_f, lev_l, lev_u int32[n]; sn_start
 *   int32[nsn+1]; map int64[nnz_a] (slot in rowidx of each input entry, CSR order). */
int kkt_export_symbolic(const kkt_handle *h, int32_t *P, int32_t *Q, int64_t *colptr,
                        int32_t *rowidx, int32_t *parent, int32_t *lev_f, int32_t *lev_l,
                        int32_t *lev_u, int32_t *sn_start, int64_t *map);

/* Device bytes that kkt_bind needs for right-hand sides of up to max_nrhs columns. */
int kkt_workspace_bytes(const kkt_handle *h, int32_t max_nrhs, size_t *bytes);

/* Setup (Algorithm 1, set up the GPU refactorization): uploads the symbolic structure and
 * schedules into d_workspace (device, >= kkt_workspace_bytes, 256-byte aligned) on stream
 * and records the device; the first bind also creates the handle's internal stream, which
 * only records the refactorization graph.  Binding again drops the recorded graph.  A handle stays on its first device: binding again on
 * another one returns STATE.  Waits for the upload.
 * Errors: ARG, NOMEM (too small), STATE, DEVICE. */
int kkt_bind(kkt_handle *h, void *d_workspace, size_t bytes, int32_t max_nrhs,
             hipStream_t stream);

/* Size of the library's static device scratch array used by kkt_bind_scratch (64 MiB per
 * device; enough for the workspace of a KKT system of about 5,000 buses). */
#define KKT_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): kkt_bind with the workspace taken from
 * the library's own static device array of KKT_SCRATCH_BYTES bytes instead of caller
 * memory.  This call allocates nothing (no device or pinned host memory, no stream, event
 * or graph); later calls on the handle allocate nothing either: its refactorizations launch
 * their levels one by one instead of recording a graph, and small read-backs go through a
 * host array inside the handle.  Every device holds one such array, kept until the process
 * ends, and at most one handle is bound to it: binding another handle on the same device
 * unbinds the previous one (its later calls return STATE) and overwrites the array, so
 * calls of handles that use it must not overlap in time (they race on one array); the
 * caller orders them.  Results are bitwise identical to the same handle bound by kkt_bind.
 * Waits for the upload.  Errors: ARG, NOMEM (kkt_workspace_bytes exceeds KKT_SCRATCH_BYTES),
 * STATE (handle already on another device), DEVICE. */
int kkt_bind_scratch(kkt_handle *h, int32_t max_nrhs, hipStream_t stream);

/* Value update and refactorization without pivoting (Algorithm 1, update the factor
 * object with the new values, refactor).  d_values: device FP64[nnz_a] in the analysed
 * CSR order, BORROWED until the next kkt_refactor or kkt_destroy (kkt_refine reads it for
 * residuals).  Asynchronous: a one-thread launch stores the values pointer in the
 * workspace, then the value update and the level launches run on stream, replayed from the
 * graph recorded at the first call after kkt_bind when opts.graph_refactor is set (the first
 * call also records it, which takes longer).  Calls
 * on one handle must be ordered by the caller (they share the workspace).  Errors: ARG,
 * STATE (not bound), DEVICE.  Tiny pivots and non-finite factors are reported by
 * kkt_refine / kkt_refactor_status. */
int kkt_refactor(kkt_handle *h, const double *d_values, hipStream_t stream);

/* Waits for the last refactorization; *perturbed = replaced pivots.  Returns OK,
 * WARN_PIVOT_PERTURBED, ERR_NONFINITE or ERR_STATE. */
int kkt_refactor_status(kkt_handle *h, int64_t *perturbed, hipStream_t stream);

/* Triangular solves (Algorithm 1, triangular solve), no refinement:
 * x = Q C (L U)^-1 P R b.  d_b, d_x: device FP64, column j at offset j*ld, nrhs columns,
 * ld >= n; d_x may equal d_b.  Asynchronous.  Errors: ARG, STATE, DEVICE. */
int kkt_solve(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld,
              hipStream_t stream);

/* One approximate preconditioner application (Section V): x = Q C x~ with x~ from
 * opts.approx_sweeps sweeps of kind opts.approx_kind on U x~ = y after as many on
 * L y = P R b, each from the zero vector.  Same buffers and ld rules as kkt_solve.
 * Asynchronous.  Errors: ARG (also when approx_sweeps is 0), STATE, DEVICE. */
int kkt_solve_approx(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld,
                     hipStream_t stream);

/* Solve followed by FGMRES(m) iterative refinement with FP64 residuals on the original A
 * (Algorithm 1: the solve is always followed by iterative refinement; Section V: a
 * configurable refinement).  Stops when berr <= berr_tol or after max_iters Arnoldi steps.
 * info: host kkt_info[nrhs] (may be NULL).  Waits for completion.  Returns OK,
 * WARN_NOT_CONVERGED (some column missed the target), or an error. */
int kkt_refine(kkt_handle *h, const double *d_b, double *d_x, int32_t nrhs, int64_t ld,
               kkt_info *info, hipStream_t stream);

/* One step of Algorithm 1 for one right-hand side: kkt_refactor(h, d_values) followed by
 * kkt_refine(h, d_b, d_x, 1, n, info), with the same results bit for bit (factors, x and
 * info).  The forward substitution of the first solve rides in the refactorization's level
 * launches: each forward level runs in the first launch after the columns its rows read are
 * factored and copied, the last levels after the last launch (replayed from a second graph
 * recorded at the first call after kkt_bind when opts.graph_refactor is set; launched one by
 * one without graphs, with the profiler on or on a capturing stream).  d_values as for
 * kkt_refactor (BORROWED); d_b, d_x: device FP64[n], d_x may equal d_b; info: host
 * kkt_info[1] (may be NULL).  Waits for completion.  Returns what kkt_refine returns; a
 * failed factorization (ERR_NONFINITE, ERR_DEVICE) is reported with info = {0, error, inf,
 * perturbed pivots}, d_x then holds no solution.  Errors also: ARG, STATE (not bound). */
int kkt_refactor_refine(kkt_handle *h, const double *d_values, const double *d_b, double *d_x,
                        kkt_info *info, hipStream_t stream);

/* Test hook: copies the factors of the last refactorization to host memory in the
 * canonical L+U CSC order (FP64[nnz_lu]) and the scale factors (FP64[n] each, may be
 * NULL).  Waits. */
int kkt_export_factors(kkt_handle *h, double *h_lu, double *h_r, double *h_c,
                       hipStream_t stream);

/* Schedule choices of the GPU refactorization (they change launch shapes and rounding
 * order, never the symbolic factorization):
 *   panel_max  widest panel cut from a supernode (1..32; default 32);
 *   small_rows narrow 16-lane path for panels of <= 4 columns and <= small_rows rows below
 *              (0..64; default 64);
 *   group      targets of one source panel grouped into one pull item (1..32; default 32);
 *   wide256    1 = a level with at least 256 wide items, all factoring panels of at most 256
 *              rows, runs them in 256-thread blocks (two per compute unit) instead of
 *              512-thread blocks (default), 0 = always 512;
 *   fuse_chains 1 = consecutive panels of one supernode are factored by one item (with the
 *              pulls between them) whenever no outside dependency would wait for it, so a
 *              wide supernode costs one launch instead of one per panel; 0 = one panel per
 *              item (default: on the grid workloads the fused items serialise trailing
 *              updates that separate items run in parallel);
 *   tiny_rows  narrow items whose panel and sources all have <= tiny_rows rows below run on
 *              4 lanes instead of 16 in the launches of levels without wide items, so four
 *              times as many are in flight (0..16; default 16; 0 = never).  Same operations
 *              in the same order: the factors do not depend on it. */
typedef struct {
    int32_t panel_max;
    int32_t small_rows;
    int32_t group;
    int32_t wide256;
    int32_t fuse_chains;
    int32_t tiny_rows;
} kkt_tuning;

/* The handle's current schedule choices. */
int kkt_get_tuning(const kkt_handle *h, kkt_tuning *t);

/* Rebuilds the schedule with the given choices (host).  A bound handle is unbound first
 * (after its last refactorization finished): bind again, since the workspace size may
 * change.  Errors: ARG (values out of range), SCHEDULE, NOMEM, DEVICE. */
int kkt_set_tuning(kkt_handle *h, const kkt_tuning *t);

/* Autotuner of the schedule: for each candidate (panel_max 32/16/8, small_rows 64/32,
 * group 32/16, wide256 1/0, fuse_chains 0/1; tiny_rows as set) builds the schedule, binds a temporary workspace (allocated and freed
 * here), refactors d_values (device FP64[nnz_a]) once and then reps times under HIP
 * events on stream, and keeps the fastest; returns with that schedule set and the handle
 * unbound (bind again).  best / best_ms (host, may be NULL) receive the choice and its
 * mean refactorization time in ms.  Errors: ARG, NOMEM, DEVICE, or a refactorization
 * error (NONFINITE). */
int kkt_autotune(kkt_handle *h, const double *d_values, int32_t reps, kkt_tuning *best, double *best_ms,
                 hipStream_t stream);

/* Batched refactorization (many same- or different-pattern systems per call): a batch
 * groups bound handles of one device and one factor precision; kkt_batch_refactor then
 * does for all of them what kkt_refactor does for one, with one launch per dependency
 * level across the batch (each handle's share of a launch runs exactly the blocks of its
 * own launch, so every result is bitwise the one of kkt_refactor alone), the value update
 * merged likewise, and all launches of a step recorded at the first call into one HIP
 * graph that later calls replay. */
typedef struct kkt_batch kkt_batch;

/* handles: host array of count distinct bound handles.  The batch keeps pointers to them
 * and to their workspaces: a handle must stay alive and bound to the same workspace while
 * the batch is used (calls return STATE otherwise).  Allocates a small device table.
 * Errors: ARG (null, duplicate, mixed device or precision), STATE (unbound), NOMEM, DEVICE. */
int kkt_batch_create(kkt_handle *const *handles, int32_t count, kkt_batch **out);

/* d_values: host array of count device pointers, the values of each handle's system in
 * its analysed CSR order (borrowed as by kkt_refactor).  Asynchronous on stream; each
 * handle is then refactored as if kkt_refactor had been called on it (kkt_refactor_status,
 * kkt_solve and kkt_refine work per handle).  Errors: ARG, STATE, DEVICE. */
int kkt_batch_refactor(kkt_batch *b, const double *const *d_values, hipStream_t stream);

/* kkt_refine of every handle of the batch with one right-hand side each: d_b, d_x host
 * arrays of count device pointers (FP64[n] of that handle), info host kkt_info[count] (may
 * be NULL).  Up to 8 handles are refined at once, each by a host thread on a stream of the
 * batch ordered after the caller's stream (which is why a batch's handles take their
 * persistent solve items by ticket, see persistent_solve = 2).  Waits.  Returns the first
 * error, else the worst warning. */
int kkt_batch_refine(kkt_batch *b, const double *const *d_b, double *const *d_x, kkt_info *info,
                     hipStream_t stream);

/* Frees the batch (not the handles).  NULL is ignored. */
void kkt_batch_destroy(kkt_batch *b);

/* Serving (a request loop with continuous admission; kkt_server.cpp).  Each pattern is
 * analysed once when registered; its resident replicas (kkt_clone of the analysed handle,
 * each bound to a workspace the server allocates) keep the symbolic structure and the
 * factors on the device between requests.  A request is one system of a registered
 * pattern: refactor (Algorithm 1) + solve + FGMRES refinement for 1..max_nrhs right-hand
 * sides.  Requests wait in arrival order; max_inflight worker threads, one HIP stream each,
 * take the first request that can run now (a free replica of its pattern, or a new replica
 * while all workspaces stay within hbm_budget bytes, evicting idle replicas of other
 * patterns, least recently used first, when that makes room), so requests that arrive
 * while others run are admitted as slots and memory free up and their work overlaps on the
 * device.  Every replica of a pattern runs the same kernels, so a result does not depend
 * on what else runs. */
typedef struct kkt_server kkt_server;
typedef struct {
    size_t hbm_budget;     /* device bytes of all replica workspaces together (default 16 GiB) */
    int32_t max_inflight;  /* requests running at once, 1..64 (default 4) */
    int32_t max_nrhs;      /* right-hand sides per request, >= 1 (default 4) */
} kkt_server_opts;
typedef struct {
    int32_t replicas, patterns;
    size_t bytes_in_use, peak_bytes;
    int64_t replicas_created, evictions, completed, queued;
} kkt_server_stats;

void kkt_server_default_opts(kkt_server_opts *o);

/* Starts the worker threads on the current device.  Errors: ARG, NOMEM, DEVICE. */
int kkt_server_create(const kkt_server_opts *opts, kkt_server **out);

/* Analyses a pattern (as kkt_analyze; host arrays borrowed for the call) and registers it;
 * *pattern receives its index.  NOMEM when one replica's workspace exceeds the budget. */
int kkt_server_add_pattern(kkt_server *s, int32_t n, const int64_t *rowptr, const int32_t *colind,
                           const double *values_k1, const kkt_opts *opts, int32_t *pattern);

/* Queues a request; returns at once with *ticket.  d_values (FP64[nnz], CSR order of the
 * pattern), d_b and d_x (nrhs columns at stride ld >= n; d_x may equal d_b) are device
 * memory of the server's device, borrowed until kkt_server_wait returns for the ticket.
 * A request runs as kkt_refactor then kkt_refine on its replica (as kkt_refactor_refine for
 * one right-hand side: the same results).  Errors: ARG, NOMEM. */
int kkt_server_submit(kkt_server *s, int32_t pattern, const double *d_values, const double *d_b, double *d_x,
                      int32_t nrhs, int64_t ld, int64_t *ticket);

/* Waits for a ticket and forgets it.  info: host kkt_info[nrhs] (may be NULL); times_ms:
 * host double[4] (may be NULL) = admission wait, time on the device, latency (submit to
 * completion), 1 if a new replica was made for it.  Returns the request's status (as
 * kkt_refine).  ARG for an unknown ticket.  Not concurrently with kkt_server_destroy. */
int kkt_server_wait(kkt_server *s, int64_t ticket, kkt_info *info, double *times_ms);

int kkt_server_get_stats(kkt_server *s, kkt_server_stats *out);

/* Stops the workers after their running requests, drops queued ones, frees every replica
 * and pattern.  NULL is ignored. */
void kkt_server_destroy(kkt_server *s);

/* Kernel classes timed by the optional launch profiler. */
#define KKT_PROF_UPDATE 0          /* equilibration, norms, value gather, counters */
#define KKT_PROF_REFACTOR_LARGE 1  /* 512-thread level launches: wide panel items up to 32 columns
                                    * (LDS-staged, matrix cores) and the level's narrow items */
#define KKT_PROF_REFACTOR_SMALL 2  /* narrow-only level launches (16 lanes per item) */
#define KKT_PROF_TO_CSR 3          /* row-ordered copy of the factors */
#define KKT_PROF_LSOLVE 4          /* forward substitution (and its Jacobi sweeps; with
                                    * kkt_refactor_refine only its last levels and the set-up,
                                    * the others ride in the refactorization's launches) */
#define KKT_PROF_USOLVE 5          /* backward substitution (and its Jacobi sweeps) */
#define KKT_PROF_RESIDUAL 6        /* residual, products with A */
#define KKT_PROF_KRYLOV 7          /* FGMRES vector kernels */
#define KKT_PROF_REFACTOR_MEDIUM 8 /* 256-thread level launches: wide items of panels up to 16
                                    * columns and the level's narrow items */
#define KKT_PROF_REFACTOR_W256 9   /* 256-thread level launches: wide items of panels up to 32
                                    * columns with factored panels of at most 256 rows, and the
                                    * level's narrow items */
#define KKT_PROF_NCLASS 10

typedef struct {
    int64_t launches[KKT_PROF_NCLASS];
    double ms[KKT_PROF_NCLASS];      /* summed GPU time between the events around the launches */
} kkt_profile;

/* Test and benchmark hook: on = 1 resets the counters and records a pair of HIP events
 * around every later kernel launch of the handle (on the caller's stream), one pair around
 * each run of consecutive refactorization level launches of one class (so a class's time per
 * launch carries the events' cost once per run); the levels are then launched one by one
 * instead of from the recorded graph.  on = 0 stops.  Adds a few microseconds per pair while
 * on. */
int kkt_profile_enable(kkt_handle *h, int32_t on);

/* Waits for the stream and returns the accumulated launch counts and times. */
int kkt_profile_read(kkt_handle *h, kkt_profile *out, hipStream_t stream);

/* Frees the handle (not the caller's workspace).  NULL is ignored. */
void kkt_destroy(kkt_handle *h);

/* Static description of a status code. */
const char *kkt_strerror(int status);

#ifdef __cplusplus
}
#endif

#endif /* KKT_H */
