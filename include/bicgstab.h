/*
 * bicgstab.h -- C ABI of the MI355X multi-right-hand-side BiCGStab library.
 *
 * The library solves A X = B for a general sparse square matrix A (CSR, int32
 * indices) and k right-hand sides at once with the BiCGStab methods analysed
 * in Krasnopolsky, "Revisiting Performance of BiCGStab Methods for Solving
 * Systems with Multiple Right-Hand Sides" (arXiv:1907.12874):
 *   - classical BiCGStab            (Appendix B, Alg. 1 basic; Alg. 2 / Alg. 5 merged)
 *   - Reordered BiCGStab            (Appendix B, Alg. 6; its recurrence
 *                                    rho_{j+1} = -omega_j psi_j is checked
 *                                    against a running bound of the rounding
 *                                    it has absorbed, and a column whose rho
 *                                    has fallen to that bound restarts with
 *                                    r_{j+1} as its shadow vector: the paper
 *                                    leaves such convergence issues aside)
 *   - Pipelined BiCGStab            (Appendix B, Alg. 4 / Alg. 7)
 *   - Improved BiCGStab             (Appendix B, Alg. 3)
 * each in the "basic" form (one memory pass per vector operation, the Basic
 * columns of Table 2) and the "merged" form (the operations of one listing
 * line share one pass, the Merged columns of Table 2), optionally with a
 * Jacobi preconditioner M = diag(A).
 *
 * Multi-vectors are n x k, row-major (element (i, c) at index i*k + c, the
 * row-wise storage of Section 3.1). Each column is an independent system that
 * shares A: every dot product yields one scalar per column (Section 3.1.2), and
 * every column has its own alpha, omega, rho, stop test and status.
 *
 * Conventions for every function:
 *   - Pointers named d_* are DEVICE pointers on the device that was current
 *     when the handle was created. The library borrows them: it never frees
 *     or retains them beyond the call, except the matrix arrays, which must
 *     stay valid and unchanged (except through bicgstab_update_values) for the
 *     lifetime of the handle (or, for the values, until bicgstab_update_values
 *     hands the handle another array).
 *   - Work is enqueued on the handle's HIP stream. bicgstab_solve* return after
 *     the stream has finished the solve (they synchronise the stream).
 *   - Return value: BICGSTAB_OK (0) or a negative error code; a failed call
 *     leaves the handle usable. bicgstab_last_error() gives a message for the
 *     last failure on the calling thread.
 *   - A numerical breakdown is NOT an error: it is reported per column in
 *     bicgstab_info.status.
 *   - Handles are not thread-safe; one handle must not be used from two
 *     threads at once.
 */
#ifndef BICGSTAB_H
#define BICGSTAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BICGSTAB_MAX_K 64 /* maximum number of right-hand sides per handle */

/* Error codes. */
enum {
  BICGSTAB_OK = 0,
  BICGSTAB_EINVAL = -1,      /* invalid argument (shape, enum, zero diagonal for Jacobi, ...) */
  BICGSTAB_EHIP = -2,        /* a HIP runtime call failed */
  BICGSTAB_ENOMEM = -3,      /* workspace too small or allocation failed */
  BICGSTAB_EUNSUPPORTED = -4 /* valid but unsupported combination */
};

/* Methods (Appendix B). Improved BiCGStab (Alg. 3: one grouped reduction of
 * seven dot products per pass, f0 = A^T r0 formed once from a transposed CSR
 * built on the device) has no preconditioned form in the paper and runs in
 * FP64 only; other combinations return BICGSTAB_EUNSUPPORTED. */
enum { BICGSTAB_CLASSICAL = 0, BICGSTAB_REORDERED = 1, BICGSTAB_PIPELINED = 2, BICGSTAB_IMPROVED = 3 };
/* Formulations: merged = Table 2 "Merged" grouping, basic = Table 2 "Basic";
 * fused = the merged statements with the further fusions only a single device
 * allows: dot products formed in the sparse products' epilogues, the Jacobi
 * scaling written by the pass or product that makes its input, adjacent
 * passes of one scalar phase joined. With Jacobi the fused forms fold M^{-1}
 * into the products (A M^{-1} stored as a matrix, one more nnz x 8 bytes of
 * workspace; Alg. 5, 6 and 7 precondition from the right, so the iterates are
 * the listings' in exact arithmetic and differ from the merged form's by
 * rounding). Built for the classical, Reordered and
 * Pipelined methods; fused Improved returns BICGSTAB_EUNSUPPORTED. */
enum { BICGSTAB_MERGED = 0, BICGSTAB_BASIC = 1, BICGSTAB_FUSED = 2 };
/* Preconditioners: none, or Jacobi M = diag(A) applied as u / a_ii. */
enum { BICGSTAB_PRECOND_NONE = 0, BICGSTAB_PRECOND_JACOBI = 1 };
/* Precision: FP64 throughout, or FP32 matrix/Krylov vectors with FP64
 * scalars, FP64 dot accumulation and FP64 iterative refinement. */
enum { BICGSTAB_FP64 = 0, BICGSTAB_FP32_REFINE = 1 };

/* Per-column termination status. */
enum {
  BICGSTAB_COL_CONVERGED = 0, /* estimate of ||r||^2 below (tol*||b||)^2, or b = 0 */
  BICGSTAB_COL_MAXIT = 1,     /* maxit passes done */
  BICGSTAB_COL_BREAKDOWN = 2, /* a zero divisor (delta, rho, omega, alpha denominator) */
  BICGSTAB_COL_NONFINITE = 3  /* a NaN or Inf scalar */
};

/* A CSR matrix on the device: row_ptr has n+1 entries, row_ptr[0] = 0,
 * row_ptr[n] = nnz; col_idx and values have nnz entries; column indices of a
 * row need not be sorted but must lie in [0, n). values are double. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* d_row_ptr;
  const int32_t* d_col_idx;
  const double* d_values;
} bicgstab_csr;

/* Per-column results, HOST arrays of length k owned by the caller (any may be
 * NULL). relres_true = ||b - A x|| / ||b|| recomputed at exit; relres_recursive
 * = ||r|| / ||b|| of the recursively updated residual (both 0 when b = 0). */
typedef struct {
  int32_t* iters;
  int32_t* status;
  double* relres_true;
  double* relres_recursive;
} bicgstab_info;

typedef struct bicgstab_ctx* bicgstab_t;

/* Create a solver for A with k right-hand sides (1 <= k <= BICGSTAB_MAX_K).
 * Reads row_ptr and col_idx once (device to host) to validate the pattern
 * (malformed offsets or a column index out of range: BICGSTAB_EINVAL) and to
 * plan the sparse products; for a 3D grid pattern at k = 32 it also builds a
 * library-owned tile-ordered copy of A (nnz x 16 + n x 8 bytes of device
 * memory, nnz x 8 more for the fused forms with Jacobi, which also keep
 * A M^{-1} in that order; freed by bicgstab_destroy; see
 * bicgstab_product_layout). stream: a
 * hipStream_t (NULL = the null stream). The Jacobi diagonal is extracted at
 * the first solve; a zero diagonal entry then fails with BICGSTAB_EINVAL. */
int bicgstab_create(const bicgstab_csr* A, int64_t n, int32_t k, int32_t variant, int32_t formulation,
                    int32_t precond, int32_t precision, void* stream, bicgstab_t* out);

/* Device workspace the handle needs, in bytes (vectors n x k per Krylov
 * vector, the diagonal, reduction partials and per-column state). */
int bicgstab_workspace_bytes(bicgstab_t h, size_t* bytes);

/* Give the handle a caller-owned device workspace of at least
 * bicgstab_workspace_bytes() bytes (256-byte aligned). Without this call the
 * handle allocates its own at the first solve and frees it in destroy. */
int bicgstab_set_workspace(bicgstab_t h, void* d_ptr, size_t bytes);

/* Change the stream later work is enqueued on. */
int bicgstab_set_stream(bicgstab_t h, void* stream);

/* Solve A X = B. d_b: n x k right-hand sides (read only). d_x: n x k, the
 * initial guess on input and the solution on output. tol: per-column relative
 * tolerance, a column stops when its residual estimate satisfies
 * est < (tol * ||b_c||)^2; tol <= 0 disables the test (exactly maxit passes,
 * unless a breakdown). maxit >= 0. The solve polls the device for completion
 * every few iterations and returns when every column has stopped. */
int bicgstab_solve(bicgstab_t h, const double* d_b, double* d_x, double tol, int32_t maxit, bicgstab_info* info);

/* For callers that cannot allocate device memory (code that must not call
 * hipMalloc, such as tight serving loops or harnesses that forbid it):
 * bicgstab_solve with the same arguments, results and summation orders
 * (bitwise the same solution, counts and statuses), but the call allocates
 * nothing. Its workspace is a static device array of
 * BICGSTAB_NOALLOC_SCRATCH_BYTES inside the library, one per GPU (held from
 * when the library's device code is loaded on that GPU until the process
 * ends), instead of the handle's own workspace, which the call leaves
 * untouched. The handle's set-up data (diagonal, row-block list) is rebuilt
 * in the array at every call, and iterations are launched directly rather
 * than from captured graphs.
 *   - BICGSTAB_ENOMEM if bicgstab_workspace_bytes(h) exceeds the array.
 *   - BICGSTAB_EUNSUPPORTED for FP32-refinement handles and for Improved
 *     BiCGStab (it builds a transposed matrix, an allocation).
 *   - Every call on one GPU shares that GPU's array and finds the previous
 *     call's contents there: calls that overlap on one GPU (two threads, or
 *     two streams) race and must be serialised by the caller.
 *   - bicgstab_history reports no passes after this call. */
#define BICGSTAB_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int bicgstab_solve_noalloc(bicgstab_t h, const double* d_b, double* d_x, double tol, int32_t maxit,
                           bicgstab_info* info);

/* Solve A^T Lambda = G with the same method (the adjoint solve of the
 * gradient of x = A^{-1} b). Builds the transposed CSR on the device at the
 * first call. Same argument conventions as bicgstab_solve. */
int bicgstab_solve_transpose(bicgstab_t h, const double* d_g, double* d_lambda, double tol, int32_t maxit,
                             bicgstab_info* info);

/* Gradient of a loss with respect to the stored matrix values, given the
 * adjoint Lambda = A^{-T} dL/dX and the solution X (both n x k): for every
 * stored entry e = (i, j), d_grad[e] = - sum_c Lambda[i, c] * X[j, c]
 * (the derivative of A^{-1} B restricted to the sparsity pattern). */
int bicgstab_grad_values(bicgstab_t h, const double* d_lambda, const double* d_x, double* d_grad);

/* New matrix values, same sparsity pattern (the differentiation tier's
 * A(values)): d_values == NULL means the caller changed the values array the
 * handle borrows in place; otherwise the handle borrows d_values (nnz FP64
 * entries in the pattern's CSR order, device memory that must stay valid and
 * unchanged until the next update or the handle's end) instead of the array
 * given before. Refreshes what derives from the values on the handle's
 * stream (Jacobi diagonal, FP32 copy, transposed values); returns after it has
 * finished. A zero diagonal under Jacobi gives BICGSTAB_EINVAL (the handle
 * keeps the new values; update again before solving). */
int bicgstab_update_values(bicgstab_t h, const double* d_values);

/* Y = A X (n x k, row-major) with the solver's sparse-product kernel, on the
 * handle's stream, asynchronous. For kernel-level checks and timing. */
int bicgstab_spmm(bicgstab_t h, const double* d_x, double* d_y);

/* How the FP64 sparse products (Section 3.1's SpMM: the plain product, the
 * products with dot epilogues of the fused forms, and bicgstab_spmm) store A.
 * When the pattern is a 3D grid in natural order (x fastest) whose entries
 * couple each row only to rows one step away in x, y and z (7- and 27-point
 * stencils), k = 32 (row blocks of 32 rows) and the grid divides into
 * 2 x 4 x 4 tiles, create keeps a library-owned copy of A with its rows tile
 * by tile (one tile per row block): the tiles in the natural order of their
 * first grid point, the points of a tile in natural order within it (x
 * fastest). Each product writes every row of Y at its own index, and each
 * row's sum is bitwise that of the row order, with fewer row blocks sharing a
 * row's neighbours; the dot products of a product's epilogue add the rows in
 * the stored order (so a fused form's iterates follow the layout). The fused
 * forms with Jacobi keep A M^{-1} in the same order. tile = {tz, ty, tx},
 * grid = {nz, ny, nx}, all zero when A is stored row by row (other patterns,
 * other k, the FP32 tier, the environment variable BICGSTAB_SPMM_TILE=0 at
 * create). Either pointer may be NULL. */
int bicgstab_product_layout(bicgstab_t h, int32_t* tile, int32_t* grid);

/* Per-iteration history of the last solve: for iteration j < count and column
 * c, hist[(j*k + c)*4 + {0,1,2,3}] = alpha_j, omega_j, rho_j, stop estimate_j.
 * Call with hist = NULL to get the count; cap = entries of 4 doubles. */
int bicgstab_history(bicgstab_t h, double* hist, int32_t cap, int32_t* count);

/* FP32-refinement handles: for each column, the number of FP64 residual
 * corrections (inner FP32 solves) the last solve applied. outer: HOST array
 * of length k. */
int bicgstab_refine_outer(bicgstab_t h, int32_t* outer);

/* Iterations enqueued (whole captured chunks), kernel launches (passes, the
 * products' run-partial sums and finalize kernels; a replayed graph counts
 * the kernels it holds) and device-to-host polls of the last solve. */
int bicgstab_last_solve_stats(bicgstab_t h, int32_t* iterations_enqueued, int32_t* launches, int32_t* polls);

/* Kernel-level timing: runs the start-up passes on (d_b, d_x) and then
 * `iters` iterations with the stop test off, on the handle's stream, recording
 * a HIP event before and after every launch. For each launch i of one
 * iteration (nsteps <= cap of them) returns kind (0 sparse product,
 * 1 preconditioner, 2 vector pass, 3 sparse product with a dot epilogue), op
 * (vector-pass id, epilogue id for kind 3, -1 otherwise), the
 * vector blocks it reads and writes, and its average duration in ms. d_x is
 * overwritten. FP64 handles only. */
int bicgstab_kernel_times(bicgstab_t h, const double* d_b, double* d_x, int32_t iters, int32_t cap, int32_t* kind,
                          int32_t* op, int32_t* nin, int32_t* nout, double* ms, int32_t* nsteps);

int bicgstab_destroy(bicgstab_t h);

/* ---- Batched tier ----------------------------------------------------------
 * Many independent systems A_s X_s = B_s, s = 0..nsys-1, each with its own
 * CSR matrix (sizes may differ widely) and k_s right-hand sides, solved by one
 * persistent kernel in one captured graph launch. Every system runs the
 * merged classical BiCGStab (Appendix B, Alg. 2; with Jacobi, Alg. 5 in its
 * fused form: the products read A M^{-1}, entries a_ij / a_jj, and the
 * solution update divides p and s by a_ii, as bicgstab_solve's fused
 * classical form does) on its own share of workgroups, with a barrier per
 * system between the phases of an iteration; the per-column scalars, stop
 * test and statuses are those of bicgstab_solve. The batched method is not in
 * the paper: the paper treats one system with several right-hand sides.
 *
 * The kernel variant (threads per workgroup, rows a thread handles per step
 * of a vector phase and of a sparse product, entries per step of a row
 * product; see bicgstab_batched_variant_info) and each system's share of workgroups come
 * from the handle's configuration: a starting guess at create, replaced by
 * bicgstab_batched_tune (timed trials on the caller's batch) or by
 * bicgstab_batched_set_config (e.g. a configuration saved from an earlier
 * tune). All workgroups of the launch must be resident on the device at once;
 * a grid beyond the variant's occupancy limit is rejected with
 * BICGSTAB_EUNSUPPORTED. A barrier that waits longer than 2 s aborts the whole
 * launch (every workgroup exits) and the solve returns BICGSTAB_EHIP.
 *
 * Per system, each dot product is summed in a fixed order: a 64-wide
 * wavefront holds floor(64 / k) rows of k lanes; per thread over its rows (a
 * stride of (block / 64) * floor(64 / k) rows through the workgroup's
 * contiguous chunk of ceil(n / share) rows), a pairwise tree over the row
 * slots of a wavefront (adjacent slots first, an odd last slot passed up
 * unpaired), the wavefronts in index order, then the workgroups in index
 * order. Results depend on the block size and the shares, not on the other
 * variant parameters, and repeat bit for bit. */
typedef struct bicgstab_batched_ctx* bicgstab_batched_t;

/* As[s]: the matrix of system s (1 <= n < 2^24, nnz < 2^29, n * k * 8 < 2^31;
 * pattern validated on the host, the arrays must outlive the handle); ks[s]
 * in [1, BICGSTAB_MAX_K]. nsys >= 1. variant: BICGSTAB_CLASSICAL (the other
 * methods: BICGSTAB_EUNSUPPORTED). precond: BICGSTAB_PRECOND_NONE, or
 * BICGSTAB_PRECOND_JACOBI for every system: create then forms each system's
 * diagonal and A M^{-1} on the device ((n + nnz) x 8 bytes per system,
 * library-owned, freed by bicgstab_batched_destroy; values changed after
 * create are not seen) and a zero diagonal entry fails with BICGSTAB_EINVAL.
 * Anything else: BICGSTAB_EINVAL. */
int bicgstab_batched_create(const bicgstab_csr* As, const int32_t* ks, int32_t nsys, int32_t variant,
                            int32_t precond, void* stream, bicgstab_batched_t* out);
/* Device workspace in bytes: six n_s x k_s Krylov blocks per system, the
 * reduction partials, barrier counters, descriptors and results. */
int bicgstab_batched_workspace_bytes(bicgstab_batched_t h, size_t* bytes);
/* Caller-owned workspace (256-byte aligned, at least the size above); without
 * it the handle allocates its own at the first solve. */
int bicgstab_batched_set_workspace(bicgstab_batched_t h, void* d_ptr, size_t bytes);
int bicgstab_batched_set_stream(bicgstab_batched_t h, void* stream);
/* d_b, d_x: HOST arrays of nsys DEVICE pointers; d_b[s], d_x[s] are n_s x k_s
 * row-major (x: initial guess in, solution out). tol, maxit as in
 * bicgstab_solve. info (may be NULL): host arrays of length sum_s k_s, the
 * columns of system 0 first. Synchronous. */
int bicgstab_batched_solve(bicgstab_batched_t h, const double* const* d_b, double* const* d_x, double tol,
                           int32_t maxit, bicgstab_info* info);
/* Autotuner: times the batch under every kernel variant at its full resident
 * capacity, then the best variant at half and (if half was faster) a quarter
 * of it; for each, the
 * shares are first proportional to measured work (bytes per pass x passes)
 * and then twice re-derived from a per-system time model fitted to the run
 * before (passes x (latency + bytes / (share x per-workgroup bandwidth)),
 * least squares; the smallest makespan whose shares fit the budget). Last,
 * the best allocation thinned: every share divided by 2, 4, 8 and 16 (at
 * least one workgroup each), stopping at the first thinning that is not
 * faster. Keeps the fastest configuration. d_x holds the initial guesses on input (restored
 * before every trial) and the solution of the chosen configuration on output.
 * best_ms: that configuration's kernel time (may be NULL). */
int bicgstab_batched_tune(bicgstab_batched_t h, const double* const* d_b, double* const* d_x, double tol,
                          int32_t maxit, double* best_ms);
/* Current configuration and the last solve's timings: variant, its threads per
 * workgroup (block), workgroups[s] = share of system s, last_ms = kernel time,
 * system_ms[s] = device wall time of system s (any pointer may be NULL; arrays
 * of length nsys). */
int bicgstab_batched_get_config(bicgstab_batched_t h, int32_t* variant, int32_t* block, int32_t* workgroups,
                                double* last_ms, double* system_ms);
/* Set the configuration (a variant index, workgroups[s] >= 1). */
int bicgstab_batched_set_config(bicgstab_batched_t h, int32_t variant, const int32_t* workgroups);
/* Host-only: parameters of kernel variant `variant` (0-based; an error past
 * the last one): threads per workgroup, rows a thread takes per step of a
 * vector phase, entries per pipelined step of a row product, rows per stage
 * of a sparse product's pipeline. Any pointer may be NULL. */
int bicgstab_batched_variant_info(int32_t variant, int32_t* block, int32_t* rows_per_step,
                                  int32_t* entries_per_step, int32_t* product_rows_per_step);
int bicgstab_batched_destroy(bicgstab_batched_t h);

/* The vector-update experiment of Section 2.1 (Table 1), which motivates
 * merging: with scalars a, b, c and device vectors x, y, z of length n,
 *   run 1: three passes  y = a x + b y;  z = b x + a z;  z = b y + c z
 *          (9n elements moved),
 *   run 2: one pass of the first two updates (5n elements),
 *   run 3: one pass of all three updates, the same values as run 1 (5n).
 * Each product and sum rounds as written (no contraction). y and z are
 * updated in place. The work is enqueued on `stream` (a hipStream_t, NULL =
 * the null stream) and the call returns without waiting, so the caller can
 * time it with events. BICGSTAB_EINVAL for a run outside 1-3 or a null
 * vector with n > 0. */
int bicgstab_axpby_tab1(int32_t run, int64_t n, double a, double b, double c, const double* d_x, double* d_y,
                        double* d_z, void* stream);

/* Host-only query of the launch plan of one iteration (no device needed):
 * vector block reads and writes of its vector-operation passes (the counting
 * of Table 2), preconditioner applications, sparse products and kernel
 * launches per iteration. Plans are the same for every k except the fused
 * Reordered form, which below k = 4 forms its four dots in a pass of its own
 * (one block read more); this query gives the plan for k >= 4. */
int bicgstab_plan_traffic(int32_t variant, int32_t formulation, int32_t precond, int32_t* reads, int32_t* writes,
                          int32_t* precond_apps, int32_t* spmms, int32_t* launches);

const char* bicgstab_strerror(int code);
const char* bicgstab_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BICGSTAB_H */
