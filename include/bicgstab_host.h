/*
 * bicgstab_host.h -- C ABI of the host-CPU executor of the same BiCGStab
 * methods (libbicgstab_host.so).
 *
 * Purpose: the paper's measurement of merged against basic vector operations
 * was taken on CPU nodes (Section 3.1.3, Table 4). This executor runs the very
 * launch plans of the GPU library (one plan step = one memory pass over the
 * n x k blocks, grouped as in the Merged or Basic column of Table 2) on the
 * host's cores with OpenMP, so that comparison can be repeated on the host
 * next to the GPU, and it gives a multi-core CPU baseline. It is a separate
 * library with its own entry points: the GPU library never calls it and has
 * no CPU path of its own.
 *
 * Methods, formulations and preconditioners are those of bicgstab.h
 * (BICGSTAB_CLASSICAL ... BICGSTAB_IMPROVED, BICGSTAB_MERGED / BASIC / FUSED,
 * BICGSTAB_PRECOND_NONE / JACOBI), FP64 only; statuses and bicgstab_info are
 * the same. Every pointer here is a HOST pointer. Multi-vectors are n x k,
 * row-major (element (i, c) at i*k + c).
 *
 * Arithmetic: the per-element updates and the per-column scalar recurrences
 * are the GPU library's own (one shared source); sparse products sum each
 * row's entries in stored order; every dot product is summed over T fixed row
 * ranges [n t / T, n (t+1) / T), each range in row order, then the T range
 * sums in order (T = the threads argument), so a solve is bitwise repeatable
 * for a given T whatever OpenMP schedules.
 *
 * Return value: BICGSTAB_OK or a negative error code (bicgstab.h);
 * bicgstab_host_last_error() gives the message of the last failure on the
 * calling thread.
 */
#ifndef BICGSTAB_HOST_H
#define BICGSTAB_HOST_H

#include <stdint.h>

#include "bicgstab.h"

#ifdef __cplusplus
extern "C" {
#endif

/* A CSR matrix in host memory: row_ptr has n+1 entries (row_ptr[0] = 0,
 * row_ptr[n] = nnz), col_idx and values nnz entries, columns in [0, n). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
} bicgstab_host_csr;

typedef struct bicgstab_host_ctx* bicgstab_host_t;

/* Create a host solver for A with k right-hand sides (1 <= k <= 64). The
 * matrix is copied (the caller's arrays may be freed afterwards); the Jacobi
 * diagonal is extracted here and a zero diagonal entry fails with
 * BICGSTAB_EINVAL; Improved BiCGStab builds A^T here. threads >= 1 fixes the
 * number of row ranges (and OpenMP threads) of every pass. Unsupported
 * combinations (as in bicgstab_create) return BICGSTAB_EUNSUPPORTED. */
int bicgstab_host_create(const bicgstab_host_csr* A, int32_t k, int32_t variant, int32_t formulation,
                         int32_t precond, int32_t threads, bicgstab_host_t* out);

/* Solve A X = B from the initial guess in x (n x k, overwritten with the
 * solution); b is n x k. Stop rule, statuses and exit residuals as
 * bicgstab_solve. maxit <= 0 runs no pass (every column MAXIT). */
int bicgstab_host_solve(bicgstab_host_t h, const double* b, double* x, double tol, int32_t maxit,
                        bicgstab_info* info);

/* Wall time of the last solve's iteration loop (the passes only: set-up,
 * start-up passes and the exit residual excluded) and the passes it ran, for
 * per-iteration timing of fixed-pass solves (tol = 0). */
int bicgstab_host_loop_time(bicgstab_host_t h, double* seconds, int32_t* passes);

/* Table 1's vector updates (Section 2.1) on host vectors of length n, on
 * `threads` fixed row ranges: run 1 = three passes y = a x + b y,
 * z = b x + a z, z = b y + c z; run 2 = the first two updates in one pass;
 * run 3 = all three in one pass (the values of run 1). y, z updated in place;
 * synchronous. */
int bicgstab_host_axpby_tab1(int32_t run, int64_t n, double a, double b, double c, const double* x, double* y,
                             double* z, int32_t threads);

/* Release the solver (NULL is ignored). */
int bicgstab_host_destroy(bicgstab_host_t h);

/* Message of the last failed call on this thread ("" if none). */
const char* bicgstab_host_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BICGSTAB_HOST_H */
