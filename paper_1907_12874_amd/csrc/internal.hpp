// Internal definitions of the HIP library: the launchers of kernels.hip and
// spmm.hip, on top of the plan definitions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "plan.hpp"

namespace bcg {

// ---- device launchers (kernels.hip) ------------------------------------------
struct SpmmMat {
  const int32_t* row_ptr;
  const int32_t* col;
  const void* val;   // double or float
  const int32_t* blk;  // row-block starts, nblk + 1 entries
  int nblk;
  int n;
  int nnz_cap;   // entries staged in LDS per row block (largest block, <= kSpmmNnzMax)
  int rows_cap;  // rows of the largest row block
  int xcd_chunk; // consecutive row blocks given to one XCD (1: plain round-robin order)
  double* bpart; // per-row-block partial sums of a product with a dot epilogue (nblk x 3k)
  const int32_t* rowmap = nullptr;  // stored row i is row rowmap[i] of Y (nullptr: the same row)
};

struct SpmmPartition {
  std::vector<int32_t> blk;
  int nnz_cap;
  int rows_cap;
};

hipError_t launch_spmm(const SpmmMat& A, const void* X, void* Y, int k, bool fp32, const Globals* glob,
                       hipStream_t s);
// Sparse product with an epilogue (SpmmEpilogue epi): dot products against W
// (one workgroup per row block stores its partial sums in bpart, nblk x 3k
// doubles at most, a second kernel sums runs of blocks into ctl.partials, and
// the finalize kernel sums the runs and runs step `fin` on dot slots slot..)
// and/or the Jacobi-scaled copy Yh = Y / diag. glob: early exit when no
// column runs.
hipError_t launch_spmm_dot(const SpmmMat& A, const void* X, void* Y, const void* W, void* Yh, const void* diag,
                           int epi, int k, bool fp32, const Ctl& ctl, int slot, int fin, double* bpart,
                           const Globals* glob, hipStream_t s, bool defer = false);
// Runs of row blocks the epilogue partials are first summed over (<= 256).
int spmm_dot_runs(int nblk);
// The one-workgroup finalize kernel after a reduction pass of nb workgroups
// and P = ndot * k pairs.
hipError_t launch_finalize(const Ctl& ctl, int P, int nb, int slot, int fin, bool early, hipStream_t s);
hipError_t launch_prec(const void* in, void* out, const void* diag, int n, int k, bool fp32, const Globals* glob,
                       hipStream_t s);
// Workgroup-count caps of the vector passes: plain streaming passes and passes
// with dot products (both 256 lanes per workgroup). The dot cap also sizes the
// reduction partials buffer.
struct GridCaps {
  int blocks;
  int dot_blocks;
};
// A scalar step handed from a pass to the next one: the pass leaves its dot
// partials (pair-major, P pairs x nb) in `part` and launches no finalize
// kernel; every workgroup of the next pass sums them in the finalize
// kernel's order and runs the step itself, and its workgroup 0 stores the new
// state. Only steps whose inputs they do not overwrite qualify (F_ALPHA,
// F_OMEGA_MERGED, F_OMEGA_BASIC), so workgroups that read the state before or
// after workgroup 0 stores it take the same decisions.
struct Pending {
  const double* part;
  int fin, slot, P, nb;
};
bool op_takes_pending(int op);
// defer: leave the dot partials for the next pass (no finalize kernel)
hipError_t launch_group(int op, const void* const* in, void* const* out, const void* diag, int n, int k, int slot,
                        int fin, const Ctl& ctl, bool fp32, const GridCaps& caps, hipStream_t s,
                        const Pending* pending = nullptr, bool defer = false);
// Workgroups of a vector pass (its dot partials per pair).
int group_blocks(int op, int n, int k, const GridCaps& caps);
hipError_t launch_setup_state(const Ctl& ctl, double tol, int maxit, int hist_cap, hipStream_t s);
hipError_t launch_mark_maxit(const Ctl& ctl, hipStream_t s);
hipError_t launch_extract_diag(const int32_t* row_ptr, const int32_t* col, const double* val, double* diag,
                               float* diag32, int n, Globals* glob, hipStream_t s);
hipError_t launch_convert_f32(const double* in, float* out, int64_t count, hipStream_t s);
// a_ij / a_jj for every stored entry (Jacobi folded into the matrix), into
// out64 and / or out32
hipError_t launch_fold_jacobi(const int32_t* col, const double* val, const double* diag, double* out64, float* out32,
                              int64_t nnz, hipStream_t s);
// The three runs of Table 1's vector updates (1: three passes, 2: two updates
// merged, 3: three updates merged).
hipError_t launch_axpby(int run, const double* x, double* y, double* z, long n, double a, double b, double c,
                        hipStream_t s);
hipError_t launch_grad_values(const int32_t* row_ptr, const int32_t* col, const double* lam, const double* x,
                              double* grad, int n, int k, hipStream_t s);
hipError_t launch_transpose_count(const int32_t* col, int64_t nnz, int32_t* counts, hipStream_t s);
hipError_t launch_scan(const int32_t* counts, int32_t* row_ptr_t, int n, hipStream_t s);
hipError_t launch_transpose_fill(const int32_t* row_ptr, const int32_t* col, int n, const int32_t* row_ptr_t,
                                 int32_t* cursor, int32_t* col_t, int32_t* perm, hipStream_t s);
hipError_t launch_transpose_sort_rows(const int32_t* row_ptr_t, int32_t* col_t, int32_t* perm, int n, hipStream_t s);
hipError_t launch_gather_values(const double* val, const int32_t* perm, double* val_t, int64_t nnz, hipStream_t s);

// Row-block partition for the CSR-stream SpMM (host).
// rows_per_lane_override <= 0 picks the default for the width.
SpmmPartition spmm_partition(const std::vector<int32_t>& row_ptr, int k, int rows_per_lane_override);

// Records the message returned by bicgstab_last_error() on this thread and
// returns code.
int set_last_error(int code, const std::string& msg);

}  // namespace bcg
