// CSR sparse matrix times row-major n x k block (gfx950).
//
// CSR-stream layout: contiguous rows are grouped into row blocks whose CSR
// entries fit in LDS. A workgroup stages its block's column indices, values
// and row offsets with coalesced loads, then lane c of each group of kp lanes
// (kp = k rounded up to a power of two) computes Y[i, c] for its rows. A lane
// takes its rows two at a time and issues the X gathers of both (up to 16)
// before it adds any of them; the products of a row are added in entry order,
// the rounding of a plain sequential sum.
#include <algorithm>

#include "internal.hpp"

namespace bcg {

namespace {

__host__ __device__ inline int pad_k_(int k) {
  int kp = 1;
  while (kp < k) kp <<= 1;
  return kp;
}

// Workgroup size and rows per lane of the product for padded width kp: up to
// 2048 outputs and 256 rows per block. (Measured on the 128^3 stencil at
// k = 32: 1024-lane workgroups with two rows per lane, column tiling and an
// XCD-contiguous block order were all slower; in plain round-robin order the
// XCDs work on neighbouring rows at the same time and share X rows through
// the Infinity Cache.)
__host__ __device__ inline int spmm_block(int kp) { return 256; }
inline int spmm_rows_per_lane(int kp) { return kp >= 8 ? 8 : kp; }

template <class T, int KPL, int BS>
__global__ __launch_bounds__(BS) void spmm_kernel(SpmmMat A, const T* __restrict__ X, T* __restrict__ Y, int k,
                                                  const Globals* glob) {
  if (glob && glob->nrun == 0) return;
  const int L = blockIdx.x;
  extern __shared__ double s_mem[];
  T* s_val = reinterpret_cast<T*>(s_mem);
  T* s_red = s_val + A.nnz_cap;
  int* s_col = reinterpret_cast<int*>(s_red + BS);
  int* s_rp = s_col + A.nnz_cap;
  const int r0 = A.blk[L], r1 = A.blk[L + 1];
  const int e0 = A.row_ptr[r0], e1 = A.row_ptr[r1];
  const int ne = e1 - e0;
  const T* __restrict__ val = static_cast<const T*>(A.val);
  constexpr int kp = 1 << KPL;
  constexpr int rpp = BS >> KPL;
  const int c = threadIdx.x & (kp - 1);
  const int rsub = threadIdx.x >> KPL;
  if (ne <= A.nnz_cap) {
    for (int i = threadIdx.x; i < ne; i += BS) {
      s_col[i] = A.col[e0 + i];
      s_val[i] = val[e0 + i];
    }
    for (int i = threadIdx.x; i <= r1 - r0; i += BS) s_rp[i] = A.row_ptr[r0 + i] - e0;
    __syncthreads();
    if (c >= k) return;
    const int nr = r1 - r0;
    for (int r = rsub; r < nr; r += 2 * rpp) {
      const int rb = r + rpp;
      const bool has_b = rb < nr;
      const int ebA = s_rp[r], eeA = s_rp[r + 1];
      const int ebB = has_b ? s_rp[rb] : 0, eeB = has_b ? s_rp[rb + 1] : 0;
      const int len = max(eeA - ebA, eeB - ebB);
      T sumA = (T)0, sumB = (T)0;
      for (int o = 0; o < len; o += 8) {
        T aA[8], xA[8], aB[8], xB[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int ea = ebA + o + j;
          if (ea < eeA) {
            aA[j] = s_val[ea];
            xA[j] = X[(size_t)s_col[ea] * k + c];
          }
          const int eb = ebB + o + j;
          if (eb < eeB) {
            aB[j] = s_val[eb];
            xB[j] = X[(size_t)s_col[eb] * k + c];
          }
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (ebA + o + j < eeA) sumA += aA[j] * xA[j];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (ebB + o + j < eeB) sumB += aB[j] * xB[j];
      }
      Y[(size_t)(r0 + r) * k + c] = sumA;
      if (has_b) Y[(size_t)(r0 + rb) * k + c] = sumB;
    }
  } else {
    // one long row (r1 == r0 + 1): lanes of the same column split its entries
    // and their sums are added in lane order
    T sum = (T)0;
    for (int base = 0; base < ne; base += A.nnz_cap) {
      const int m = min(A.nnz_cap, ne - base);
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += BS) {
        s_col[i] = A.col[e0 + base + i];
        s_val[i] = val[e0 + base + i];
      }
      __syncthreads();
      if (c < k)
        for (int e = rsub; e < m; e += rpp) sum += s_val[e] * X[(size_t)s_col[e] * k + c];
    }
    s_red[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x < kp && c < k) {
      T s = (T)0;
      for (int g = 0; g < rpp; ++g) s += s_red[g * kp + c];
      Y[(size_t)r0 * k + c] = s;
    }
  }
}

template <class T, int BS>
hipError_t spmm_launch_bs(const SpmmMat& A, const T* x, T* y, int k, const Globals* glob, hipStream_t s) {
  const int kp = pad_k_(k);
  const unsigned grid = (unsigned)A.nblk;
  const size_t lds = (size_t)A.nnz_cap * sizeof(T) + (size_t)BS * sizeof(T) + (size_t)A.nnz_cap * 4 +
                     (size_t)(A.rows_cap + 1) * 4 + 16;
  switch (kp) {
#define SPMM_CASE(KP, KPL) \
  case KP: hipLaunchKernelGGL((spmm_kernel<T, KPL, BS>), dim3(grid), dim3(BS), lds, s, A, x, y, k, glob); break;
    SPMM_CASE(1, 0)
    SPMM_CASE(2, 1)
    SPMM_CASE(4, 2)
    SPMM_CASE(8, 3)
    SPMM_CASE(16, 4)
    SPMM_CASE(32, 5)
    SPMM_CASE(64, 6)
#undef SPMM_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t spmm_dispatch(const SpmmMat& A, const void* X, void* Y, int k, const Globals* glob, hipStream_t s) {
  const T* x = static_cast<const T*>(X);
  T* y = static_cast<T*>(Y);
  if (spmm_block(pad_k_(k)) == 256) return spmm_launch_bs<T, 256>(A, x, y, k, glob, s);
  return spmm_launch_bs<T, 1024>(A, x, y, k, glob, s);
}

}  // namespace

// Row blocks: contiguous rows, block size x rows-per-lane / kp rows at most,
// and no more than kSpmmNnzMax entries unless a single row is longer (that row
// gets a block of its own, processed in chunks). Also returns the LDS extent
// every launch needs: the largest block's staged entries and rows.
SpmmPartition spmm_partition(const std::vector<int32_t>& row_ptr, int k, int rows_per_lane_override) {
  const int n = (int)row_ptr.size() - 1;
  const int kp = pad_k_(k);
  const int rpl = rows_per_lane_override > 0 ? rows_per_lane_override : spmm_rows_per_lane(kp);
  int rows_target = spmm_block(kp) * rpl / kp;
  if (rows_target > kSpmmRowsMax) rows_target = kSpmmRowsMax;
  if (rows_target < 1) rows_target = 1;
  SpmmPartition P;
  P.blk.push_back(0);
  P.nnz_cap = 1;
  P.rows_cap = 1;
  int r0 = 0;
  while (r0 < n) {
    int r = r0 + 1;  // always take at least one row
    while (r < n && r - r0 < rows_target && row_ptr[r + 1] - row_ptr[r0] <= kSpmmNnzMax) ++r;
    P.blk.push_back(r);
    const int ne = row_ptr[r] - row_ptr[r0];
    P.nnz_cap = std::max(P.nnz_cap, std::min(ne, kSpmmNnzMax));
    P.rows_cap = std::max(P.rows_cap, r - r0);
    r0 = r;
  }
  return P;
}

hipError_t launch_spmm(const SpmmMat& A, const void* X, void* Y, int k, bool fp32, const Globals* glob,
                       hipStream_t s) {
  if (A.nblk <= 0) return hipSuccess;
  return fp32 ? spmm_dispatch<float>(A, X, Y, k, glob, s) : spmm_dispatch<double>(A, X, Y, k, glob, s);
}

}  // namespace bcg
