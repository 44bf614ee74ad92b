// CSR sparse matrix times row-major n x k block (gfx950).
//
// CSR-stream layout: contiguous rows are grouped into row blocks whose CSR
// entries fit in LDS. A workgroup stages its block's column indices, values
// and row offsets with coalesced loads, then each group of kp / CPL lanes
// (kp = k rounded up to a power of two) computes the k outputs of one row,
// CPL adjacent columns per lane. Where k allows, a lane's columns fill one
// 16-byte gather per entry (two FP64 or four FP32 columns) instead of several
// narrower ones, which cuts the gather instructions and measured 15-25% faster
// on the 128^3 stencil at k = 4..32 (FP64, two columns); such a lane takes its
// rows one at a time. With one column (odd k) a lane takes its rows two at a
// time and issues the gathers of both before it adds any.
// Either way the products of a row are added in entry order, the rounding of a
// plain sequential sum. Two forms of the inner loop: the plain product guards
// each slot and reads a product's value with its column index (STYLE 0); the
// product with a dot epilogue uses branch-free slots with 32-bit gather offsets
// (STYLE 1), which keeps its register count, and so the workgroups in flight
// per compute unit, up. Output rows are written with nontemporal stores: the
// block is far larger than the caches and is read back only by a later pass.
//
// The same row-block body serves the sparse product with a dot epilogue
// (beyond the paper's grouping: dots of the written rows formed in the
// product): each workgroup stores its per-column partial sums block-major,
// a second kernel sums them over runs of blocks, and the finalize kernel sums
// the runs, every sum in a fixed order.
#include <algorithm>
#include <initializer_list>

#include "internal.hpp"
#include "reduce.hpp"

namespace bcg {

namespace {

__host__ __device__ inline int pad_k_(int k) {
  int kp = 1;
  while (kp < k) kp <<= 1;
  return kp;
}

// Workgroup size, columns per lane and rows per lane of the product: even k
// takes two columns per lane and two rows per lane (1024 outputs per block);
// odd k one column and up to eight rows per lane. (Measured on the 128^3
// stencil: 512- and 1024-lane workgroups, four or eight rows per lane at
// CPL = 2, and column tiling were slower.)
constexpr int kSpmmBlock = 256;
inline int spmm_cols_per_lane(int k) { return (k % 2 == 0) ? 2 : 1; }
inline int spmm_rows_per_lane(int k) {
  const int kp = pad_k_(k);
  return spmm_cols_per_lane(k) == 2 ? 2 : (kp >= 8 ? 8 : kp);
}

// Row block of workgroup w. Workgroups are dealt to the 8 XCDs in turn
// (XCD = w mod 8); with C > 1, runs of C consecutive row blocks go to one XCD,
// so rows a few blocks apart (the neighbours of a stencil row) meet in the
// same L2. A bijection of [0, nblk): the tail beyond a multiple of 8C keeps
// the plain order.
__device__ __forceinline__ int block_of(int w, int nblk, int C) {
  if (C <= 1) return w;
  const int full = nblk / (8 * C) * (8 * C);
  if (w >= full) return w;
  const int x = w & 7, q = w >> 3;
  return ((q / C) * 8 + x) * C + (q % C);
}

typedef __attribute__((address_space(1))) const char gcchar;

// Element (j, c) of the row-major block X: through a 32-bit byte offset from
// the uniform base when the whole block is below 4 GiB (OFF32), else 64-bit.
template <class T, bool OFF32>
__device__ __forceinline__ T load_x(const T* X, int j, int k, int c) {
  if constexpr (OFF32) {
    const unsigned off = ((unsigned)j * (unsigned)k + (unsigned)c) * (unsigned)sizeof(T);
    return *(const __attribute__((address_space(1))) T*)((gcchar*)X + off);
  } else {
    return X[(size_t)j * k + c];
  }
}

template <class T, int N>
struct VecOf {
  typedef T type __attribute__((ext_vector_type(N)));
};

// Elements (j, c) .. (j, c + N - 1) of X in one load (c a multiple of N, k a
// multiple of N, X aligned to N elements).
template <class T, int N, bool OFF32>
__device__ __forceinline__ typename VecOf<T, N>::type load_xv(const T* X, int j, int k, int c) {
  typedef typename VecOf<T, N>::type V;
  if constexpr (OFF32) {
    const unsigned off = ((unsigned)j * (unsigned)k + (unsigned)c) * (unsigned)sizeof(T);
    return *(const __attribute__((address_space(1))) V*)((gcchar*)X + off);
  } else {
    return *(const V*)(X + (size_t)j * k + c);
  }
}

// Row `row`, columns c .. c + CPL - 1 of Y, nontemporal.
template <class T, int CPL>
__device__ __forceinline__ void store_y(T* Y, int row, int k, int c, const T (&v)[CPL]) {
  if constexpr (CPL == 1) {
    __builtin_nontemporal_store(v[0], Y + (size_t)row * k + c);
  } else {
    typename VecOf<T, CPL>::type t;
#pragma unroll
    for (int h = 0; h < CPL; ++h) t[h] = v[h];
    __builtin_nontemporal_store(t, (typename VecOf<T, CPL>::type*)(Y + (size_t)row * k + c));
  }
}

struct NoEpilogue {
  template <class T, int CPL>
  __device__ __forceinline__ void operator()(int, const T (&)[CPL]) {}
};

// Dots of the written rows against W (E_DOT_W: (y, w); E_PPT: (y, w), (y, y),
// (w, w)), per lane in the order the lane writes its rows.
// The product's epilogue on each finished row: the dots of the row against
// W (E_DOT_W: (y, w); E_PPT: (y, w), (y, y), (w, w)), acc[d * CPL + h]
// holding dot d of column c + h, and / or the Jacobi-scaled copy
// Yh = y / a_ii (E_PREC, E_DOT_W_PREC).
template <class T, int EPI, int CPL>
struct DotEpilogue {
  const T* W;
  T* Yh;
  const T* diag;
  const T* X;  // the product's input, read at the row itself for E_RE4
  int k, c;
  double acc[kMaxEpilogueDots * CPL];
  __device__ __forceinline__ void operator()(int row, const T (&y)[CPL]) {
    if constexpr (epilogue_prec(EPI)) {
      const T d = diag[row];
      T yh[CPL];
#pragma unroll
      for (int h = 0; h < CPL; ++h) yh[h] = y[h] / d;
      store_y<T, CPL>(Yh, row, k, c, yh);
    }
    if constexpr (epilogue_dots(EPI) > 0) {
      // the epilogue's operand block is read once: nontemporal, as in the
      // vector passes
      T w[CPL];
      if constexpr (CPL == 1) {
        w[0] = __builtin_nontemporal_load(W + (size_t)row * k + c);
      } else {
        const typename VecOf<T, CPL>::type t =
            __builtin_nontemporal_load((const typename VecOf<T, CPL>::type*)(W + (size_t)row * k + c));
#pragma unroll
        for (int h = 0; h < CPL; ++h) w[h] = t[h];
      }
      if constexpr (EPI == E_RE4) {
        // x at the row itself: the product has just gathered it, so an
        // ordinary load (served by the caches)
        T xv[CPL];
        if constexpr (CPL == 1) {
          xv[0] = X[(size_t)row * k + c];
        } else {
          const typename VecOf<T, CPL>::type t = *(const typename VecOf<T, CPL>::type*)(X + (size_t)row * k + c);
#pragma unroll
          for (int h = 0; h < CPL; ++h) xv[h] = t[h];
        }
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
          const double yv = (double)y[h], xx = (double)xv[h], wv = (double)w[h];
          acc[h] += yv * xx;
          acc[CPL + h] += yv * yv;
          acc[2 * CPL + h] += yv * wv;
          acc[3 * CPL + h] += xx * xx;
        }
      } else {
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
          const double yv = (double)y[h];
          const double wv = (double)w[h];
          acc[h] += yv * wv;
          if (EPI == E_PPT) {
            acc[CPL + h] += yv * yv;
            acc[2 * CPL + h] += wv * wv;
          }
        }
      }
    }
  }
};

// Y rows of row block L; every finished row (its own row index, its CPL values)
// goes to epi, in the stored order (the block's dot partials follow it).
// KPL = log2(kp); lane c0 = (lane mod (kp / CPL)) * CPL holds columns c0 ..
// c0 + CPL - 1 (all below k, or all at or above it: CPL divides k).
template <class T, int KPL, int CPL, int BS, bool OFF32, int STYLE, class Epi>
__device__ __forceinline__ void row_block(const SpmmMat& A, const T* __restrict__ X, T* __restrict__ Y, int k, int L,
                                          Epi& epi) {
  extern __shared__ double s_mem[];
  T* s_val = reinterpret_cast<T*>(s_mem);
  T* s_red = s_val + A.nnz_cap;
  int* s_col = reinterpret_cast<int*>(s_red + CPL * BS);
  int* s_rp = s_col + A.nnz_cap;
  int* s_map = s_rp + A.rows_cap + 1;  // rows of Y when the stored rows are permuted
  const int r0 = A.blk[L], r1 = A.blk[L + 1];
  const int e0 = A.row_ptr[r0], e1 = A.row_ptr[r1];
  const int ne = e1 - e0;
  const T* __restrict__ val = static_cast<const T*>(A.val);
  constexpr int LPL = KPL - (CPL == 4 ? 2 : CPL == 2 ? 1 : 0);  // log2 of the lanes per row
  constexpr int lpr = 1 << LPL;
  constexpr int rpp = BS >> LPL;                  // rows per pass of the workgroup
  const int c = (threadIdx.x & (lpr - 1)) * CPL;
  const int rsub = threadIdx.x >> LPL;
  if (ne <= A.nnz_cap) {
    for (int i = threadIdx.x; i < ne; i += BS) {
      s_col[i] = A.col[e0 + i];
      s_val[i] = val[e0 + i];
    }
    for (int i = threadIdx.x; i <= r1 - r0; i += BS) s_rp[i] = A.row_ptr[r0 + i] - e0;
    // the Y row of each staged row (its own index unless the rows are stored
    // permuted): staged always, so the row loop carries no branch on it
    const int32_t* __restrict__ rmap = A.rowmap;
    for (int i = threadIdx.x; i < r1 - r0; i += BS) s_map[i] = rmap ? rmap[r0 + i] : r0 + i;
    __syncthreads();
    if (c >= k) return;
    const int nr = r1 - r0;
    auto yrow = [&](int r) { return s_map[r]; };
    if constexpr (CPL > 1) {
      typedef typename VecOf<T, CPL>::type V;
      for (int r = rsub; r < nr; r += rpp) {
        const int eb = s_rp[r], ee = s_rp[r + 1];
        T sv[CPL];
#pragma unroll
        for (int h = 0; h < CPL; ++h) sv[h] = (T)0;
        if constexpr (STYLE == 0) {
          for (int o = eb; o < ee; o += 8) {
            T av[8];
            V xv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (o + j < ee) {
                av[j] = s_val[o + j];
                xv[j] = load_xv<T, CPL, OFF32>(X, s_col[o + j], k, c);
              }
#pragma unroll
            for (int j = 0; j < 8; ++j)
              if (o + j < ee)
#pragma unroll
                for (int h = 0; h < CPL; ++h) sv[h] += av[j] * xv[j][h];
          }
        } else {
          // branch-free: a slot past the row's end gathers row 0 of X and is
          // not added (a select)
          const int last = max(ee - 1, 0);
          for (int o = eb; o < ee; o += 8) {
            V xv[8];
#pragma unroll
            for (int j = 0; j < 8; ++j)
              xv[j] = load_xv<T, CPL, OFF32>(X, o + j < ee ? s_col[min(o + j, last)] : 0, k, c);
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const T a = s_val[min(o + j, last)];
#pragma unroll
              for (int h = 0; h < CPL; ++h) {
                const T t = sv[h] + a * xv[j][h];
                sv[h] = o + j < ee ? t : sv[h];
              }
            }
          }
        }
        store_y<T, CPL>(Y, yrow(r), k, c, sv);
        epi(yrow(r), sv);
      }
    } else {
      for (int r = rsub; r < nr; r += 2 * rpp) {
        const int rb = r + rpp;
        const bool has_b = rb < nr;
        const int ebA = s_rp[r], eeA = s_rp[r + 1];
        const int ebB = has_b ? s_rp[rb] : 0, eeB = has_b ? s_rp[rb + 1] : 0;
        const int len = max(eeA - ebA, eeB - ebB);
        T sumA = (T)0, sumB = (T)0;
        if constexpr (STYLE == 0) {
          // guarded slots, the value of a product read with its column index
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
        } else {
          // Branch-free: a slot past its row's end gathers row 0 of X (always a
          // valid address) and its product is not added (a select, so the sums
          // are those of the entries alone, in order). Every gather of the step
          // is then in flight before the first is used.
          const int lastA = max(eeA - 1, 0), lastB = max(eeB - 1, 0);
          for (int o = 0; o < len; o += 8) {
            T xA[8], xB[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int ea = ebA + o + j, eb = ebB + o + j;
              const int ja = ea < eeA ? s_col[min(ea, lastA)] : 0;
              const int jb = eb < eeB ? s_col[min(eb, lastB)] : 0;
              xA[j] = load_x<T, OFF32>(X, ja, k, c);
              xB[j] = load_x<T, OFF32>(X, jb, k, c);
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int ea = ebA + o + j;
              const T t = sumA + s_val[min(ea, lastA)] * xA[j];
              sumA = ea < eeA ? t : sumA;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
              const int eb = ebB + o + j;
              const T t = sumB + s_val[min(eb, lastB)] * xB[j];
              sumB = eb < eeB ? t : sumB;
            }
          }
        }
        const T outA[1] = {sumA};
        store_y<T, 1>(Y, yrow(r), k, c, outA);
        epi(yrow(r), outA);
        if (has_b) {
          const T outB[1] = {sumB};
          store_y<T, 1>(Y, yrow(rb), k, c, outB);
          epi(yrow(rb), outB);
        }
      }
    }
  } else {
    // one long row (r1 == r0 + 1): lanes of the same columns split its entries
    // and their sums are added in lane order (its Y row staged like the rows of
    // a block; the barriers below order the store before its use)
    if (threadIdx.x == 0) s_map[0] = A.rowmap ? A.rowmap[r0] : r0;
    T sum[CPL];
#pragma unroll
    for (int h = 0; h < CPL; ++h) sum[h] = (T)0;
    for (int base = 0; base < ne; base += A.nnz_cap) {
      const int m = min(A.nnz_cap, ne - base);
      __syncthreads();
      for (int i = threadIdx.x; i < m; i += BS) {
        s_col[i] = A.col[e0 + base + i];
        s_val[i] = val[e0 + base + i];
      }
      __syncthreads();
      if (c < k)
        for (int e = rsub; e < m; e += rpp) {
          if constexpr (CPL > 1) {
            const typename VecOf<T, CPL>::type xv = load_xv<T, CPL, OFF32>(X, s_col[e], k, c);
#pragma unroll
            for (int h = 0; h < CPL; ++h) sum[h] += s_val[e] * xv[h];
          } else {
            sum[0] += s_val[e] * load_x<T, OFF32>(X, s_col[e], k, c);
          }
        }
    }
#pragma unroll
    for (int h = 0; h < CPL; ++h) s_red[h * BS + threadIdx.x] = sum[h];
    __syncthreads();
    if (threadIdx.x < lpr && c < k) {
      T out[CPL];
#pragma unroll
      for (int h = 0; h < CPL; ++h) {
        T v = (T)0;
        for (int g = 0; g < rpp; ++g) v += s_red[h * BS + g * lpr + threadIdx.x];
        out[h] = v;
      }
      store_y<T, CPL>(Y, s_map[0], k, c, out);
      epi(s_map[0], out);
    }
  }
}

template <class T, int KPL, int CPL, int BS, bool OFF32, int STYLE>
__global__ __launch_bounds__(BS) void spmm_kernel(SpmmMat A, const T* __restrict__ X, T* __restrict__ Y, int k,
                                                  const Globals* glob) {
  if (glob && glob->nrun == 0) return;
  NoEpilogue none;
  row_block<T, KPL, CPL, BS, OFF32, STYLE>(A, X, Y, k, block_of(blockIdx.x, A.nblk, A.xcd_chunk), none);
}

// The product with an epilogue: one workgroup per row block, as the plain
// product; the block's ND x k partial sums (if the epilogue forms dots) go to
// bpart[L * P + d * k + c] (block-major, P = ND * k).
template <class T, int KPL, int CPL, int BS, bool OFF32, int STYLE, int EPI>
__global__ __launch_bounds__(BS) void spmm_dot_kernel(SpmmMat A, const T* __restrict__ X, T* __restrict__ Y,
                                                      const T* __restrict__ W, T* __restrict__ Yh,
                                                      const T* __restrict__ diag, int k, double* __restrict__ bpart,
                                                      const Globals* glob) {
  if (glob && glob->nrun == 0) return;
  constexpr int ND = epilogue_dots(EPI);
  constexpr int LPL = KPL - (CPL == 4 ? 2 : CPL == 2 ? 1 : 0);
  const int L = block_of(blockIdx.x, A.nblk, A.xcd_chunk);
  DotEpilogue<T, EPI, CPL> epi{W, Yh, diag, X, k, (int)(threadIdx.x & ((1 << LPL) - 1)) * CPL, {}};
  row_block<T, KPL, CPL, BS, OFF32, STYLE>(A, X, Y, k, L, epi);
  // lanes past k returned from the row loop with their sums still zero
  if constexpr (ND > 0) store_block_partials_strided<ND, BS, CPL>(epi.acc, bpart + (size_t)L * ND * k, k, LPL, 1);
}

// Sums the block-major partials of nb row blocks over G runs of consecutive
// blocks: out[p * G + g] = sum of bpart[b * P + p] for b in run g, in block
// order; the finalize kernel then sums the G runs of each pair in run order.
// Each workgroup sums one run of row blocks, pair by pair, in block order.
// The run is staged through LDS in chunks that all 256 threads load (up to
// kRunLoads independent loads each), so the pass is not bound by the latency
// of one thread's chain of loads; thread p then adds the chunk's partials of
// pair p in block order, the same order as a plain loop over the run.
constexpr int kRunLoads = 24;
constexpr int kRunChunk = 256 * kRunLoads;  // doubles per chunk (48 KB)

__global__ __launch_bounds__(256) void reduce_runs_kernel(const double* __restrict__ bpart, int nb, int P,
                                                          double* __restrict__ out, int G, const Globals* glob) {
  if (glob && glob->nrun == 0) return;
  __shared__ double s_chunk[kRunChunk];
  const int g = blockIdx.x;
  const int t = threadIdx.x;
  const int b0 = (int)((long)nb * g / G), b1 = (int)((long)nb * (g + 1) / G);
  const int per = kRunChunk / P;  // whole blocks per chunk (P <= 256 by the launcher)
  double v = 0.0;
  for (int c0 = b0; c0 < b1; c0 += per) {
    const int nbk = min(per, b1 - c0);
    const int cnt = nbk * P;
    const double* src = bpart + (size_t)c0 * P;
    double tmp[kRunLoads];
#pragma unroll
    for (int j = 0; j < kRunLoads; ++j) {
      const int i = t + 256 * j;
      tmp[j] = i < cnt ? src[i] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kRunLoads; ++j) {
      const int i = t + 256 * j;
      if (i < cnt) s_chunk[i] = tmp[j];
    }
    __syncthreads();
    if (t < P)
      for (int j = 0; j < nbk; ++j) v += s_chunk[j * P + t];
    __syncthreads();
  }
  if (t < P) out[(size_t)t * G + g] = v;
}

template <class T, int CPL, int BS, bool OFF32, int STYLE>
hipError_t spmm_launch_bs(const SpmmMat& A, const T* x, T* y, int k, const Globals* glob, hipStream_t s) {
  const int kp = pad_k_(k);
  const unsigned grid = (unsigned)A.nblk;
  const size_t lds = (size_t)A.nnz_cap * sizeof(T) + (size_t)CPL * BS * sizeof(T) + (size_t)A.nnz_cap * 4 +
                     (size_t)(A.rows_cap + 1) * 4 + (size_t)A.rows_cap * 4 + 16;
  if (kp < CPL) return hipErrorInvalidValue;
  switch (kp) {
#define SPMM_CASE(KP, KPL)                                                                                         \
  case KP:                                                                                                         \
    hipLaunchKernelGGL((spmm_kernel<T, KPL, (KP >= CPL ? CPL : 1), BS, OFF32, STYLE>), dim3(grid), dim3(BS), lds, s, \
                       A, x, y, k, glob);                                                                          \
    break;
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

template <class T, int CPL, int BS, bool OFF32, int STYLE, int EPI>
hipError_t spmm_dot_launch(const SpmmMat& A, const T* x, T* y, const T* w, T* yh, const T* diag, int k, double* bpart,
                           const Globals* glob, hipStream_t s) {
  const int kp = pad_k_(k);
  const unsigned grid = (unsigned)A.nblk;
  const size_t lds = (size_t)A.nnz_cap * sizeof(T) + (size_t)CPL * BS * sizeof(T) + (size_t)A.nnz_cap * 4 +
                     (size_t)(A.rows_cap + 1) * 4 + (size_t)A.rows_cap * 4 + 16;
  if (kp < CPL) return hipErrorInvalidValue;
  switch (kp) {
#define SPMM_DOT_CASE(KP, KPL)                                                                                    \
  case KP:                                                                                                        \
    hipLaunchKernelGGL((spmm_dot_kernel<T, KPL, (KP >= CPL ? CPL : 1), BS, OFF32, STYLE, EPI>), dim3(grid), dim3(BS), \
                       lds, s, A, x, y, w, yh, diag, k, bpart, glob);                                             \
    break;
    SPMM_DOT_CASE(1, 0)
    SPMM_DOT_CASE(2, 1)
    SPMM_DOT_CASE(4, 2)
    SPMM_DOT_CASE(8, 3)
    SPMM_DOT_CASE(16, 4)
    SPMM_DOT_CASE(32, 5)
    SPMM_DOT_CASE(64, 6)
#undef SPMM_DOT_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// X block bytes below 4 GiB: 32-bit gather offsets.
inline bool off32(const SpmmMat& A, int k, size_t elem) { return (size_t)A.n * (size_t)k * elem < ((size_t)1 << 32); }

// Columns per lane of a launch: one 16-byte gather per entry where k and the
// operands' alignment allow it (two FP64 or four FP32 columns), else two
// FP32 columns (8 bytes), else one column; the sums are the same whichever.
template <class T>
int lane_cols(int k, std::initializer_list<const void*> ptrs) {
  auto aligned = [&](size_t a) {
    for (const void* p : ptrs)
      if (((uintptr_t)p % a) != 0) return false;
    return true;
  };
  if (sizeof(T) == 4 && k % 4 == 0 && aligned(16)) return 4;
  if (k % 2 == 0 && aligned(2 * sizeof(T))) return 2;
  return 1;
}

template <class T>
hipError_t spmm_dispatch(const SpmmMat& A, const void* X, void* Y, int k, const Globals* glob, hipStream_t s) {
  const T* x = static_cast<const T*>(X);
  T* y = static_cast<T*>(Y);
  switch (lane_cols<T>(k, {X, Y})) {
    case 4:
      if constexpr (sizeof(T) == 4) return spmm_launch_bs<T, 4, kSpmmBlock, false, 0>(A, x, y, k, glob, s);
      return hipErrorInvalidValue;
    case 2: return spmm_launch_bs<T, 2, kSpmmBlock, false, 0>(A, x, y, k, glob, s);
    default: return spmm_launch_bs<T, 1, kSpmmBlock, false, 0>(A, x, y, k, glob, s);
  }
}

template <class T, int CPL, int EPI>
hipError_t spmm_epi_launch(const SpmmMat& A, const T* x, T* y, const T* w, T* yh, const T* diag, int k,
                           double* bpart, const Globals* glob, hipStream_t s) {
  return off32(A, k, sizeof(T)) ? spmm_dot_launch<T, CPL, kSpmmBlock, true, 1, EPI>(A, x, y, w, yh, diag, k, bpart, glob, s)
                                : spmm_dot_launch<T, CPL, kSpmmBlock, false, 1, EPI>(A, x, y, w, yh, diag, k, bpart, glob,
                                                                                    s);
}

template <class T, int CPL>
hipError_t spmm_dot_dispatch_cpl(const SpmmMat& A, const T* x, T* y, const T* w, T* yh, const T* diag, int epi, int k,
                                 double* bpart, const Globals* glob, hipStream_t s) {
  switch (epi) {
    case E_DOT_W: return spmm_epi_launch<T, CPL, E_DOT_W>(A, x, y, w, yh, diag, k, bpart, glob, s);
    case E_PPT: return spmm_epi_launch<T, CPL, E_PPT>(A, x, y, w, yh, diag, k, bpart, glob, s);
    case E_PREC: return spmm_epi_launch<T, CPL, E_PREC>(A, x, y, w, yh, diag, k, bpart, glob, s);
    case E_DOT_W_PREC: return spmm_epi_launch<T, CPL, E_DOT_W_PREC>(A, x, y, w, yh, diag, k, bpart, glob, s);
    case E_RE4: return spmm_epi_launch<T, CPL, E_RE4>(A, x, y, w, yh, diag, k, bpart, glob, s);
    default: return hipErrorInvalidValue;
  }
}

template <class T>
hipError_t spmm_dot_dispatch(const SpmmMat& A, const void* X, void* Y, const void* W, void* Yh, const void* Diag,
                             int epi, int k, double* bpart, const Globals* glob, hipStream_t s) {
  const T* x = static_cast<const T*>(X);
  T* y = static_cast<T*>(Y);
  const T* w = static_cast<const T*>(W);
  T* yh = static_cast<T*>(Yh);
  const T* diag = static_cast<const T*>(Diag);
  switch (lane_cols<T>(k, {X, Y, W, Yh})) {
    case 4:
      if constexpr (sizeof(T) == 4) return spmm_dot_dispatch_cpl<T, 4>(A, x, y, w, yh, diag, epi, k, bpart, glob, s);
      return hipErrorInvalidValue;
    case 2: return spmm_dot_dispatch_cpl<T, 2>(A, x, y, w, yh, diag, epi, k, bpart, glob, s);
    default: return spmm_dot_dispatch_cpl<T, 1>(A, x, y, w, yh, diag, epi, k, bpart, glob, s);
  }
}

}  // namespace

// Row blocks: contiguous rows, block size x columns-per-lane x rows-per-lane
// / kp rows at most, and no more than kSpmmNnzMax entries unless a single row
// is longer (that row gets a block of its own, processed in chunks). Also returns the LDS extent
// every launch needs: the largest block's staged entries and rows.
SpmmPartition spmm_partition(const std::vector<int32_t>& row_ptr, int k, int rows_per_lane_override) {
  const int n = (int)row_ptr.size() - 1;
  const int kp = pad_k_(k);
  const int rpl = rows_per_lane_override > 0 ? rows_per_lane_override : spmm_rows_per_lane(k);
  int rows_target = kSpmmBlock * spmm_cols_per_lane(k) * rpl / kp;
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

int spmm_dot_runs(int nblk) { return std::max(1, std::min(nblk, 256)); }

hipError_t launch_spmm_dot(const SpmmMat& A, const void* X, void* Y, const void* W, void* Yh, const void* diag,
                           int epi, int k, bool fp32, const Ctl& ctl, int slot, int fin, double* bpart,
                           const Globals* glob, hipStream_t s, bool defer) {
  if (epi < 0 || epi >= E_NUM || (epilogue_dots(epi) > 0 && !W) || (epilogue_prec(epi) && (!Yh || !diag)))
    return hipErrorInvalidValue;
  const int P = epilogue_dots(epi) * k;
  if (P > 256) return hipErrorInvalidValue;  // one thread per pair in reduce_runs_kernel
  const int G = spmm_dot_runs(A.nblk);
  if (A.nblk > 0) {
    hipError_t e = fp32 ? spmm_dot_dispatch<float>(A, X, Y, W, Yh, diag, epi, k, bpart, glob, s)
                        : spmm_dot_dispatch<double>(A, X, Y, W, Yh, diag, epi, k, bpart, glob, s);
    if (e != hipSuccess) return e;
    if (P > 0) {
      hipLaunchKernelGGL(reduce_runs_kernel, dim3(G), dim3(256), 0, s, bpart, A.nblk, P, ctl.partials, G, glob);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (P == 0 && fin == F_NONE) return hipSuccess;
  if (defer) return hipSuccess;  // the run partials stay for the next pass
  // with no rows the partials are not written: the finalize then sums nothing
  return launch_finalize(ctl, A.nblk > 0 ? P : 0, G, slot, fin, glob != nullptr, s);
}

}  // namespace bcg
