// Per-workgroup partial sums of per-column dot products (device code shared
// by the vector passes and the sparse product's dot epilogue).
#pragma once

#include "internal.hpp"

namespace bcg {

// ND dot products per column; acc[d * CPL + h] holds this thread's running
// sum for column (lane mod 2^lpl) * CPL + h, 2^lpl lanes per row (CPL = 1:
// 2^lpl = kp). Fixed order: the row slots of a 64-wide wavefront by xor
// shuffles, then the wavefronts in index order. Pair t = d * k + c goes to
// out[t * stride].
template <int ND, int BS, int CPL = 1>
__device__ __forceinline__ void store_block_partials_strided(const double* acc, double* out, int k, int lpl,
                                                             size_t stride) {
  __shared__ double s_w[BS / 64][ND][kMaxK];
  const int lpr = 1 << lpl;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < ND; ++d)
#pragma unroll
    for (int h = 0; h < CPL; ++h) {
      double v = acc[d * CPL + h];
      for (int off = lpr; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
      if (lane < lpr && lane * CPL + h < kMaxK) s_w[wave][d][lane * CPL + h] = v;
    }
  __syncthreads();
  const int P = ND * k;
  for (int t = threadIdx.x; t < P; t += BS) {
    const int d = t / k, c = t - d * k;
    double v = s_w[0][d][c];
#pragma unroll
    for (int w = 1; w < BS / 64; ++w) v += s_w[w][d][c];
    out[(size_t)t * stride] = v;
  }
}

// Pair-major, partials[(d * k + c) * nb + b], for the finalize kernel.
template <int ND, int BS>
__device__ __forceinline__ void store_block_partials(const double* acc, double* partials, int k, int kpl, int nb,
                                                     int b) {
  store_block_partials_strided<ND, BS>(acc, partials + b, k, kpl, (size_t)nb);
}

}  // namespace bcg
