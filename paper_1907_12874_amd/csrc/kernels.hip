// HIP kernels for gfx950 (CDNA4, wave64).
//
// Everything on the BiCGStab path is bound by HBM bandwidth (a sparse product
// and streaming vector passes of 0.1-0.75 flop per byte), so nothing here uses
// the matrix cores. The kernels are written for memory traffic:
//   * n x k blocks are row-major; a workgroup of 256 lanes covers 256/kp rows
//     x kp columns (kp = k rounded up to a power of two, at most 64), so each
//     load instruction of a wave reads whole contiguous rows;
//   * the sparse product stages a row block's CSR entries in LDS with
//     coalesced loads (a CSR-stream layout), then gathers X rows;
//   * a vector pass computes all its dot products (one per column) while it
//     streams, reduces them inside the wave with xor shuffles between lanes of
//     the same column and across waves through LDS, and stores one partial per
//     workgroup; a one-workgroup finalize kernel sums the partials in a fixed
//     order (results are bitwise repeatable) and runs the per-column scalar
//     recurrence, so no streaming workgroup needs a device-scope fence;
//   * all arithmetic is IEEE with no contraction (the library is built with
//     -ffp-contract=off) and Jacobi divides by a_ii, so the vector updates and
//     the products round exactly like a plain sequential evaluation.
#include <math.h>

#include <algorithm>

#include "internal.hpp"
#include "reduce.hpp"

namespace bcg {

// ------------------------------------------------------------------ helpers ---

// Block operands of the streaming passes are read with nontemporal loads:
// each element is used once per pass, and loads that do not claim cache lines
// leave the L2 and the Infinity Cache to data that is reused (the matrix and
// the gathered rows of the sparse products). Measured on the 128^3 workload:
// every vector pass 5-13% faster, 2.77 -> 2.58 ms per classical merged
// iteration at k = 32 and 0.217 -> 0.194 ms at k = 1.
template <class T>
__device__ __forceinline__ double ldv(const void* p, size_t e) {
  return (double)__builtin_nontemporal_load(static_cast<const T*>(p) + e);
}
// Outputs of the streaming passes are written with nontemporal stores: a
// block is read back only by a later pass, after far more data than the
// caches hold has gone through them (measured 3-6% faster at k = 32).
template <class T>
__device__ __forceinline__ void stv(void* p, size_t e, double v) {
  __builtin_nontemporal_store((T)v, static_cast<T*>(p) + e);
}

__device__ __forceinline__ int log2_pow2(int kp) { return 31 - __clz(kp); }

__host__ __device__ inline int pad_k(int k) {
  int kp = 1;
  while (kp < k) kp <<= 1;
  return kp;
}

}  // namespace bcg

#include "method.hpp"

namespace bcg {

// ---------------------------------------------------- cross-block reduction ---

struct GArgs {
  const void* in[kMaxPassIn];
  void* out[kMaxPassOut];
  const void* diag;  // a_ii (storage type) for USE_D ops
  long n;
  int k, kpl, slot, fin;
  Ctl ctl;
  Pending pend;  // a scalar step left by the previous pass (pend.fin = F_NONE: none)
};

// Dot products leave the streaming pass as one partial sum per workgroup and
// pair (dot d, column c), stored pair-major: partials[p * nb + b]. A separate
// one-workgroup finalize kernel then sums them and runs the scalar step: the
// kernel boundary orders the partial stores before their reads, so no
// workgroup of a pass needs a device-scope fence or atomic (on this
// multi-XCD part a device-scope release writes back the L2, and one per
// workgroup serialises the whole pass).
constexpr int kFinBlock = 1024;
constexpr int kFinLanes = 16;  // finalize lanes per (dot, column) pair

template <int ND, int BS>
__device__ __forceinline__ void block_reduce_store(const double* acc, const GArgs& a) {
  store_block_partials<ND, BS>(acc, a.ctl.partials, a.k, a.kpl, gridDim.x, blockIdx.x);
}

// One workgroup: sum the nb partials of each of the P pairs (lane g of the
// kFinLanes lanes of a pair sums workgroups g, g + kFinLanes, ... in order,
// then the lane sums are added in lane order), write the dot slots, run the
// finalize step. Every sum has a fixed order, so results are bitwise
// repeatable. The per-column state of the k columns and the globals are
// staged in LDS with one parallel load before the scalar step and stored back
// after it, so the step's chain of reads and writes of scalars costs LDS
// latency instead of one device-memory round trip per dependent access.
__global__ __launch_bounds__(kFinBlock) void finalize_kernel(Ctl ctl, int P, int nb, int slot, int fin, int early) {
  if (early && ctl.glob->nrun == 0) return;
  __shared__ double s_g[kFinBlock];
  __shared__ double s_sc[S_NSCAL * kMaxK];
  __shared__ int s_ist[I_NINT * kMaxK];
  __shared__ Globals s_glob;
  const int k = ctl.k;
  const int t = threadIdx.x;
  const bool step = fin != F_NONE;
  if (step) {
    for (int i = t; i < S_NSCAL * kMaxK; i += kFinBlock)
      if ((i & (kMaxK - 1)) < k) s_sc[i] = ctl.sc[i];
    for (int i = t; i < I_NINT * kMaxK; i += kFinBlock)
      if ((i & (kMaxK - 1)) < k) s_ist[i] = ctl.ist[i];
    if (t == 0) s_glob = *ctl.glob;
  }
  Ctl L = ctl;
  if (step) {
    L.sc = s_sc;
    L.ist = s_ist;
    L.glob = &s_glob;
  }
  if (P > 0) {
    // a fixed number of lanes per pair, whatever P: the summation order of a
    // dot product then depends only on the pass's grid, not on how many dots
    // the pass forms
    constexpr int G = kFinLanes;
    constexpr int PP = kFinBlock / G;  // pairs per round
    for (int p0 = 0; p0 < P; p0 += PP) {
      const int p = p0 + t / G, g = t % G;
      double v = 0.0;
      if (t < PP * G && p < P) {
        const double* q = ctl.partials + (size_t)p * nb;
#pragma unroll 8
        for (int b = g; b < nb; b += G) v += q[b];
      }
      s_g[t] = v;
      __syncthreads();
      if (t < PP && p0 + t < P) {
        double sum = 0.0;
        for (int j = 0; j < G; ++j) sum += s_g[t * G + j];
        const int pp = p0 + t, d = pp / k, c = pp - d * k;
        SC(L, S_D0 + slot + d, c) = sum;
      }
      __syncthreads();
    }
  }
  if (!step) return;
  __syncthreads();
  if (t < k) finalize_column(fin, t, L);
  __syncthreads();
  if (t == 0) finalize_global(fin, L);
  __syncthreads();
  for (int i = t; i < S_NSCAL * kMaxK; i += kFinBlock)
    if ((i & (kMaxK - 1)) < k) ctl.sc[i] = s_sc[i];
  for (int i = t; i < I_NINT * kMaxK; i += kFinBlock)
    if ((i & (kMaxK - 1)) < k) ctl.ist[i] = s_ist[i];
  if (t == 0) *ctl.glob = s_glob;
}

// ---------------------------------------------------------- group kernel ---

// The scalar step a pass took over from the pass before (Pending): every
// workgroup stages the k columns' state in LDS, sums the pending partials in
// the finalize kernel's order (kFinLanes lanes per pair, lane g over
// workgroups g, g + kFinLanes, ..., then the lanes in order), and runs the
// step on its LDS copy, whose scalars the pass then uses. Workgroup 0 stores
// the new state. The step must not overwrite its own inputs (it reads the
// state another workgroup may be storing at the same time): F_ALPHA,
// F_OMEGA_MERGED and F_OMEGA_BASIC write only alpha, omega, the estimate, a
// pending stop and (for a column that stops) its status, which every
// workgroup computes alike.
struct PendState {
  double sc[S_NSCAL * kMaxK];
  int ist[I_NINT * kMaxK];
  Globals glob;
  double red[kBlock];
};

template <int BS>
__device__ void take_pending(const GArgs& a, PendState& ps, Ctl& L) {
  const int k = a.k, t = threadIdx.x;
  for (int i = t; i < S_NSCAL * kMaxK; i += BS)
    if ((i & (kMaxK - 1)) < k) ps.sc[i] = a.ctl.sc[i];
  for (int i = t; i < I_NINT * kMaxK; i += BS)
    if ((i & (kMaxK - 1)) < k) ps.ist[i] = a.ctl.ist[i];
  if (t == 0) ps.glob = *a.ctl.glob;
  __syncthreads();
  L = a.ctl;
  L.sc = ps.sc;
  L.ist = ps.ist;
  L.glob = &ps.glob;
  constexpr int G = kFinLanes;
  constexpr int PP = BS / G;
  const int P = a.pend.P, nb = a.pend.nb;
  for (int p0 = 0; p0 < P; p0 += PP) {
    const int p = p0 + t / G, g = t % G;
    double v = 0.0;
    if (p < P) {
      const double* q = a.pend.part + (size_t)p * nb;
#pragma unroll 8
      for (int b = g; b < nb; b += G) v += q[b];
    }
    ps.red[t] = v;
    __syncthreads();
    if (t < PP && p0 + t < P) {
      double sum = 0.0;
      for (int j = 0; j < G; ++j) sum += ps.red[t * G + j];
      const int pp = p0 + t, d = pp / k, c = pp - d * k;
      SC(L, S_D0 + a.pend.slot + d, c) = sum;
    }
    __syncthreads();
  }
  if (t < k) finalize_column(a.pend.fin, t, L);
  __syncthreads();
  if (t == 0) finalize_global(a.pend.fin, L);
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int i = t; i < S_NSCAL * kMaxK; i += BS)
      if ((i & (kMaxK - 1)) < k) a.ctl.sc[i] = ps.sc[i];
    for (int i = t; i < I_NINT * kMaxK; i += BS)
      if ((i & (kMaxK - 1)) < k) a.ctl.ist[i] = ps.ist[i];
    if (t == 0) *a.ctl.glob = ps.glob;
  }
}

// The passes that take over a pending scalar step (those that follow an
// alpha or omega reduction in the plans).
template <class Op>
struct TakesPending {
  static constexpr bool value = false;
};
template <>
struct TakesPending<KSubAlpha> {
  static constexpr bool value = true;
};
template <>
struct TakesPending<KXUpd> {
  static constexpr bool value = true;
};
template <>
struct TakesPending<KCXrRho> {
  static constexpr bool value = true;
};
template <>
struct TakesPending<KFXrRhoD> {
  static constexpr bool value = true;
};

bool op_takes_pending(int op) {
  return op == OP_SUB_ALPHA || op == OP_XUPD || op == OP_C_XR_RHO || op == OP_F_XR_RHO_D;
}

template <class Op, class T, int U, int BS, bool PEND>
__global__ __launch_bounds__(BS) void group_kernel(GArgs a) {
  // A pass that takes a pending step has no early exit: its workgroup 0 may
  // store the running-column count while other workgroups start, so their
  // waves could read different counts; with no column running the step and
  // the pass do nothing anyway.
  if (!PEND && Op::EARLY && a.ctl.glob->nrun == 0) return;
  // the scalars this pass uses: the device state, or the LDS copy after a
  // pending scalar step
  __shared__ PendState ps;  // unused (and not allocated) without PEND
  Ctl cs = a.ctl;
  if constexpr (PEND) take_pending<BS>(a, ps, cs);
  const int kpl = a.kpl;
  const int kp = 1 << kpl;
  const int k = a.k;
  const int c = threadIdx.x & (kp - 1);
  bool on = c < k;
  if (on) {
    if (Op::PART == PART_RUN)
      on = IS(cs, I_STATUS, c) == ST_RUNNING;
    else if (Op::PART == PART_ZEROB)
      on = IS(cs, I_ZEROB, c) != 0;
  }
  constexpr int NI = Op::NIN + (Op::USE_D ? 1 : 0) > 0 ? Op::NIN + (Op::USE_D ? 1 : 0) : 1;
  constexpr int NO = Op::NOUT > 0 ? Op::NOUT : 1;
  constexpr int ND = Op::NDOT > 0 ? Op::NDOT : 1;
  double acc[ND];
#pragma unroll
  for (int d = 0; d < ND; ++d) acc[d] = 0.0;
  if (on) {
    Coef cf;
    cf.alpha = SC(cs, S_ALPHA, c);
    cf.omega = SC(cs, S_OMEGA, c);
    cf.beta = SC(cs, S_BETA, c);
    cf.scale = SC(cs, S_SCALE, c);
    cf.delta = SC(cs, S_DELTA, c);
    cf.c1 = SC(cs, S_C1, c);
    cf.c2 = SC(cs, S_C2, c);
    // outputs in COUT are written only where the column restarts
    const unsigned wmask = Op::COUT == 0u || IS(cs, I_RESTART, c) != 0 ? ~0u : ~Op::COUT;
    const int rpb = BS >> kpl;
    const long n = a.n;
    const long stride = (long)gridDim.x * rpb;
    long row = (long)blockIdx.x * rpb + (threadIdx.x >> kpl);
    for (; row + (U - 1) * stride < n; row += U * stride) {
      double v[U][NI];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = (size_t)(row + u * stride) * k + c;
#pragma unroll
        for (int i = 0; i < Op::NIN; ++i)
          v[u][i] = ((Op::XIN >> i) & 1) ? ldv<double>(a.in[i], e) : ldv<T>(a.in[i], e);
        if constexpr (Op::USE_D) v[u][Op::NIN] = ldv<T>(a.diag, (size_t)(row + u * stride));
      }
      // passes with dot products: keep every load of the step ahead of the
      // arithmetic (the scheduler otherwise sinks loads next to their use,
      // fewer registers but one memory latency per row instead of per step)
      if constexpr (Op::NDOT > 0) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const size_t e = (size_t)(row + u * stride) * k + c;
        double o[NO];
        Op::template f<T>(v[u], cf, o, acc);
#pragma unroll
        for (int j = 0; j < Op::NOUT; ++j) {
          if (!((wmask >> j) & 1)) continue;
          if ((Op::XOUT >> j) & 1)
            stv<double>(a.out[j], e, o[j]);
          else
            stv<T>(a.out[j], e, o[j]);
        }
      }
    }
    for (; row < n; row += stride) {
      const size_t e = (size_t)row * k + c;
      double v1[NI];
#pragma unroll
      for (int i = 0; i < Op::NIN; ++i) v1[i] = ((Op::XIN >> i) & 1) ? ldv<double>(a.in[i], e) : ldv<T>(a.in[i], e);
      if constexpr (Op::USE_D) v1[Op::NIN] = ldv<T>(a.diag, (size_t)row);
      double o[NO];
      Op::template f<T>(v1, cf, o, acc);
#pragma unroll
      for (int j = 0; j < Op::NOUT; ++j) {
        if (!((wmask >> j) & 1)) continue;
        if ((Op::XOUT >> j) & 1)
          stv<double>(a.out[j], e, o[j]);
        else
          stv<T>(a.out[j], e, o[j]);
      }
    }
  }
  if constexpr (Op::NDOT > 0) block_reduce_store<Op::NDOT, BS>(acc, a);
}

template <class Op>
int op_blocks(long n, int kpl, const GridCaps& caps) {
  const int cap = Op::NDOT > 0 ? caps.dot_blocks : caps.blocks;
  const int rpb = kBlock >> kpl;
  long blocks = (n + rpb - 1) / rpb;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  return (int)blocks;
}

template <class Op, class T>
hipError_t launch_op(const GArgs& a0, const GridCaps& caps, hipStream_t s, bool defer) {
  GArgs a = a0;
  constexpr int BS = kBlock;
  const int blocks = op_blocks<Op>(a.n, a.kpl, caps);
  constexpr int U = Op::NIN <= 4 ? 4 : 2;
  if (a.pend.fin != F_NONE) {
    if constexpr (TakesPending<Op>::value)
      hipLaunchKernelGGL((group_kernel<Op, T, U, BS, true>), dim3((unsigned)blocks), dim3(BS), 0, s, a);
    else
      return hipErrorInvalidValue;  // the host hands pending steps only to the passes above
  } else {
    hipLaunchKernelGGL((group_kernel<Op, T, U, BS, false>), dim3((unsigned)blocks), dim3(BS), 0, s, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (defer) return hipSuccess;  // the partials stay for the next pass
  if (Op::NDOT > 0 || a.fin != F_NONE) {
    hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinBlock), 0, s, a.ctl, Op::NDOT * a.k, (int)blocks, a.slot,
                       a.fin, Op::EARLY ? 1 : 0);
    e = hipGetLastError();
  }
  return e;
}

template <class T>
hipError_t dispatch_op(int op, const GArgs& a, const GridCaps& grid_cap, hipStream_t s, bool defer) {
  switch (op) {
    case OP_INIT: return launch_op<KInit, T>(a, grid_cap, s, defer);
    case OP_INIT_P: return launch_op<KInitP, T>(a, grid_cap, s, defer);
    case OP_ZEROB: return launch_op<KZeroB, T>(a, grid_cap, s, defer);
    case OP_COPY: return launch_op<KCopy, T>(a, grid_cap, s, defer);
    case OP_FILL0: return launch_op<KFill0, T>(a, grid_cap, s, defer);
    case OP_EXIT: return launch_op<KExit, T>(a, grid_cap, s, defer);
    case OP_DOT: return launch_op<KDot, T>(a, grid_cap, s, defer);
    case OP_DOTSELF: return launch_op<KDotSelf, T>(a, grid_cap, s, defer);
    case OP_SUB_ALPHA: return launch_op<KSubAlpha, T>(a, grid_cap, s, defer);
    case OP_SUB_OMEGA: return launch_op<KSubOmega, T>(a, grid_cap, s, defer);
    case OP_XUPD: return launch_op<KXUpd, T>(a, grid_cap, s, defer);
    case OP_PUPD: return launch_op<KPUpd, T>(a, grid_cap, s, defer);
    case OP_C_PPT: return launch_op<KCPpt, T>(a, grid_cap, s, defer);
    case OP_C_XR_RHO: return launch_op<KCXrRho, T>(a, grid_cap, s, defer);
    case OP_C_R_RHO: return launch_op<KCRRho, T>(a, grid_cap, s, defer);
    case OP_R_G3: return launch_op<KRG3, T>(a, grid_cap, s, defer);
    case OP_R_XZV: return launch_op<KRXzv, T>(a, grid_cap, s, defer);
    case OP_P_G1: return launch_op<KPG1, T>(a, grid_cap, s, defer);
    case OP_P_G2: return launch_op<KPG2, T>(a, grid_cap, s, defer);
    case OP_P_G3: return launch_op<KPG3, T>(a, grid_cap, s, defer);
    case OP_PP_G12: return launch_op<KPPG12, T>(a, grid_cap, s, defer);
    case OP_PP_G34: return launch_op<KPPG34, T>(a, grid_cap, s, defer);
    case OP_REF_RESID: return launch_op<KRefResid, T>(a, grid_cap, s, defer);
    case OP_REF_SCALE: return launch_op<KRefScale, T>(a, grid_cap, s, defer);
    case OP_REF_UPDATE: return launch_op<KRefUpdate, T>(a, grid_cap, s, defer);
    case OP_F_SUB_ALPHA_H: return launch_op<KFSubAlphaH, T>(a, grid_cap, s, defer);
    case OP_F_PUPD_H: return launch_op<KFPUpdH, T>(a, grid_cap, s, defer);
    case OP_F_XR_RHO_H: return launch_op<KFXrRhoH, T>(a, grid_cap, s, defer);
    case OP_IB_INIT: return launch_op<KIbInit, T>(a, grid_cap, s, defer);
    case OP_IB_G1: return launch_op<KIbG1, T>(a, grid_cap, s, defer);
    case OP_IB_G2: return launch_op<KIbG2, T>(a, grid_cap, s, defer);
    case OP_IB_G3: return launch_op<KIbG3, T>(a, grid_cap, s, defer);
    case OP_IB_Z: return launch_op<KIbZ, T>(a, grid_cap, s, defer);
    case OP_IB_V: return launch_op<KIbV, T>(a, grid_cap, s, defer);
    case OP_IB_X: return launch_op<KIbX, T>(a, grid_cap, s, defer);
    case OP_RE_R: return launch_op<KReR, T>(a, grid_cap, s, defer);
    case OP_F_XR_RHO_D: return launch_op<KFXrRhoD, T>(a, grid_cap, s, defer);
    case OP_F_P_G23: return launch_op<KFPG23, T>(a, grid_cap, s, defer);
    case OP_F_P_G23D: return launch_op<KFPG23D, T>(a, grid_cap, s, defer);
    case OP_F_RE_XVD: return launch_op<KFReXvD, T>(a, grid_cap, s, defer);
    case OP_F_RE_XV: return launch_op<KFReXv, T>(a, grid_cap, s, defer);
    case OP_R_DOTS: return launch_op<KRDots, T>(a, grid_cap, s, defer);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_finalize(const Ctl& ctl, int P, int nb, int slot, int fin, bool early, hipStream_t s) {
  hipLaunchKernelGGL(finalize_kernel, dim3(1), dim3(kFinBlock), 0, s, ctl, P, nb, slot, fin, early ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_group(int op, const void* const* in, void* const* out, const void* diag, int n, int k, int slot,
                        int fin, const Ctl& ctl, bool fp32, const GridCaps& grid_cap, hipStream_t s,
                        const Pending* pending, bool defer) {
  GArgs a;
  for (int i = 0; i < kMaxPassIn; ++i) a.in[i] = in[i];
  for (int i = 0; i < kMaxPassOut; ++i) a.out[i] = out[i];
  a.diag = diag;
  a.n = n;
  a.k = k;
  int kp = pad_k(k);
  int kpl = 0;
  while ((1 << kpl) < kp) ++kpl;
  a.kpl = kpl;
  a.slot = slot;
  a.fin = fin;
  a.ctl = ctl;
  a.pend = pending ? *pending : Pending{nullptr, F_NONE, 0, 0, 0};
  if (pending && (pending->P > kMaxK * 7 || !op_takes_pending(op))) return hipErrorInvalidValue;
  return fp32 ? dispatch_op<float>(op, a, grid_cap, s, defer) : dispatch_op<double>(op, a, grid_cap, s, defer);
}

// Workgroups of a vector pass (for the pair-major partial layout).
int group_blocks(int op, int n, int k, const GridCaps& caps) {
  int kpl = 0;
  while ((1 << kpl) < pad_k(k)) ++kpl;
  const GridCaps c = caps;
  return op_info(op).ndot > 0 ? op_blocks<KDot>(n, kpl, c) : op_blocks<KCopy>(n, kpl, c);
}

// ------------------------------------------------------- preconditioner ---

template <class T>
__global__ __launch_bounds__(kBlock) void prec_kernel(const T* __restrict__ in, T* __restrict__ out,
                                                      const T* __restrict__ diag, long n, int k, int kpl,
                                                      const Globals* glob) {
  if (glob && glob->nrun == 0) return;
  const int kp = 1 << kpl;
  const int c = threadIdx.x & (kp - 1);
  if (c >= k) return;
  const int rpb = kBlock >> kpl;
  const long stride = (long)gridDim.x * rpb;
  long row = (long)blockIdx.x * rpb + (threadIdx.x >> kpl);
  // four rows per step, every load of the step issued before the divisions
  constexpr int U = 4;
  for (; row + (U - 1) * stride < n; row += U * stride) {
    T v[U], d[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u] = __builtin_nontemporal_load(in + (size_t)(row + u * stride) * k + c);
      d[u] = diag[row + u * stride];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) __builtin_nontemporal_store(v[u] / d[u], out + (size_t)(row + u * stride) * k + c);
  }
  for (; row < n; row += stride) {
    const size_t e = (size_t)row * k + c;
    __builtin_nontemporal_store(__builtin_nontemporal_load(in + e) / diag[row], out + e);
  }
}

hipError_t launch_prec(const void* in, void* out, const void* diag, int n, int k, bool fp32, const Globals* glob,
                       hipStream_t s) {
  const int kp = pad_k(k);
  int kpl = 0;
  while ((1 << kpl) < kp) ++kpl;
  const int rpb = kBlock >> kpl;
  long blocks = (n + rpb - 1) / rpb;
  if (blocks > 512) blocks = 512;  // the streaming passes' grid: two waves per SIMD, four rows per step
  if (blocks < 1) blocks = 1;
  if (fp32)
    hipLaunchKernelGGL(prec_kernel<float>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const float*)in, (float*)out,
                       (const float*)diag, (long)n, k, kpl, glob);
  else
    hipLaunchKernelGGL(prec_kernel<double>, dim3((unsigned)blocks), dim3(kBlock), 0, s, (const double*)in,
                       (double*)out, (const double*)diag, (long)n, k, kpl, glob);
  return hipGetLastError();
}

// ------------------------------------------------------------- set-up ---

__global__ void setup_state_kernel(Ctl C, double tol, int maxit, int hist_cap) {
  const int c = threadIdx.x;
  if (c < C.k) {
    IS(C, I_STATUS, c) = ST_RUNNING;
    IS(C, I_PEND, c) = -1;
    IS(C, I_ITERS, c) = 0;
    IS(C, I_ZEROB, c) = 0;
  }
  if (c == 0) {
    C.glob->nrun = C.k;
    C.glob->it = 0;
    C.glob->maxit = maxit;
    C.glob->hist_cap = hist_cap;
    C.glob->tol = tol;
  }
}

hipError_t launch_setup_state(const Ctl& ctl, double tol, int maxit, int hist_cap, hipStream_t s) {
  hipLaunchKernelGGL(setup_state_kernel, dim3(1), dim3(kMaxK), 0, s, ctl, tol, maxit, hist_cap);
  return hipGetLastError();
}

__global__ void mark_maxit_kernel(Ctl C) {
  const int c = threadIdx.x;
  if (c < C.k && IS(C, I_STATUS, c) == ST_RUNNING) {
    IS(C, I_STATUS, c) = ST_MAXIT;
    IS(C, I_ITERS, c) = 0;
  }
  __syncthreads();
  if (c == 0) C.glob->nrun = 0;
}

hipError_t launch_mark_maxit(const Ctl& ctl, hipStream_t s) {
  hipLaunchKernelGGL(mark_maxit_kernel, dim3(1), dim3(kMaxK), 0, s, ctl);
  return hipGetLastError();
}

__global__ void extract_diag_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
                                    const double* __restrict__ val, double* diag, float* diag32, int n,
                                    Globals* glob) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
    if (col[e] == i) d += val[e];
  diag[i] = d;
  if (diag32) diag32[i] = (float)d;
  if (d == 0.0) atomicAdd(&glob->zero_diag, 1);
}

hipError_t launch_extract_diag(const int32_t* row_ptr, const int32_t* col, const double* val, double* diag,
                               float* diag32, int n, Globals* glob, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(extract_diag_kernel, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, row_ptr, col, val,
                     diag, diag32, n, glob);
  return hipGetLastError();
}

__global__ void convert_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

hipError_t launch_convert_f32(const double* in, float* out, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(convert_f32_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, in, out, count);
  return hipGetLastError();
}

// A M^{-1} with M = diag(A): entry e = (i, j) becomes a_ij / a_jj (one
// division, as the oracle forms it), in FP64 or rounded once to FP32.
__global__ void fold_jacobi_kernel(const int32_t* __restrict__ col, const double* __restrict__ val,
                                   const double* __restrict__ diag, double* __restrict__ out64,
                                   float* __restrict__ out32, int64_t nnz) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
    const double v = val[e] / diag[col[e]];
    if (out64) out64[e] = v;
    if (out32) out32[e] = (float)v;
  }
}

hipError_t launch_fold_jacobi(const int32_t* col, const double* val, const double* diag, double* out64, float* out32,
                              int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  int64_t blocks = (nnz + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(fold_jacobi_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, col, val, diag, out64, out32,
                     nnz);
  return hipGetLastError();
}

// ------------------------------------------------- merging demonstration ---
// The three groups of vector updates of Section 2.1 (Table 1): run 1 makes the
// updates y = a x + b y, z = b x + a z, z = b y + c z as three passes, run 2
// the first two in one pass, run 3 all three in one pass. The shape of the
// streaming vector passes: a grid-stride loop with four elements per lane in
// flight, 512 workgroups; STEP selects the single update of a run-1 pass
// (0, 1, 2) or the merged run (3: run 2, 4: run 3).
template <int STEP>
__device__ __forceinline__ void axpby_elem(const double* __restrict__ x, double* __restrict__ y,
                                           double* __restrict__ z, long i, double a, double b, double c) {
  const double xv = STEP == 2 ? 0.0 : x[i];
  double yv = STEP == 1 ? 0.0 : y[i];
  double zv = STEP == 0 ? 0.0 : z[i];
  if (STEP == 0 || STEP >= 3) yv = a * xv + b * yv;
  if (STEP == 1 || STEP >= 3) zv = b * xv + a * zv;
  if (STEP == 2 || STEP == 4) zv = b * yv + c * zv;
  if (STEP == 0 || STEP >= 3) __builtin_nontemporal_store(yv, y + i);
  if (STEP >= 1) __builtin_nontemporal_store(zv, z + i);
}

template <int STEP>
__global__ __launch_bounds__(kBlock) void axpby_kernel(const double* __restrict__ x, double* __restrict__ y,
                                                       double* __restrict__ z, long n, double a, double b,
                                                       double c) {
  constexpr int U = 4;
  const long stride = (long)gridDim.x * kBlock;
  long i = (long)blockIdx.x * kBlock + threadIdx.x;
  for (; i + (U - 1) * stride < n; i += U * stride) {
    double xv[U], yv[U], zv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = i + u * stride;
      xv[u] = STEP == 2 ? 0.0 : x[e];
      yv[u] = STEP == 1 ? 0.0 : y[e];
      zv[u] = STEP == 0 ? 0.0 : z[e];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long e = i + u * stride;
      if (STEP == 0 || STEP >= 3) yv[u] = a * xv[u] + b * yv[u];
      if (STEP == 1 || STEP >= 3) zv[u] = b * xv[u] + a * zv[u];
      if (STEP == 2 || STEP == 4) zv[u] = b * yv[u] + c * zv[u];
      if (STEP == 0 || STEP >= 3) __builtin_nontemporal_store(yv[u], y + e);
      if (STEP >= 1) __builtin_nontemporal_store(zv[u], z + e);
    }
  }
  for (; i < n; i += stride) axpby_elem<STEP>(x, y, z, i, a, b, c);
}

hipError_t launch_axpby(int run, const double* x, double* y, double* z, long n, double a, double b, double c,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  long blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 512) blocks = 512;
  const dim3 g((unsigned)blocks), t(kBlock);
  if (run == 1) {
    hipLaunchKernelGGL(axpby_kernel<0>, g, t, 0, s, x, y, z, n, a, b, c);
    hipLaunchKernelGGL(axpby_kernel<1>, g, t, 0, s, x, y, z, n, a, b, c);
    hipLaunchKernelGGL(axpby_kernel<2>, g, t, 0, s, x, y, z, n, a, b, c);
  } else if (run == 2) {
    hipLaunchKernelGGL(axpby_kernel<3>, g, t, 0, s, x, y, z, n, a, b, c);
  } else if (run == 3) {
    hipLaunchKernelGGL(axpby_kernel<4>, g, t, 0, s, x, y, z, n, a, b, c);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------- adjoint ---

// grad[e] = - sum_c lam[i, c] * x[j, c] for every stored entry e = (i, j).
// kp lanes per row: lane c reads column c of the contiguous rows lam[i, :] and
// x[j, :]; the k products are summed by xor shuffles inside each lane group.
__global__ __launch_bounds__(kBlock) void grad_values_kernel(const int32_t* __restrict__ row_ptr,
                                                            const int32_t* __restrict__ col,
                                                            const double* __restrict__ lam,
                                                            const double* __restrict__ x, double* __restrict__ grad,
                                                            long n, int k, int kpl) {
  const int kp = 1 << kpl;
  const int c = threadIdx.x & (kp - 1);
  const int rpb = kBlock >> kpl;
  const long stride = (long)gridDim.x * rpb;
  // every lane of a group runs the same trip count (row bounds are per group)
  for (long i = (long)blockIdx.x * rpb + (threadIdx.x >> kpl); i < n; i += stride) {
    const double li = c < k ? lam[(size_t)i * k + c] : 0.0;
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int j = col[e];
      double v = c < k ? li * x[(size_t)j * k + c] : 0.0;
      for (int off = 1; off < kp; off <<= 1) v += __shfl_xor(v, off, kp);
      if (c == 0) grad[e] = -v;
    }
  }
}

hipError_t launch_grad_values(const int32_t* row_ptr, const int32_t* col, const double* lam, const double* x,
                              double* grad, int n, int k, hipStream_t s) {
  const int kp = pad_k(k);
  int kpl = 0;
  while ((1 << kpl) < kp) ++kpl;
  const int rpb = kBlock >> kpl;
  long blocks = (n + rpb - 1) / rpb;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(grad_values_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, row_ptr, col, lam, x, grad,
                     (long)n, k, kpl);
  return hipGetLastError();
}

// Transposed CSR: count entries per column, exclusive scan, scatter, then
// sort every row of the transpose by original row index so the result (and
// every product with it) does not depend on the order of the atomics.
__global__ void transpose_count_kernel(const int32_t* __restrict__ col, int64_t nnz, int32_t* counts) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
    atomicAdd(&counts[col[e]], 1);
}

hipError_t launch_transpose_count(const int32_t* col, int64_t nnz, int32_t* counts, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  int64_t blocks = (nnz + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(transpose_count_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, col, nnz, counts);
  return hipGetLastError();
}

// Single-workgroup exclusive scan: row_ptr_t[0] = 0, row_ptr_t[i+1] = sum of
// counts[0..i]. Each thread scans a contiguous chunk; chunk totals are scanned
// in LDS.
__global__ __launch_bounds__(1024) void scan_kernel(const int32_t* __restrict__ counts, int32_t* __restrict__ out,
                                                    int n) {
  __shared__ int32_t s_tot[1024];
  const int t = threadIdx.x;
  const int chunk = (n + 1023) / 1024;
  const int b = t * chunk, e = min(n, b + chunk);
  int32_t sum = 0;
  for (int i = b; i < e; ++i) sum += counts[i];
  s_tot[t] = sum;
  __syncthreads();
  if (t == 0) {
    int32_t acc = 0;
    for (int i = 0; i < 1024; ++i) {
      const int32_t v = s_tot[i];
      s_tot[i] = acc;
      acc += v;
    }
    out[0] = 0;
  }
  __syncthreads();
  int32_t acc = s_tot[t];
  for (int i = b; i < e; ++i) {
    acc += counts[i];
    out[i + 1] = acc;
  }
}

hipError_t launch_scan(const int32_t* counts, int32_t* row_ptr_t, int n, hipStream_t s) {
  hipLaunchKernelGGL(scan_kernel, dim3(1), dim3(1024), 0, s, counts, row_ptr_t, n);
  return hipGetLastError();
}

__global__ void transpose_fill_kernel(const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col, int n,
                                      const int32_t* __restrict__ row_ptr_t, int32_t* cursor, int32_t* col_t,
                                      int32_t* perm) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    for (int e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      const int j = col[e];
      const int pos = row_ptr_t[j] + atomicAdd(&cursor[j], 1);
      col_t[pos] = i;
      perm[pos] = e;
    }
  }
}

hipError_t launch_transpose_fill(const int32_t* row_ptr, const int32_t* col, int n, const int32_t* row_ptr_t,
                                 int32_t* cursor, int32_t* col_t, int32_t* perm, hipStream_t s) {
  int blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(transpose_fill_kernel, dim3(blocks), dim3(kBlock), 0, s, row_ptr, col, n, row_ptr_t, cursor,
                     col_t, perm);
  return hipGetLastError();
}

__global__ void transpose_sort_kernel(const int32_t* __restrict__ row_ptr_t, int32_t* col_t, int32_t* perm, int n) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const int b = row_ptr_t[j], e = row_ptr_t[j + 1];
    for (int a = b + 1; a < e; ++a) {  // insertion sort (rows are short)
      const int key = col_t[a], pv = perm[a];
      int q = a - 1;
      while (q >= b && col_t[q] > key) {
        col_t[q + 1] = col_t[q];
        perm[q + 1] = perm[q];
        --q;
      }
      col_t[q + 1] = key;
      perm[q + 1] = pv;
    }
  }
}

hipError_t launch_transpose_sort_rows(const int32_t* row_ptr_t, int32_t* col_t, int32_t* perm, int n, hipStream_t s) {
  int blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(transpose_sort_kernel, dim3(blocks), dim3(kBlock), 0, s, row_ptr_t, col_t, perm, n);
  return hipGetLastError();
}

__global__ void gather_values_kernel(const double* __restrict__ val, const int32_t* __restrict__ perm,
                                     double* __restrict__ val_t, int64_t nnz) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nnz; p += (int64_t)gridDim.x * blockDim.x)
    val_t[p] = val[perm[p]];
}

hipError_t launch_gather_values(const double* val, const int32_t* perm, double* val_t, int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  int64_t blocks = (nnz + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(gather_values_kernel, dim3((unsigned)blocks), dim3(kBlock), 0, s, val, perm, val_t, nnz);
  return hipGetLastError();
}

}  // namespace bcg
