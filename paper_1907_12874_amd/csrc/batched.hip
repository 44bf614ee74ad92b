// Batched tier: many independent systems A_s X_s = B_s (uneven sizes, k_s
// right-hand sides each) solved by one persistent kernel launch.
//
// Every system owns a contiguous range of workgroups; its workgroups split its
// rows into contiguous chunks and run the merged classical BiCGStab (Alg. 2,
// or with Jacobi Alg. 5 in its fused form: the products read A M^{-1} and the
// solution update divides p and s by a_ii) with a per-system barrier between
// the phases of an iteration:
//   A  v = A p, partial delta = (v, r0)            | barrier | alpha
//   B  s = r - alpha v                             | barrier (neighbours read s)
//   C  t = A s, partial phi, psi, theta            | barrier | omega, stop test
//   D  x += alpha p + omega s, r = s - omega t,    | barrier | beta, close pass
//      partial rho' = (r, r0)
//   E  p = r + beta (p - omega v)                  | barrier (neighbours read p)
// Each phase stores its dot partials in its own slot; after the barrier every
// workgroup of the system sums the same partials in the same order and so
// takes bitwise the same scalar decisions without a further barrier. The
// scalar recurrence, stop test and breakdown rules are those of the
// single-system path.
//
// All workgroups of a launch must be resident at once: the host keeps the
// grid within half the occupancy limit. A barrier waits at most a fixed wall
// time; if that passes (or another workgroup gave up) the workgroup raises the
// abort flag and returns, so every wave exits and the host reports an error.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bicgstab.h"
#include "internal.hpp"

namespace bcg {
namespace {

struct BSys {
  const int32_t* row_ptr;
  const int32_t* col;
  const double* val;
  const double* val_f;  // values of the iteration's products: A, or A M^{-1} with Jacobi
  const double* diag;   // a_ii with Jacobi, else null
  const double* b;
  double* x;
  double* vec;   // r, r0, p, v, s, t: 6 blocks of n*k
  double* part;  // [4 slots][nw][4 dots][kp]
  int32_t* out_iters;
  int32_t* out_status;
  double* out_relres;
  double* out_relres_rec;
  unsigned* bar;
  unsigned long long* clk;  // [2]: wall clock at start / end of the system
  int n, k, kpl, nw, w0, maxlen;  // maxlen: entries of the system's longest row
};

struct BGlob {
  double tol;
  long long wait_ticks;  // longest barrier wait in wall-clock ticks
  int maxit;
  int nsys;
  int* abort_flag;
};

// Global-memory views of the arrays: pointers read from the descriptors are
// generic; as global pointers the loads take a uniform base and a 32-bit
// offset.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) const double gcdouble;
typedef __attribute__((address_space(1))) const int32_t gcint;
typedef __attribute__((address_space(1))) char gchar;

// Element e of a global array through a 32-bit byte offset (every array of a
// system fits in 32 bits: n * k * 8 < 2^31 and nnz < 2^29, checked at create;
// the partials take a few MB), so the load or store takes a uniform base and
// no 64-bit address arithmetic.
template <class T>
__device__ __forceinline__ T& at(T* base, unsigned e) {
  return *(T*)((gchar*)base + e * (unsigned)sizeof(T));
}

// Element (j, c) of a row-major n x k block: j * k + c with a 24-bit multiply
// (a full-rate instruction; n < 2^24 and k <= 64 are checked at create).
__device__ __forceinline__ unsigned xoff(int j, int k, int c) {
  return __umul24((unsigned)j, (unsigned)k) + (unsigned)c;
}

// Barrier over the nw workgroups of one system: a monotonic counter; the
// barrier with ordinal e completes when the counter reaches (e + 1) * nw.
// Every wave first waits for its own stores to complete, then one thread
// releases at agent scope, arrives, waits and acquires. Returns false on abort.
// On this multi-XCD part the agent-scope release writes back the L2 of the
// workgroup's XCD and the acquire invalidates its L1 and L2; both complete
// asynchronously, so the thread waits for each (s_waitcnt) before it arrives
// and before the workgroup barrier lets the other waves load: without the
// first wait the arrival could be seen before the written-back data, without
// the second another wave's load could be served from a line the
// invalidation has not reached yet (both seen as rare stale reads of other
// workgroups' blocks and partials when the waits were left to the compiler).
// A system on a single workgroup needs only the workgroup barrier: its waves
// share one compute unit and its L1, so a workgroup-scope release / acquire
// (__syncthreads) orders their global stores and loads, and no agent-scope
// fence (which writes back the L2) or counter is needed.
__device__ bool sys_barrier(unsigned* bar, unsigned target, int* abort_flag, long long wait_ticks, int nw) {
  __shared__ int s_ok;
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (nw == 1) return true;
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int ok = 1;
    const unsigned long long t0 = wall_clock64();
    while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
          (long long)(wall_clock64() - t0) > wait_ticks) {
        __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    __builtin_amdgcn_s_waitcnt(0);
    s_ok = ok;
  }
  __syncthreads();
  return s_ok != 0;
}

// Per-column partial sums of ND dots over this workgroup's rows, in a fixed
// order, stored to the system's partial slot. A wavefront holds rpw = 64 / k
// rows of k lanes (lane = row slot * k + column); its slots are added by a
// pairwise tree, adjacent slots first (slot s takes slot s + off when s is a
// multiple of 2 off and s + off < rpw: an odd last slot passes up unpaired),
// then the wavefronts in index order.
template <int BS, int ND>
__device__ void store_partials(const BSys& S, int slot, int w, const double (&acc)[4],
                               double (*s_w)[4][kMaxK]) {
  const int kp = 1 << S.kpl;
  const int k = S.k, rpw = 64 / k;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int rs = lane / k;
#pragma unroll
  for (int d = 0; d < ND; ++d) {
    double v = acc[d];
    if ((k & (k - 1)) == 0) {
      // k a power of two: the same tree by xor shuffles (every slot ends
      // with the sum its leader gets)
      for (int off = k; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    } else {
      for (int off = 1; off < rpw; off <<= 1) {
        const double o = __shfl(v, min(lane + off * k, 63), 64);
        if ((rs & (2 * off - 1)) == 0 && rs + off < rpw) v += o;
      }
    }
    if (lane < k) s_w[wave][d][lane] = v;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ND * k; t += BS) {
    const int d = t / k, c = t - d * k;
    double v = s_w[0][d][c];
#pragma unroll
    for (int q = 1; q < BS / 64; ++q) v += s_w[q][d][c];
    at((gdouble*)S.part, (unsigned)(((slot * S.nw + w) * 4 + d) * kp + c)) = v;
  }
}

// Sum a slot's partials over the system's workgroups (index order) into out.
template <int BS, int ND>
__device__ void reduce_partials(const BSys& S, int slot, double (*out)[kMaxK]) {
  const int kp = 1 << S.kpl;
  for (int t = threadIdx.x; t < ND * S.k; t += BS) {
    const int d = t / S.k, c = t - d * S.k;
    double v = 0.0;
    // 16 partials loaded at once (not one dependent load per workgroup),
    // then added in workgroup order
    for (int q0 = 0; q0 < S.nw; q0 += 16) {
      double pv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j)
        pv[j] = at((gcdouble*)S.part, (unsigned)(((slot * S.nw + min(q0 + j, S.nw - 1)) * 4 + d) * kp + c));
#pragma unroll
      for (int j = 0; j < 16; ++j) v = q0 + j < S.nw ? v + pv[j] : v;
    }
    out[d][c] = v;
  }
  __syncthreads();
}

// Sparse products: (A X)[row, c] for the rows row, row + rpp, ... below row1
// of a thread, each row's entries added in stored order with no contraction
// (bitwise the CSR product of the single-system path), handed to
// emit(row, e, y, q) in increasing row order, where q holds NP operands of
// element e = (row, c) that pre(e, q) loads (the other block the phase reads
// at that element).
//
// A row's product is a chain of three dependent loads: its row offsets, then
// its column indices and values, then the gathered X entries. The rows of a
// thread are software-pipelined so that the chain of one row overlaps those
// of the next two: while the gathers of a stage (RU rows) are in flight, the
// column indices of the next stage and the row offsets of the stage after
// are loaded, and every load of the loop body is unconditional (rows past
// row1 load a valid row's entries and are not emitted), so a stage costs
// about one memory round trip instead of three. The first CH entries of a row
// go through the pipeline; a longer row adds the rest afterwards, CH at a
// time, still in entry order. A slot past the row's end repeats its last
// entry and its product is not added (a select); an empty row's slots load
// entry 0 (a system without entries points at a zero dummy entry) and add
// nothing.
template <int CH, int RU, int NP, class Pre, class Emit>
__device__ __forceinline__ void product_rows_ch(const BSys& S, const double* V, const gdouble* __restrict__ X,
                                                int row, int rpp, int row1, int c, Pre pre, Emit emit) {
  if (row >= row1) return;
  gcint* __restrict__ rp = (gcint*)S.row_ptr;
  gcint* __restrict__ col = (gcint*)S.col;
  gcdouble* __restrict__ val = (gcdouble*)V;
  const int k = S.k;
  const int last = row1 - 1;
  // stage being computed: rows row + u * rpp, their offsets and column indices
  int eb[RU], ne[RU], cj[RU][CH];
  // row offsets of the next stage (raw, so no wait is forced before they are used)
  int pa[RU], pb[RU];
  auto load_cols = [&](const int (&a)[RU], const int (&b)[RU]) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      eb[u] = a[u];
      ne[u] = b[u] - a[u];
#pragma unroll
      for (int j = 0; j < CH; ++j) cj[u][j] = at(col, (unsigned)(ne[u] > 0 ? eb[u] + min(j, ne[u] - 1) : 0));
    }
  };
  auto load_offsets = [&](int r) {
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int rr = min(r + u * rpp, last);
      pa[u] = at(rp, (unsigned)rr);
      pb[u] = at(rp, (unsigned)rr + 1u);
    }
  };
  load_offsets(row);
  load_cols(pa, pb);
  load_offsets(row + RU * rpp);
  for (;;) {
    double xv[RU][CH], av[RU][CH], q[RU][NP > 0 ? NP : 1];
#pragma unroll
    for (int u = 0; u < RU; ++u) {
#pragma unroll
      for (int j = 0; j < CH; ++j) xv[u][j] = at(X, xoff(cj[u][j], k, c));
#pragma unroll
      for (int j = 0; j < CH; ++j) av[u][j] = at(val, (unsigned)(ne[u] > 0 ? eb[u] + min(j, ne[u] - 1) : 0));
      if constexpr (NP > 0) pre(xoff(min(row + u * rpp, last), k, c), q[u]);
    }
    // the stage's offsets and entry ranges, kept for the sums below
    int ebc[RU], nec[RU];
#pragma unroll
    for (int u = 0; u < RU; ++u) ebc[u] = eb[u], nec[u] = ne[u];
    const int nrow = row + RU * rpp;
    load_cols(pa, pb);
    load_offsets(nrow + RU * rpp);
#pragma unroll
    for (int u = 0; u < RU; ++u) {
      const int rr = row + u * rpp;
      if (rr >= row1) break;
      double z = 0.0;
#pragma unroll
      for (int j = 0; j < CH; ++j) {
        const double t = z + av[u][j] * xv[u][j];
        z = j < nec[u] ? t : z;
      }
      // entries past the first CH (rows longer than a step)
      for (int o = CH; o < nec[u]; o += CH) {
        int cl[CH];
        double al[CH], xl[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const int e = ebc[u] + min(o + j, nec[u] - 1);
          cl[j] = at(col, (unsigned)e);
          al[j] = at(val, (unsigned)e);
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) xl[j] = at(X, xoff(cl[j], k, c));
#pragma unroll
        for (int j = 0; j < CH; ++j) {
          const double t = z + al[j] * xl[j];
          z = o + j < nec[u] ? t : z;
        }
      }
      emit(rr, xoff(rr, k, c), z, q[u]);
    }
    if (nrow >= row1) break;
    row = nrow;
  }
}

// The product with CH pipelined slots at most: fewer when no row of the
// system has more entries (5 for a 5-point, 7 for a 7-point stencil), so no
// slot is spent on padding every row shares. The sums are the same (a slot
// past a row's end is never added). V: the values (A's, or A M^{-1}'s).
template <int CH, int RU, int NP, class Pre, class Emit>
__device__ __forceinline__ void product_rows(const BSys& S, const double* V, const gdouble* __restrict__ X, int row,
                                             int rpp, int row1, int c, Pre pre, Emit emit) {
  if constexpr (CH > 5) {
    if (S.maxlen <= 5) return product_rows_ch<5, RU, NP>(S, V, X, row, rpp, row1, c, pre, emit);
  }
  if constexpr (CH > 7) {
    if (S.maxlen <= 7) return product_rows_ch<7, RU, NP>(S, V, X, row, rpp, row1, c, pre, emit);
  }
  product_rows_ch<CH, RU, NP>(S, V, X, row, rpp, row1, c, pre, emit);
}

enum { B_RHO = 0, B_ALPHA, B_OMEGA, B_BETA, B_EPS2, B_BB, B_NS };

// VU: rows per step of a thread in the vector phases (all their loads issued
// before any is used); RU: rows per stage of the sparse products' pipeline;
// CH: entries per pipelined step of a row product. A thread still visits its
// rows in increasing order, so its partial sums keep their order.
template <int BS, int VU, int CH, int RU>
__global__ __launch_bounds__(BS) void batched_kernel(const BGlob* __restrict__ Gp, const BSys* __restrict__ sys,
                                                     const int32_t* __restrict__ wg_sys) {
  const BGlob G = *Gp;
  const int sidx = wg_sys[blockIdx.x];
  const BSys S = sys[sidx];
  const int w = blockIdx.x - S.w0;
  const int kp = 1 << S.kpl;
  // a wavefront holds 64 / k rows of k lanes (lane = row slot * k + column);
  // the lanes past the last whole row take no row (c = k)
  const int rpw = 64 / S.k;
  const int lane = threadIdx.x & 63;
  const int rslot = min(lane / S.k, rpw - 1);
  const int c = lane / S.k < rpw ? lane - rslot * S.k : S.k;
  const int rsub = (threadIdx.x >> 6) * rpw + rslot;
  const int rpp = (BS / 64) * rpw;
  const int n = S.n, k = S.k;
  const size_t nk = (size_t)n * k;
  const int chunk = (n + S.nw - 1) / S.nw;
  const int row0 = min(n, w * chunk), row1 = min(n, row0 + chunk);
  gdouble* __restrict__ r = (gdouble*)S.vec;
  gdouble* __restrict__ r0 = r + nk;
  gdouble* __restrict__ p = r0 + nk;
  gdouble* __restrict__ v = p + nk;
  gdouble* __restrict__ s = v + nk;
  gdouble* __restrict__ t = s + nk;
  gcdouble* __restrict__ b = (gcdouble*)S.b;
  gdouble* __restrict__ x = (gdouble*)S.x;

  __shared__ double s_w[BS / 64][4][kMaxK];
  __shared__ double sc[B_NS][kMaxK];
  __shared__ double dsum[4][kMaxK];
  __shared__ int st[kMaxK], pend[kMaxK], iters[kMaxK], zerob[kMaxK];
  __shared__ int nrun;
  unsigned epoch = 0;
  auto barrier = [&]() { return sys_barrier(S.bar, (++epoch) * (unsigned)S.nw, G.abort_flag, G.wait_ticks, S.nw); };
  // element offsets fit in 32 bits (checked at create): uniform base + 32-bit offset addressing
  auto eidx = [&](int row) { return xoff(row, k, c); };
  if (w == 0 && threadIdx.x == 0) S.clk[0] = wall_clock64();

  // ---- start: r = b - A x0, r0 = r, p = r; partial (r, r), (b, b)
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (c < k)
    product_rows<CH, RU, 1>(
        S, S.val, x, row0 + rsub, rpp, row1, c, [&](unsigned e, double(&q)[1]) { q[0] = at(b, e); },
        [&](int, unsigned e, double z, const double(&q)[1]) {
          const double bv = q[0];
          const double res = bv - z;
          at(r, e) = res;
          at(r0, e) = res;
          at(p, e) = res;
          acc[0] += res * res;
          acc[1] += bv * bv;
        });
  store_partials<BS, 2>(S, 0, w, acc, s_w);
  if (!barrier()) return;
  reduce_partials<BS, 2>(S, 0, dsum);
  if (threadIdx.x < kp) {
    const int cc = threadIdx.x;
    const double rr = dsum[0][cc], bb = dsum[1][cc];
    pend[cc] = -1;
    iters[cc] = 0;
    zerob[cc] = 0;
    sc[B_ALPHA][cc] = 0.0;
    sc[B_OMEGA][cc] = 1.0;
    sc[B_BETA][cc] = 0.0;
    sc[B_BB][cc] = bb;
    const double eps2 = G.tol > 0.0 ? G.tol * G.tol * bb : -INFINITY;
    sc[B_EPS2][cc] = eps2;
    sc[B_RHO][cc] = rr;
    int status = ST_RUNNING;
    if (cc >= k) status = ST_CONVERGED;
    else if (!isfinite(bb)) status = ST_NONFINITE;
    else if (bb == 0.0) {
      status = ST_CONVERGED;
      zerob[cc] = 1;
    } else if (!isfinite(rr)) status = ST_NONFINITE;
    else if (rr < eps2) status = ST_CONVERGED;
    else if (G.maxit <= 0) status = ST_MAXIT;
    st[cc] = status;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int nr = 0;
    for (int cc = 0; cc < k; ++cc) nr += st[cc] == ST_RUNNING;
    nrun = nr;
  }
  __syncthreads();
  // a zero right-hand side has the zero solution
  if (c < k && zerob[c])
    for (int row = row0 + rsub; row < row1; row += rpp) at(x, eidx(row)) = 0.0;
  if (!barrier()) return;

  for (int it = 0; it < G.maxit && nrun > 0; ++it) {
    // ---- A: v = A p; delta = (v, r0)
    const bool run1 = c < k && st[c] == ST_RUNNING;
    acc[0] = 0.0;
    if (run1)
      product_rows<CH, RU, 1>(
          S, S.val_f, p, row0 + rsub, rpp, row1, c, [&](unsigned e, double(&q)[1]) { q[0] = at(r0, e); },
          [&](int, unsigned e, double z, const double(&q)[1]) {
            at(v, e) = z;
            acc[0] += z * q[0];
          });
    store_partials<BS, 1>(S, 1, w, acc, s_w);
    if (!barrier()) return;
    reduce_partials<BS, 1>(S, 1, dsum);
    if (threadIdx.x < k && st[threadIdx.x] == ST_RUNNING) {
      const int cc = threadIdx.x;
      const double delta = dsum[0][cc];
      if (delta == 0.0) {
        st[cc] = ST_BREAKDOWN;
        iters[cc] = it + 1;
      } else {
        const double alpha = sc[B_RHO][cc] / delta;
        if (!isfinite(alpha)) {
          st[cc] = ST_NONFINITE;
          iters[cc] = it + 1;
        } else {
          sc[B_ALPHA][cc] = alpha;
        }
      }
    }
    __syncthreads();
    // ---- B: s = r - alpha v
    const bool run2 = c < k && st[c] == ST_RUNNING;
    if (run2) {
      const double alpha = sc[B_ALPHA][c];
      for (int row = row0 + rsub; row < row1; row += VU * rpp) {
        double rv[VU], vv[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) {
            rv[u] = at(r, eidx(rr));
            vv[u] = at(v, eidx(rr));
          }
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) at(s, eidx(rr)) = rv[u] - alpha * vv[u];
        }
      }
    }
    if (!barrier()) return;
    // ---- C: t = A s; phi = (t, s), psi = (t, t), theta = (s, s)
    acc[0] = acc[1] = acc[2] = 0.0;
    if (run2)
      product_rows<CH, RU, 1>(
          S, S.val_f, s, row0 + rsub, rpp, row1, c, [&](unsigned e, double(&q)[1]) { q[0] = at(s, e); },
          [&](int, unsigned e, double tt, const double(&q)[1]) {
            const double ss = q[0];
            at(t, e) = tt;
            acc[0] += tt * ss;
            acc[1] += tt * tt;
            acc[2] += ss * ss;
          });
    store_partials<BS, 3>(S, 2, w, acc, s_w);
    if (!barrier()) return;
    reduce_partials<BS, 3>(S, 2, dsum);
    if (threadIdx.x < k && st[threadIdx.x] == ST_RUNNING) {
      const int cc = threadIdx.x;
      const double phi = dsum[0][cc], psi = dsum[1][cc], theta = dsum[2][cc];
      const double omega = psi != 0.0 ? phi / psi : 0.0;
      const double est = theta - omega * phi;
      if (!(isfinite(omega) && isfinite(est))) {
        st[cc] = ST_NONFINITE;
        iters[cc] = it + 1;
      } else {
        sc[B_OMEGA][cc] = omega;
        if (est < sc[B_EPS2][cc])
          pend[cc] = ST_CONVERGED;
        else if (omega == 0.0)
          pend[cc] = ST_BREAKDOWN;
      }
    }
    __syncthreads();
    // ---- D: x += alpha p + omega s; r = s - omega t; rho' = (r, r0)
    // (with Jacobi x += alpha p / a_ii + omega s / a_ii: Alg. 5's p-hat and
    // s-hat, formed here for the update alone)
    const bool run3 = c < k && st[c] == ST_RUNNING;
    acc[0] = 0.0;
    auto phase_d = [&](auto jac) {
      constexpr bool J = decltype(jac)::value;
      gcdouble* __restrict__ dg = (gcdouble*)S.diag;
      const double alpha = sc[B_ALPHA][c], omega = sc[B_OMEGA][c];
      for (int row = row0 + rsub; row < row1; row += VU * rpp) {
        double xv[VU], pv[VU], sv[VU], tv[VU], qv[VU], dv[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) {
            const unsigned e = eidx(rr);
            xv[u] = at(x, e);
            pv[u] = at(p, e);
            sv[u] = at(s, e);
            tv[u] = at(t, e);
            qv[u] = at(r0, e);
            if constexpr (J) dv[u] = at(dg, (unsigned)rr);
          }
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) {
            const unsigned e = eidx(rr);
            if constexpr (J)
              at(x, e) = xv[u] + alpha * (pv[u] / dv[u]) + omega * (sv[u] / dv[u]);
            else
              at(x, e) = xv[u] + alpha * pv[u] + omega * sv[u];
            const double res = sv[u] - omega * tv[u];
            at(r, e) = res;
            acc[0] += res * qv[u];
          }
        }
      }
    };
    if (run3) {
      if (S.diag)
        phase_d(std::true_type{});
      else
        phase_d(std::false_type{});
    }
    store_partials<BS, 1>(S, 3, w, acc, s_w);
    if (!barrier()) return;
    reduce_partials<BS, 1>(S, 3, dsum);
    if (threadIdx.x < k && st[threadIdx.x] == ST_RUNNING) {
      const int cc = threadIdx.x;
      if (pend[cc] >= 0) {
        st[cc] = pend[cc];
        iters[cc] = it + 1;
      } else {
        const double rho1 = dsum[0][cc];
        const double beta = (rho1 / sc[B_RHO][cc]) * (sc[B_ALPHA][cc] / sc[B_OMEGA][cc]);
        if (rho1 == 0.0) {
          st[cc] = ST_BREAKDOWN;
          iters[cc] = it + 1;
        } else if (!isfinite(beta)) {
          st[cc] = ST_NONFINITE;
          iters[cc] = it + 1;
        } else {
          sc[B_BETA][cc] = beta;
          sc[B_RHO][cc] = rho1;
          if (it + 1 >= G.maxit) {
            st[cc] = ST_MAXIT;
            iters[cc] = it + 1;
          }
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      int nr = 0;
      for (int cc = 0; cc < k; ++cc) nr += st[cc] == ST_RUNNING;
      nrun = nr;
    }
    __syncthreads();
    // ---- E: p = r + beta (p - omega v)
    if (c < k && st[c] == ST_RUNNING) {
      const double beta = sc[B_BETA][c], omega = sc[B_OMEGA][c];
      for (int row = row0 + rsub; row < row1; row += VU * rpp) {
        double rv[VU], pv[VU], vv[VU];
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) {
            const unsigned e = eidx(rr);
            rv[u] = at(r, e);
            pv[u] = at(p, e);
            vv[u] = at(v, e);
          }
        }
#pragma unroll
        for (int u = 0; u < VU; ++u) {
          const int rr = row + u * rpp;
          if (rr < row1) at(p, eidx(rr)) = rv[u] + beta * (pv[u] - omega * vv[u]);
        }
      }
    }
    if (!barrier()) return;
  }

  // ---- exit: partial (b - A x, b - A x) and (r, r) per column
  acc[0] = acc[1] = 0.0;
  if (c < k)
    product_rows<CH, RU, 2>(
        S, S.val, x, row0 + rsub, rpp, row1, c,
        [&](unsigned e, double(&q)[2]) {
          q[0] = at(b, e);
          q[1] = at(r, e);
        },
        [&](int, unsigned e, double z, const double(&q)[2]) {
          const double d = q[0] - z;
          acc[0] += d * d;
          acc[1] += q[1] * q[1];
        });
  store_partials<BS, 2>(S, 0, w, acc, s_w);
  if (!barrier()) return;
  if (w != 0) return;
  reduce_partials<BS, 2>(S, 0, dsum);
  if (threadIdx.x < k) {
    const int cc = threadIdx.x;
    const double bb = sc[B_BB][cc];
    const bool zero = zerob[cc] != 0;
    S.out_status[cc] = st[cc] == ST_RUNNING ? ST_MAXIT : st[cc];
    S.out_iters[cc] = st[cc] == ST_RUNNING ? G.maxit : iters[cc];
    S.out_relres[cc] = zero ? 0.0 : sqrt(dsum[0][cc]) / sqrt(bb);
    S.out_relres_rec[cc] = zero ? 0.0 : sqrt(dsum[1][cc]) / sqrt(bb);
  }
  if (threadIdx.x == 0) S.clk[1] = wall_clock64();
}

__global__ void batched_reset_kernel(unsigned* bars, int nsys, int* abort_flag) {
  for (int i = threadIdx.x; i < nsys; i += blockDim.x) bars[i] = 0u;
  if (threadIdx.x == 0) *abort_flag = 0;
}

constexpr double kBarrierWaitSeconds = 2.0;

// Kernel variants the tuner chooses from: threads per workgroup, rows per
// step in the vector phases, entries per pipelined step of a row product,
// rows per stage of the sparse products' pipeline.
struct Variant {
  int block, rows, entries, product_rows;
};
constexpr Variant kVariants[] = {{256, 2, 8, 1}, {1024, 2, 8, 1}, {512, 2, 8, 1},
                                 {512, 4, 8, 1}, {512, 2, 8, 2}, {512, 8, 8, 1}};
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

template <int V>
constexpr auto variant_kernel() {
  return batched_kernel<kVariants[V].block, kVariants[V].rows, kVariants[V].entries, kVariants[V].product_rows>;
}

const void* kernel_of(int v) {
  switch (v) {
    case 0: return (const void*)variant_kernel<0>();
    case 1: return (const void*)variant_kernel<1>();
    case 2: return (const void*)variant_kernel<2>();
    case 3: return (const void*)variant_kernel<3>();
    case 4: return (const void*)variant_kernel<4>();
    default: return (const void*)variant_kernel<5>();
  }
}

hipError_t launch_variant(int v, int wgs, hipStream_t st, const BGlob* G, const BSys* S, const int32_t* W) {
  switch (v) {
    case 0: hipLaunchKernelGGL(variant_kernel<0>(), dim3(wgs), dim3(kVariants[0].block), 0, st, G, S, W); break;
    case 1: hipLaunchKernelGGL(variant_kernel<1>(), dim3(wgs), dim3(kVariants[1].block), 0, st, G, S, W); break;
    case 2: hipLaunchKernelGGL(variant_kernel<2>(), dim3(wgs), dim3(kVariants[2].block), 0, st, G, S, W); break;
    case 3: hipLaunchKernelGGL(variant_kernel<3>(), dim3(wgs), dim3(kVariants[3].block), 0, st, G, S, W); break;
    case 4: hipLaunchKernelGGL(variant_kernel<4>(), dim3(wgs), dim3(kVariants[4].block), 0, st, G, S, W); break;
    default: hipLaunchKernelGGL(variant_kernel<5>(), dim3(wgs), dim3(kVariants[5].block), 0, st, G, S, W); break;
  }
  return hipGetLastError();
}

}  // namespace
}  // namespace bcg

using namespace bcg;

namespace {
int bfail(int code, const std::string& m) { return bcg::set_last_error(code, m); }
#define BCHK(expr)                                                                                            \
  do {                                                                                                        \
    hipError_t e_ = (expr);                                                                                   \
    if (e_ != hipSuccess) return bfail(BICGSTAB_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)
size_t al256(size_t b) { return (b + 255) & ~size_t(255); }
int next_pow2(int k) {
  int p = 1;
  while (p < k) p <<= 1;
  return p;
}
int log2i(int p) {
  int l = 0;
  while ((1 << l) < p) ++l;
  return l;
}
}  // namespace

struct bicgstab_batched_ctx {
  int nsys = 0;
  std::vector<int64_t> n, nnz;
  std::vector<int> maxlen;  // entries of each system's longest row
  std::vector<int> k;
  std::vector<const int32_t*> rp, col;
  std::vector<const double*> val;
  // Jacobi: per system a_ii and A M^{-1} (entries a_ij / a_jj), formed at
  // create in one library-owned allocation
  int precond = BICGSTAB_PRECOND_NONE;
  char* jac = nullptr;
  std::vector<const double*> diag, val_f;
  size_t total_cols = 0;
  int kp_max = 1;
  hipStream_t user_stream = nullptr, ws = nullptr;
  hipEvent_t ev = nullptr, t0 = nullptr, t1 = nullptr;
  int device = 0, cus = 0;
  double wall_hz = 1e8;
  int cap[kNumVariants] = {};  // resident workgroups of each variant on the device
  int pool_wgs = 0;
  // configuration
  int variant = 1;
  std::vector<int> nw;
  // fixed workspace layout (offsets from base)
  size_t o_glob = 0, o_sys = 0, o_wg = 0, o_dummy = 0, o_bar = 0, o_res = 0, o_part = 0, bytes_needed = 0;
  size_t res_bytes = 0, stage_bytes = 0;
  std::vector<size_t> o_vec;
  char* base = nullptr;
  size_t bytes = 0;
  bool owned = false;
  std::vector<char> stage, res;
  // captured launch, valid while (variant, workgroups, base) are unchanged
  hipGraphExec_t graph = nullptr;
  int graph_variant = -1, graph_wgs = 0;
  char* graph_base = nullptr;
  // last solve
  double last_ms = 0.0;
  std::vector<double> sys_ms;
  std::vector<int> sys_iters;
};

namespace {

int total_wgs(const std::vector<int>& nw) {
  int t = 0;
  for (int v : nw) t += v;
  return t;
}

int max_wgs(const bicgstab_batched_ctx* h, int s, int budget) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(h->n[s] / 64, budget));
}

// Bytes one iteration of system s moves: two sparse products (values, column
// indices, row pointers, the gathered and written blocks) and the vector
// passes of the merged classical form (14 block reads, 4 writes).
double pass_bytes(const bicgstab_batched_ctx* h, int s) {
  const double blk = 8.0 * (double)h->n[s] * h->k[s];
  return 2.0 * (12.0 * h->nnz[s] + 4.0 * h->n[s] + 2.0 * blk) + 18.0 * blk;
}

// Workgroups proportional to bytes x passes, at least one each.
std::vector<int> proportional(const bicgstab_batched_ctx* h, int budget, const std::vector<double>& passes) {
  std::vector<double> wgt(h->nsys);
  double tot = 0.0;
  for (int s = 0; s < h->nsys; ++s) tot += wgt[s] = pass_bytes(h, s) * std::max(1.0, passes[s]);
  std::vector<int> nw(h->nsys);
  const int spare = std::max(0, budget - h->nsys);
  for (int s = 0; s < h->nsys; ++s)
    nw[s] = std::min(max_wgs(h, s, budget), 1 + (int)std::floor(spare * wgt[s] / tot));
  return nw;
}

// Model of the time of system s: passes_s * (L + pass_bytes_s / (nw_s * B)),
// with L (per-pass latency: barriers and reductions) and B (bytes per ms one
// workgroup streams) fitted by least squares to the measured per-system times
// of the last run. Then the smallest makespan T whose allocation fits the
// budget (bisection over T; each system takes the fewest workgroups that
// finish it within T).
std::vector<int> model_allocation(const bicgstab_batched_ctx* h, int budget) {
  const int m = h->nsys;
  double sx = 0, sy = 0, sxx = 0, sxy = 0;
  int cnt = 0;
  for (int s = 0; s < m; ++s) {
    if (h->sys_iters[s] < 1 || h->sys_ms[s] <= 0.0) continue;
    const double xx = pass_bytes(h, s) / h->nw[s];
    const double yy = h->sys_ms[s] / h->sys_iters[s];
    sx += xx, sy += yy, sxx += xx * xx, sxy += xx * yy;
    ++cnt;
  }
  double L = 0.0, invB = 0.0;
  if (cnt >= 2 && cnt * sxx - sx * sx > 0.0) {
    invB = (cnt * sxy - sx * sy) / (cnt * sxx - sx * sx);
    L = (sy - invB * sx) / cnt;
  }
  if (!(invB > 0.0) || !(L >= 0.0)) {
    // degenerate fit: no latency term, throughput from the totals
    L = 0.0;
    invB = sx > 0.0 ? sy / sx : 1e-9;
  }
  std::vector<int> nw(m);
  auto alloc = [&](double T) {
    long long tot = 0;
    for (int s = 0; s < m; ++s) {
      const double it = std::max(1, h->sys_iters[s]);
      const double room = T / it - L;
      const int cap = max_wgs(h, s, budget);
      int v = cap;
      if (room > 0.0) v = (int)std::min<double>(cap, std::ceil(pass_bytes(h, s) * invB / room));
      nw[s] = std::max(1, v);
      tot += nw[s];
    }
    return tot;
  };
  double lo = 0.0, hi = 0.0;
  for (int s = 0; s < m; ++s) {
    const double it = std::max(1, h->sys_iters[s]);
    hi = std::max(hi, it * (L + pass_bytes(h, s) * invB));
  }
  for (int i = 0; i < 60; ++i) {
    const double mid = 0.5 * (lo + hi);
    if (alloc(mid) <= budget) hi = mid;
    else lo = mid;
  }
  alloc(hi);
  return nw;
}

void compute_layout(bicgstab_batched_ctx* h) {
  size_t off = 0;
  auto take = [&](size_t b) {
    const size_t o = off;
    off += al256(b);
    return o;
  };
  h->o_glob = take(sizeof(BGlob));
  h->o_sys = take(sizeof(BSys) * h->nsys);
  h->o_wg = take(4 * (size_t)h->pool_wgs);
  h->o_dummy = take(16);  // a zero entry (column 0, value 0) for systems without entries
  h->stage_bytes = off;  // [glob][sys][wg map][dummy] uploaded at each solve
  h->o_bar = take(4 * (size_t)h->nsys);
  // results, read back in one copy: iters, status, relres, relres_rec, clocks, abort flag
  h->res_bytes = 4 * h->total_cols * 2 + 8 * h->total_cols * 2 + 16 * (size_t)h->nsys + 8;
  h->o_res = take(h->res_bytes);
  h->o_part = take(8 * (size_t)h->pool_wgs * 4 * 4 * h->kp_max);
  h->o_vec.resize(h->nsys);
  for (int s = 0; s < h->nsys; ++s) h->o_vec[s] = take(6 * 8 * (size_t)h->n[s] * h->k[s]);
  h->bytes_needed = off;
}

// Result region offsets (relative to o_res).
size_t res_iters(const bicgstab_batched_ctx*) { return 0; }
size_t res_status(const bicgstab_batched_ctx* h) { return 4 * h->total_cols; }
size_t res_relres(const bicgstab_batched_ctx* h) { return 8 * h->total_cols; }
size_t res_relres_rec(const bicgstab_batched_ctx* h) { return 16 * h->total_cols; }
size_t res_clk(const bicgstab_batched_ctx* h) { return 24 * h->total_cols; }
size_t res_abort(const bicgstab_batched_ctx* h) { return 24 * h->total_cols + 16 * (size_t)h->nsys; }

int ensure_memory(bicgstab_batched_ctx* h) {
  if (h->base && h->bytes >= h->bytes_needed) return BICGSTAB_OK;
  if (h->base && !h->owned) return bfail(BICGSTAB_ENOMEM, "batched workspace smaller than bicgstab_batched_workspace_bytes");
  void* p = nullptr;
  BCHK(hipMalloc(&p, h->bytes_needed));
  h->base = (char*)p;
  h->bytes = h->bytes_needed;
  h->owned = true;
  return BICGSTAB_OK;
}

// Check a configuration against the kernel's assumptions: every workgroup of
// the launch must be resident at once.
int check_config(const bicgstab_batched_ctx* h, int variant, const std::vector<int>& nw) {
  if (variant < 0 || variant >= kNumVariants) return bfail(BICGSTAB_EINVAL, "unknown batched kernel variant");
  if ((int)nw.size() != h->nsys) return bfail(BICGSTAB_EINVAL, "one workgroup count per system expected");
  for (int s = 0; s < h->nsys; ++s)
    if (nw[s] < 1 || (int64_t)nw[s] > std::max<int64_t>(1, h->n[s]))
      return bfail(BICGSTAB_EINVAL, "system " + std::to_string(s) + ": workgroup count out of range");
  const int wgs = total_wgs(nw);
  if (wgs > h->cap[variant] || wgs > h->pool_wgs)
    return bfail(BICGSTAB_EUNSUPPORTED, "batched grid of " + std::to_string(wgs) +
                                            " workgroups exceeds the resident capacity (" +
                                            std::to_string(h->cap[variant]) + ")");
  return BICGSTAB_OK;
}

// One solve with the current configuration.
int run(bicgstab_batched_ctx* h, const double* const* b, double* const* x, double tol, int maxit) {
  int rc = check_config(h, h->variant, h->nw);
  if (rc) return rc;
  const int wgs = total_wgs(h->nw);
  // barrier ordinals must not wrap: (5 maxit + 3) barriers of up to nw arrivals
  for (int s = 0; s < h->nsys; ++s)
    if ((5.0 * maxit + 4.0) * h->nw[s] >= 4294967295.0)
      return bfail(BICGSTAB_EINVAL, "maxit too large for the batched barrier counters");
  rc = ensure_memory(h);
  if (rc) return rc;
  // stage: parameters, system descriptors, workgroup -> system map
  h->stage.assign(h->stage_bytes, 0);
  BGlob g;
  g.tol = tol;
  g.wait_ticks = (long long)(kBarrierWaitSeconds * h->wall_hz);
  g.maxit = maxit;
  g.nsys = h->nsys;
  g.abort_flag = (int*)(h->base + h->o_res + res_abort(h));
  std::memcpy(h->stage.data() + h->o_glob, &g, sizeof g);
  BSys* S = (BSys*)(h->stage.data() + h->o_sys);
  int32_t* wg = (int32_t*)(h->stage.data() + h->o_wg);
  char* resb = h->base + h->o_res;
  size_t col0 = 0, part0 = 0;
  int w0 = 0;
  for (int s = 0; s < h->nsys; ++s) {
    if (!b[s] || !x[s]) return bfail(BICGSTAB_EINVAL, "system " + std::to_string(s) + ": null b or x");
    const int kp = next_pow2(h->k[s]);
    BSys& d = S[s];
    d.row_ptr = h->rp[s];
    d.col = h->nnz[s] > 0 ? h->col[s] : (const int32_t*)(h->base + h->o_dummy);
    d.val = h->nnz[s] > 0 ? h->val[s] : (const double*)(h->base + h->o_dummy + 8);
    d.val_f = h->precond == BICGSTAB_PRECOND_JACOBI && h->nnz[s] > 0 ? h->val_f[s] : d.val;
    d.diag = h->precond == BICGSTAB_PRECOND_JACOBI ? h->diag[s] : nullptr;
    d.b = b[s];
    d.x = x[s];
    d.vec = (double*)(h->base + h->o_vec[s]);
    d.part = (double*)(h->base + h->o_part) + part0;
    d.out_iters = (int32_t*)(resb + res_iters(h)) + col0;
    d.out_status = (int32_t*)(resb + res_status(h)) + col0;
    d.out_relres = (double*)(resb + res_relres(h)) + col0;
    d.out_relres_rec = (double*)(resb + res_relres_rec(h)) + col0;
    d.bar = (unsigned*)(h->base + h->o_bar) + s;
    d.clk = (unsigned long long*)(resb + res_clk(h)) + 2 * s;
    d.n = (int)h->n[s];
    d.k = h->k[s];
    d.kpl = log2i(kp);
    d.nw = h->nw[s];
    d.w0 = w0;
    d.maxlen = h->maxlen[s];
    for (int q = 0; q < d.nw; ++q) wg[w0 + q] = s;
    w0 += d.nw;
    col0 += h->k[s];
    part0 += (size_t)d.nw * 4 * 4 * kp;
  }
  if (part0 > (size_t)h->pool_wgs * 4 * 4 * h->kp_max) return bfail(BICGSTAB_EINVAL, "partial pool overflow");
  BCHK(hipSetDevice(h->device));
  BCHK(hipEventRecord(h->ev, h->user_stream));
  BCHK(hipStreamWaitEvent(h->ws, h->ev, 0));
  BCHK(hipMemcpyAsync(h->base, h->stage.data(), h->stage_bytes, hipMemcpyHostToDevice, h->ws));
  if (!h->graph || h->graph_variant != h->variant || h->graph_wgs != wgs || h->graph_base != h->base) {
    if (h->graph) {
      (void)hipGraphExecDestroy(h->graph);
      h->graph = nullptr;
    }
    const BGlob* dG = (const BGlob*)(h->base + h->o_glob);
    const BSys* dS = (const BSys*)(h->base + h->o_sys);
    const int32_t* dW = (const int32_t*)(h->base + h->o_wg);
    hipGraph_t graph = nullptr;
    BCHK(hipStreamBeginCapture(h->ws, hipStreamCaptureModeThreadLocal));
    hipLaunchKernelGGL(batched_reset_kernel, dim3(1), dim3(256), 0, h->ws, (unsigned*)(h->base + h->o_bar), h->nsys,
                       g.abort_flag);
    hipError_t le = hipGetLastError();
    if (le == hipSuccess) le = launch_variant(h->variant, wgs, h->ws, dG, dS, dW);
    const hipError_t ce = hipStreamEndCapture(h->ws, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return bfail(BICGSTAB_EHIP, std::string("batched capture: ") + hipGetErrorString(le != hipSuccess ? le : ce));
    }
    const hipError_t ie = hipGraphInstantiate(&h->graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ie != hipSuccess) {
      h->graph = nullptr;
      return bfail(BICGSTAB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
    }
    h->graph_variant = h->variant;
    h->graph_wgs = wgs;
    h->graph_base = h->base;
  }
  BCHK(hipEventRecord(h->t0, h->ws));
  BCHK(hipGraphLaunch(h->graph, h->ws));
  BCHK(hipEventRecord(h->t1, h->ws));
  h->res.resize(h->res_bytes);
  BCHK(hipMemcpyAsync(h->res.data(), resb, h->res_bytes, hipMemcpyDeviceToHost, h->ws));
  BCHK(hipStreamSynchronize(h->ws));
  float ms = 0.f;
  BCHK(hipEventElapsedTime(&ms, h->t0, h->t1));
  h->last_ms = ms;
  int abort_flag = 0;
  std::memcpy(&abort_flag, h->res.data() + res_abort(h), 4);
  if (abort_flag) return bfail(BICGSTAB_EHIP, "batched kernel: a system barrier timed out");
  const int32_t* its = (const int32_t*)(h->res.data() + res_iters(h));
  const unsigned long long* clk = (const unsigned long long*)(h->res.data() + res_clk(h));
  h->sys_ms.assign(h->nsys, 0.0);
  h->sys_iters.assign(h->nsys, 0);
  col0 = 0;
  for (int s = 0; s < h->nsys; ++s) {
    h->sys_ms[s] = (double)(clk[2 * s + 1] - clk[2 * s]) / h->wall_hz * 1e3;
    int mx = 0;
    for (int c = 0; c < h->k[s]; ++c) mx = std::max(mx, its[col0 + c]);
    h->sys_iters[s] = mx;
    col0 += h->k[s];
  }
  return BICGSTAB_OK;
}

void destroy_ctx(bicgstab_batched_ctx* h) {
  if (h->ws) (void)hipStreamSynchronize(h->ws);
  if (h->graph) (void)hipGraphExecDestroy(h->graph);
  if (h->owned && h->base) (void)hipFree(h->base);
  if (h->jac) (void)hipFree(h->jac);
  if (h->ws) (void)hipStreamDestroy(h->ws);
  for (hipEvent_t e : {h->ev, h->t0, h->t1})
    if (e) (void)hipEventDestroy(e);
  delete h;
}

// Jacobi set-up: every system's diagonal (a zero entry is an error) and its
// Jacobi-folded values A M^{-1}, one division per entry, as the single-system
// path forms them.
int build_jacobi(bicgstab_batched_ctx* h) {
  size_t total = 256;  // a zero-diagonal counter first
  std::vector<size_t> od(h->nsys), of(h->nsys);
  for (int s = 0; s < h->nsys; ++s) {
    od[s] = total;
    total += ((size_t)h->n[s] * 8 + 255) / 256 * 256;
    of[s] = total;
    total += ((size_t)h->nnz[s] * 8 + 255) / 256 * 256;
  }
  if (hipMalloc((void**)&h->jac, total) != hipSuccess) {
    h->jac = nullptr;
    (void)hipGetLastError();
    return bfail(BICGSTAB_ENOMEM, "Jacobi set-up: device allocation failed");
  }
  Globals* g = (Globals*)h->jac;
  BCHK(hipMemsetAsync(g, 0, sizeof(Globals), h->ws));
  for (int s = 0; s < h->nsys; ++s) {
    double* d = (double*)(h->jac + od[s]);
    double* f = (double*)(h->jac + of[s]);
    h->diag.push_back(d);
    h->val_f.push_back(f);
    BCHK(launch_extract_diag(h->rp[s], h->col[s], h->val[s], d, nullptr, (int)h->n[s], g, h->ws));
    BCHK(launch_fold_jacobi(h->col[s], h->val[s], d, f, nullptr, h->nnz[s], h->ws));
  }
  Globals hg;
  BCHK(hipMemcpyAsync(&hg, g, sizeof hg, hipMemcpyDeviceToHost, h->ws));
  BCHK(hipStreamSynchronize(h->ws));
  if (hg.zero_diag > 0)
    return bfail(BICGSTAB_EINVAL, "Jacobi preconditioner: " + std::to_string(hg.zero_diag) + " zero diagonal entries");
  return BICGSTAB_OK;
}

}  // namespace

extern "C" {

int bicgstab_batched_create(const bicgstab_csr* As, const int32_t* ks, int32_t nsys, int32_t variant,
                            int32_t precond, void* stream, bicgstab_batched_t* out) {
  if (!As || !ks || !out || nsys < 1) return bfail(BICGSTAB_EINVAL, "null argument or no systems");
  *out = nullptr;
  if (variant < BICGSTAB_CLASSICAL || variant > BICGSTAB_IMPROVED ||
      (precond != BICGSTAB_PRECOND_NONE && precond != BICGSTAB_PRECOND_JACOBI))
    return bfail(BICGSTAB_EINVAL, "unknown variant or preconditioner");
  if (variant != BICGSTAB_CLASSICAL)
    return bfail(BICGSTAB_EUNSUPPORTED, "the batched kernel runs the classical method only");
  auto* h = new bicgstab_batched_ctx();
  h->nsys = nsys;
  h->precond = precond;
  h->user_stream = (hipStream_t)stream;
  for (int s = 0; s < nsys; ++s) {
    const bicgstab_csr& A = As[s];
    // element offsets of the n x k blocks and of the CSR arrays are 32-bit
    // byte offsets in the kernel, and row indices go through 24-bit multiplies
    if (A.n < 1 || A.n >= ((int64_t)1 << 24) || A.nnz < 0 || A.nnz >= ((int64_t)1 << 29) || ks[s] < 1 ||
        ks[s] > BICGSTAB_MAX_K || A.n * (int64_t)ks[s] * 8 >= ((int64_t)1 << 31) || !A.d_row_ptr ||
        (A.nnz > 0 && (!A.d_col_idx || !A.d_values))) {
      destroy_ctx(h);
      return bfail(BICGSTAB_EINVAL, "system " + std::to_string(s) +
                                        ": invalid matrix or k (n >= 2^24, nnz >= 2^29 or n*k*8 >= 2^31)");
    }
    // validate the pattern on the host: no kernel may index out of bounds
    std::vector<int32_t> rp((size_t)A.n + 1), cols((size_t)A.nnz);
    if (hipMemcpy(rp.data(), A.d_row_ptr, rp.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        (A.nnz > 0 && hipMemcpy(cols.data(), A.d_col_idx, cols.size() * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
      destroy_ctx(h);
      return bfail(BICGSTAB_EHIP, "reading a batched matrix failed");
    }
    bool ok = rp[0] == 0 && rp[A.n] == A.nnz;
    for (int64_t i = 0; ok && i < A.n; ++i) ok = rp[i + 1] >= rp[i];
    for (int32_t cc : cols) ok = ok && cc >= 0 && cc < A.n;
    if (!ok) {
      destroy_ctx(h);
      return bfail(BICGSTAB_EINVAL, "system " + std::to_string(s) + ": malformed CSR");
    }
    h->n.push_back(A.n);
    h->nnz.push_back(A.nnz);
    int ml = 0;
    for (int64_t i = 0; i < A.n; ++i) ml = std::max(ml, rp[i + 1] - rp[i]);
    h->maxlen.push_back(ml);
    h->k.push_back(ks[s]);
    h->rp.push_back(A.d_row_ptr);
    h->col.push_back(A.d_col_idx);
    h->val.push_back(A.d_values);
    h->total_cols += ks[s];
    h->kp_max = std::max(h->kp_max, next_pow2(ks[s]));
  }
  hipDeviceProp_t prop;
  int wall_khz = 0;
  if (hipGetDevice(&h->device) != hipSuccess || hipGetDeviceProperties(&prop, h->device) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, h->device) != hipSuccess ||
      hipStreamCreateWithFlags(&h->ws, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev, hipEventDisableTiming) != hipSuccess || hipEventCreate(&h->t0) != hipSuccess ||
      hipEventCreate(&h->t1) != hipSuccess) {
    destroy_ctx(h);
    return bfail(BICGSTAB_EHIP, "device set-up failed");
  }
  if (wall_khz > 0) h->wall_hz = 1e3 * wall_khz;
  h->cus = prop.multiProcessorCount;
  if (precond == BICGSTAB_PRECOND_JACOBI) {
    const int rc = build_jacobi(h);
    if (rc) {
      destroy_ctx(h);
      return rc;
    }
  }
  for (int v = 0; v < kNumVariants; ++v) {
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel_of(v), kVariants[v].block, 0) != hipSuccess) {
      destroy_ctx(h);
      return bfail(BICGSTAB_EHIP, "occupancy query failed");
    }
    h->cap[v] = per * h->cus;
    h->pool_wgs = std::max(h->pool_wgs, h->cap[v]);
  }
  h->variant = 1;
  if (h->cap[h->variant] < nsys) {
    destroy_ctx(h);
    return bfail(BICGSTAB_EUNSUPPORTED, "more systems than resident workgroups");
  }
  compute_layout(h);
  // starting configuration: the whole resident capacity, shares by bytes x a
  // pass estimate that grows with the system size
  std::vector<double> est(nsys);
  for (int s = 0; s < nsys; ++s) est[s] = 2.0 * std::pow((double)h->n[s], 0.4);
  h->nw = proportional(h, h->cap[h->variant], est);
  *out = h;
  return BICGSTAB_OK;
}

int bicgstab_batched_workspace_bytes(bicgstab_batched_t h, size_t* bytes) {
  if (!h || !bytes) return bfail(BICGSTAB_EINVAL, "null argument");
  *bytes = h->bytes_needed;
  return BICGSTAB_OK;
}

int bicgstab_batched_set_workspace(bicgstab_batched_t h, void* d_ptr, size_t bytes) {
  if (!h || !d_ptr) return bfail(BICGSTAB_EINVAL, "null argument");
  if (((uintptr_t)d_ptr & 255) != 0) return bfail(BICGSTAB_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < h->bytes_needed) return bfail(BICGSTAB_ENOMEM, "workspace smaller than bicgstab_batched_workspace_bytes");
  if (h->owned && h->base) {
    (void)hipStreamSynchronize(h->ws);
    (void)hipFree(h->base);
  }
  h->base = (char*)d_ptr;
  h->bytes = bytes;
  h->owned = false;
  return BICGSTAB_OK;
}

int bicgstab_batched_set_stream(bicgstab_batched_t h, void* stream) {
  if (!h) return bfail(BICGSTAB_EINVAL, "null handle");
  h->user_stream = (hipStream_t)stream;
  return BICGSTAB_OK;
}

int bicgstab_batched_solve(bicgstab_batched_t h, const double* const* d_b, double* const* d_x, double tol,
                           int32_t maxit, bicgstab_info* info) {
  if (!h || !d_b || !d_x) return bfail(BICGSTAB_EINVAL, "null argument");
  if (maxit < 0) return bfail(BICGSTAB_EINVAL, "maxit < 0");
  const int rc = run(h, d_b, d_x, tol, maxit);
  if (rc) return rc;
  if (info) {
    const size_t tc = h->total_cols;
    const char* r = h->res.data();
    if (info->iters) std::memcpy(info->iters, r + res_iters(h), 4 * tc);
    if (info->status) std::memcpy(info->status, r + res_status(h), 4 * tc);
    if (info->relres_true) std::memcpy(info->relres_true, r + res_relres(h), 8 * tc);
    if (info->relres_recursive) std::memcpy(info->relres_recursive, r + res_relres_rec(h), 8 * tc);
  }
  return BICGSTAB_OK;
}

int bicgstab_batched_tune(bicgstab_batched_t h, const double* const* d_b, double* const* d_x, double tol,
                          int32_t maxit, double* best_ms) {
  if (!h || !d_b || !d_x) return bfail(BICGSTAB_EINVAL, "null argument");
  if (maxit < 0) return bfail(BICGSTAB_EINVAL, "maxit < 0");
  for (int s = 0; s < h->nsys; ++s)
    if (!d_x[s] || !d_b[s]) return bfail(BICGSTAB_EINVAL, "system " + std::to_string(s) + ": null b or x");
  // the caller's initial guesses are restored before every trial
  std::vector<size_t> xb(h->nsys);
  size_t tot = 0;
  for (int s = 0; s < h->nsys; ++s) tot += xb[s] = 8 * (size_t)h->n[s] * h->k[s];
  void* save = nullptr;
  BCHK(hipSetDevice(h->device));
  BCHK(hipMalloc(&save, tot));
  auto copy_x = [&](bool to_save) -> int {
    size_t off = 0;
    for (int s = 0; s < h->nsys; ++s) {
      char* sv = (char*)save + off;
      if (to_save) BCHK(hipMemcpyAsync(sv, d_x[s], xb[s], hipMemcpyDeviceToDevice, h->ws));
      else BCHK(hipMemcpyAsync(d_x[s], sv, xb[s], hipMemcpyDeviceToDevice, h->ws));
      off += xb[s];
    }
    BCHK(hipStreamSynchronize(h->ws));
    return BICGSTAB_OK;
  };
  int rc = BICGSTAB_OK;
  if (hipEventRecord(h->ev, h->user_stream) != hipSuccess || hipStreamWaitEvent(h->ws, h->ev, 0) != hipSuccess)
    rc = bfail(BICGSTAB_EHIP, "stream ordering failed");
  if (!rc) rc = copy_x(true);
  double best = 1e300;
  int best_variant = h->variant;
  std::vector<int> best_nw = h->nw;
  auto trial = [&]() -> int {
    int r = copy_x(false);
    if (r) return r;
    r = run(h, d_b, d_x, tol, maxit);
    if (r) return r;
    if (h->last_ms < best) {
      best = h->last_ms;
      best_variant = h->variant;
      best_nw = h->nw;
    }
    return BICGSTAB_OK;
  };
  // allocation for one (variant, budget): shares by measured work, then twice
  // from the time model fitted to the run before
  auto tune_allocation = [&](int v, int budget) -> int {
    if (budget < h->nsys) return BICGSTAB_OK;
    std::vector<double> passes(h->sys_iters.begin(), h->sys_iters.end());
    h->variant = v;
    h->nw = proportional(h, budget, passes);
    int r = trial();
    for (int round = 0; round < 2 && !r; ++round) {
      h->nw = model_allocation(h, budget);
      r = trial();
    }
    return r;
  };
  // a first run measures pass counts and per-system times
  if (!rc) rc = trial();
  // every variant at its full resident capacity
  for (int v = 0; v < kNumVariants && !rc; ++v) rc = tune_allocation(v, h->cap[v]);
  // the best variant at smaller budgets, until one is not faster
  const int bv = best_variant;
  for (int div : {2, 4}) {
    if (rc) break;
    const double before = best;
    rc = tune_allocation(bv, h->cap[bv] / div);
    if (!(best < before)) break;
  }
  // the best allocation thinned: every system on 1/2 .. 1/16 of its
  // workgroups (at least one), until a thinning is not faster. A pass's
  // barriers cost more the more workgroups they join, so a system whose
  // passes are short can finish sooner on fewer (a 4,096-row system alone:
  // 18.5 us per pass on 8 workgroups, 41.5 on the 64 its row count allows);
  // a batch of large systems only slows down (and 1/16 of its workgroups
  // would take seconds)
  const std::vector<int> base = best_nw;
  const int base_variant = best_variant;
  for (int div : {2, 4, 8, 16}) {
    if (rc) break;
    h->variant = base_variant;
    bool changed = false;
    for (int s = 0; s < h->nsys; ++s) {
      h->nw[s] = std::max(1, base[s] / div);
      changed |= h->nw[s] != base[s];
    }
    if (!changed) break;
    const double before = best;
    rc = trial();
    if (!(best < before)) break;
  }
  h->variant = best_variant;
  h->nw = best_nw;
  // leave the best configuration's solution in x
  if (!rc) rc = trial();
  (void)hipFree(save);
  if (rc) return rc;
  if (best_ms) *best_ms = best;
  return BICGSTAB_OK;
}

int bicgstab_batched_get_config(bicgstab_batched_t h, int32_t* variant, int32_t* block, int32_t* workgroups,
                                double* last_ms, double* system_ms) {
  if (!h) return bfail(BICGSTAB_EINVAL, "null handle");
  if (variant) *variant = h->variant;
  if (block) *block = kVariants[h->variant].block;
  for (int s = 0; s < h->nsys; ++s) {
    if (workgroups) workgroups[s] = h->nw[s];
    if (system_ms) system_ms[s] = s < (int)h->sys_ms.size() ? h->sys_ms[s] : 0.0;
  }
  if (last_ms) *last_ms = h->last_ms;
  return BICGSTAB_OK;
}

int bicgstab_batched_set_config(bicgstab_batched_t h, int32_t variant, const int32_t* workgroups) {
  if (!h || !workgroups) return bfail(BICGSTAB_EINVAL, "null argument");
  std::vector<int> nw(workgroups, workgroups + h->nsys);
  const int rc = check_config(h, variant, nw);
  if (rc) return rc;
  h->variant = variant;
  h->nw = nw;
  return BICGSTAB_OK;
}

int bicgstab_batched_variant_info(int32_t variant, int32_t* block, int32_t* rows_per_step,
                                  int32_t* entries_per_step, int32_t* product_rows_per_step) {
  if (variant < 0 || variant >= kNumVariants) return bfail(BICGSTAB_EINVAL, "unknown batched kernel variant");
  if (block) *block = kVariants[variant].block;
  if (rows_per_step) *rows_per_step = kVariants[variant].rows;
  if (entries_per_step) *entries_per_step = kVariants[variant].entries;
  if (product_rows_per_step) *product_rows_per_step = kVariants[variant].product_rows;
  return BICGSTAB_OK;
}

int bicgstab_batched_destroy(bicgstab_batched_t h) {
  if (!h) return BICGSTAB_OK;
  (void)hipSetDevice(h->device);
  destroy_ctx(h);
  return BICGSTAB_OK;
}

}  // extern "C"
