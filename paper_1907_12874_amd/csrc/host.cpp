// Host-CPU executor of the launch plans (libbicgstab_host.so).
//
// The paper measured the effect of merging vector operations on CPU nodes
// (Section 3.1.3, Table 4). This executor runs the GPU library's own launch
// plans (plans.cpp: one step = one memory pass over n x k row-major blocks,
// grouped as in the Merged or Basic column of Table 2) on the host's cores,
// with the GPU library's own per-element bodies and per-column scalar steps
// (method.hpp), so merged and basic forms can be timed on the host exactly as
// they are on the GPU. Each pass is one OpenMP parallel region over T fixed
// contiguous row ranges; dot products are summed per range in row order and
// then over the ranges in order, so a solve is bitwise repeatable for a given
// T. FP64 only.
#include <omp.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <memory>
#include <string>
#include <vector>

#include "../../include/bicgstab_host.h"
#include "method.hpp"
#include "plan.hpp"

namespace {

using namespace bcg;

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

struct bicgstab_host_ctx {
  int64_t n = 0;
  int k = 0;
  int variant = 0, formulation = 0, precond = 0;
  int threads = 1;
  std::vector<int32_t> rp, col;
  std::vector<double> val;
  std::vector<double> val_fold;  // A M^{-1} (Jacobi folded into the values), when a plan step needs it
  std::vector<int32_t> rpt, colt;  // A^T (Improved BiCGStab's f0 = A^T r0)
  std::vector<double> valt;
  std::vector<double> diag;
  Plan plan;
  std::vector<std::vector<double>> store;  // one n x k block per plan vector
  double* vec[V_NUM] = {};
  std::vector<double> sc;
  std::vector<int> ist;
  Globals glob{};
  std::vector<double> red;  // per-range dot partials: threads x 7 x k
  Ctl ctl{};
  double loop_seconds = 0.0;  // wall time of the last solve's iteration loop
  int loop_passes = 0;        // passes that loop ran
};

namespace {

typedef bicgstab_host_ctx Ctx;

// Rows of range t of T: [n t / T, n (t + 1) / T).
inline int64_t range_begin(int64_t n, int t, int T) { return n * t / T; }

// Runs body(t, r0, r1) for every row range t of T on the OpenMP team (a
// thread takes ranges tid, tid + nth, ... if the team is smaller than T).
template <class F>
void for_ranges(const Ctx& h, F&& body) {
  const int T = h.threads;
  const int64_t n = h.n;
#pragma omp parallel num_threads(T)
  {
    const int nth = omp_get_num_threads(), tid = omp_get_thread_num();
    for (int t = tid; t < T; t += nth) body(t, range_begin(n, t, T), range_begin(n, t + 1, T));
  }
}

// Dot slots slot.. of every column from the per-range partials (ranges in
// order, each summed from 0), then the scalar step fin.
void finish_dots(Ctx& h, int ndot, int slot, int fin) {
  const int k = h.k;
  for (int d = 0; d < ndot; ++d)
    for (int c = 0; c < k; ++c) {
      double s = 0.0;
      for (int t = 0; t < h.threads; ++t) s += h.red[((size_t)t * 7 + d) * k + c];
      h.sc[(size_t)(S_D0 + slot + d) * kMaxK + c] = s;
    }
  if (fin != F_NONE) {
    for (int c = 0; c < k; ++c) finalize_column(fin, c, h.ctl);
    finalize_global(fin, h.ctl);
  }
}

// Y = A X over all columns, each row's entries in stored order.
void spmm(const Ctx& h, const std::vector<int32_t>& rp, const std::vector<int32_t>& col,
          const std::vector<double>& val, const double* X, double* Y) {
  const int k = h.k;
  for_ranges(h, [&](int, int64_t r0, int64_t r1) {
    double acc[kMaxK];
    for (int64_t i = r0; i < r1; ++i) {
      for (int c = 0; c < k; ++c) acc[c] = 0.0;
      for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
        const double a = val[e];
        const double* xr = X + (size_t)col[e] * k;
        for (int c = 0; c < k; ++c) acc[c] += a * xr[c];
      }
      double* yr = Y + (size_t)i * k;
      for (int c = 0; c < k; ++c) yr[c] = acc[c];
    }
  });
}

// The product with an epilogue: the dots (y, w), or (y, w), (y, y), (w, w),
// or (y, x), (y, y), (y, w), (x, x), and / or the Jacobi-scaled copy
// yh = y / a_ii.
void spmm_dot(Ctx& h, const double* X, double* Y, const double* W, double* Yh, int epi, int slot, int fin,
              bool fold) {
  const int k = h.k;
  const std::vector<double>& val = fold ? h.val_fold : h.val;
  const int nd = epilogue_dots(epi);
  const bool scaled = epilogue_prec(epi);
  for_ranges(h, [&](int t, int64_t r0, int64_t r1) {
    double acc[kMaxK];
    double* part = &h.red[(size_t)t * 7 * k];
    for (int i = 0; i < nd * k; ++i) part[i] = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      for (int c = 0; c < k; ++c) acc[c] = 0.0;
      for (int32_t e = h.rp[i]; e < h.rp[i + 1]; ++e) {
        const double a = val[e];
        const double* xr = X + (size_t)h.col[e] * k;
        for (int c = 0; c < k; ++c) acc[c] += a * xr[c];
      }
      double* yr = Y + (size_t)i * k;
      for (int c = 0; c < k; ++c) yr[c] = acc[c];
      if (scaled)
        for (int c = 0; c < k; ++c) Yh[(size_t)i * k + c] = acc[c] / h.diag[i];
      if (epi == E_RE4) {
        // (y, x), (y, y), (y, w), (x, x) with x at the row itself
        const double* wr = W + (size_t)i * k;
        const double* xr = X + (size_t)i * k;
        for (int c = 0; c < k; ++c) {
          part[c] += acc[c] * xr[c];
          part[k + c] += acc[c] * acc[c];
          part[2 * k + c] += acc[c] * wr[c];
          part[3 * k + c] += xr[c] * xr[c];
        }
      } else if (nd > 0) {
        const double* wr = W + (size_t)i * k;
        for (int c = 0; c < k; ++c) {
          part[c] += acc[c] * wr[c];
          if (nd == 3) {
            part[k + c] += acc[c] * acc[c];
            part[2 * k + c] += wr[c] * wr[c];
          }
        }
      }
    }
  });
  if (nd > 0 || fin != F_NONE) finish_dots(h, nd, slot, fin);
}

void prec(const Ctx& h, const double* in, double* out) {
  const int k = h.k;
  for_ranges(h, [&](int, int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i)
      for (int c = 0; c < k; ++c) out[(size_t)i * k + c] = in[(size_t)i * k + c] / h.diag[i];
  });
}

inline double& SCh(Ctx& h, int slot, int c) { return h.sc[(size_t)slot * kMaxK + c]; }
inline int& ISh(Ctx& h, int slot, int c) { return h.ist[(size_t)slot * kMaxK + c]; }

// One vector pass of op Op: the columns that take part get the op's body on
// every row; its dots go to slots slot..; then the scalar step fin.
template <class Op>
void group(Ctx& h, const Step& st, double* const* vp) {
  if (Op::EARLY && h.glob.nrun == 0) return;
  const int k = h.k;
  bool on[kMaxK];
  unsigned wmask[kMaxK];
  Coef cf[kMaxK];
  for (int c = 0; c < k; ++c) {
    on[c] = true;
    // outputs in COUT are written only where the column restarts
    wmask[c] = Op::COUT == 0u || ISh(h, I_RESTART, c) != 0 ? ~0u : ~Op::COUT;
    if (Op::PART == PART_RUN) on[c] = ISh(h, I_STATUS, c) == ST_RUNNING;
    if (Op::PART == PART_ZEROB) on[c] = ISh(h, I_ZEROB, c) != 0;
    cf[c].alpha = SCh(h, S_ALPHA, c);
    cf[c].omega = SCh(h, S_OMEGA, c);
    cf[c].beta = SCh(h, S_BETA, c);
    cf[c].scale = SCh(h, S_SCALE, c);
    cf[c].delta = SCh(h, S_DELTA, c);
    cf[c].c1 = SCh(h, S_C1, c);
    cf[c].c2 = SCh(h, S_C2, c);
  }
  const double* in[kMaxPassIn] = {};
  double* out[kMaxPassOut] = {};
  for (int i = 0; i < Op::NIN; ++i) in[i] = vp[st.in[i]];
  for (int j = 0; j < Op::NOUT; ++j) out[j] = vp[st.out[j]];
  constexpr int NI = Op::NIN + (Op::USE_D ? 1 : 0) > 0 ? Op::NIN + (Op::USE_D ? 1 : 0) : 1;
  constexpr int NO = Op::NOUT > 0 ? Op::NOUT : 1;
  constexpr int ND = Op::NDOT > 0 ? Op::NDOT : 1;
  for_ranges(h, [&](int t, int64_t r0, int64_t r1) {
    double* part = &h.red[(size_t)t * 7 * k];
    double acc[kMaxK][ND];
    for (int c = 0; c < k; ++c)
      for (int d = 0; d < ND; ++d) acc[c][d] = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
      for (int c = 0; c < k; ++c) {
        if (!on[c]) continue;
        const size_t e = (size_t)i * k + c;
        double v[NI], o[NO];
        for (int q = 0; q < Op::NIN; ++q) v[q] = in[q][e];
        if (Op::USE_D) v[Op::NIN] = h.diag[i];
        Op::template f<double>(v, cf[c], o, acc[c]);
        for (int j = 0; j < Op::NOUT; ++j)
          if ((wmask[c] >> j) & 1) out[j][e] = o[j];
      }
    }
    if (Op::NDOT > 0)
      for (int d = 0; d < Op::NDOT; ++d)
        for (int c = 0; c < k; ++c) part[(size_t)d * k + c] = acc[c][d];
  });
  if (Op::NDOT > 0 || st.fin != F_NONE) finish_dots(h, Op::NDOT, st.slot, st.fin);
}

int run_group(Ctx& h, const Step& st, double* const* vp) {
  switch (st.op) {
#define G(ID, OP) \
  case ID: group<OP>(h, st, vp); return BICGSTAB_OK;
    G(OP_INIT, KInit)
    G(OP_INIT_P, KInitP)
    G(OP_ZEROB, KZeroB)
    G(OP_COPY, KCopy)
    G(OP_FILL0, KFill0)
    G(OP_EXIT, KExit)
    G(OP_DOT, KDot)
    G(OP_DOTSELF, KDotSelf)
    G(OP_SUB_ALPHA, KSubAlpha)
    G(OP_SUB_OMEGA, KSubOmega)
    G(OP_XUPD, KXUpd)
    G(OP_PUPD, KPUpd)
    G(OP_C_PPT, KCPpt)
    G(OP_C_XR_RHO, KCXrRho)
    G(OP_C_R_RHO, KCRRho)
    G(OP_R_G3, KRG3)
    G(OP_R_XZV, KRXzv)
    G(OP_P_G1, KPG1)
    G(OP_P_G2, KPG2)
    G(OP_P_G3, KPG3)
    G(OP_PP_G12, KPPG12)
    G(OP_PP_G34, KPPG34)
    G(OP_F_SUB_ALPHA_H, KFSubAlphaH)
    G(OP_F_PUPD_H, KFPUpdH)
    G(OP_F_XR_RHO_H, KFXrRhoH)
    G(OP_IB_INIT, KIbInit)
    G(OP_IB_G1, KIbG1)
    G(OP_IB_G2, KIbG2)
    G(OP_IB_G3, KIbG3)
    G(OP_IB_Z, KIbZ)
    G(OP_IB_V, KIbV)
    G(OP_IB_X, KIbX)
    G(OP_RE_R, KReR)
    G(OP_F_XR_RHO_D, KFXrRhoD)
    G(OP_F_P_G23, KFPG23)
    G(OP_F_P_G23D, KFPG23D)
    G(OP_F_RE_XVD, KFReXvD)
    G(OP_F_RE_XV, KFReXv)
    G(OP_R_DOTS, KRDots)
#undef G
    default: return fail(BICGSTAB_EINVAL, "host executor: op not available on the host");
  }
}

int run_step(Ctx& h, const Step& st, double* const* vp, bool early_exit = true) {
  if (early_exit && h.glob.nrun == 0 && st.kind != K_GROUP) return BICGSTAB_OK;
  switch (st.kind) {
    case K_SPMM: spmm(h, h.rp, h.col, st.fold ? h.val_fold : h.val, vp[st.in[0]], vp[st.out[0]]); return BICGSTAB_OK;
    case K_SPMM_T: spmm(h, h.rpt, h.colt, h.valt, vp[st.in[0]], vp[st.out[0]]); return BICGSTAB_OK;
    case K_SPMM_DOT:
      spmm_dot(h, vp[st.in[0]], vp[st.out[0]], epilogue_dots(st.op) > 0 ? vp[st.in[1]] : nullptr,
               epilogue_prec(st.op) ? vp[st.out[1]] : nullptr, st.op, st.slot, st.fin, st.fold != 0);
      return BICGSTAB_OK;
    case K_PREC: prec(h, vp[st.in[0]], vp[st.out[0]]); return BICGSTAB_OK;
    case K_GROUP: return run_group(h, st, vp);
  }
  return fail(BICGSTAB_EINVAL, "host executor: unknown step");
}

// A^T in CSR with each row's entries in increasing column order (the rows of
// A are visited in order).
void build_transpose(Ctx& h) {
  const int64_t n = h.n;
  const size_t nnz = h.col.size();
  h.rpt.assign(n + 1, 0);
  for (size_t e = 0; e < nnz; ++e) ++h.rpt[h.col[e] + 1];
  for (int64_t i = 0; i < n; ++i) h.rpt[i + 1] += h.rpt[i];
  std::vector<int32_t> cur(h.rpt.begin(), h.rpt.end() - 1);
  h.colt.resize(nnz);
  h.valt.resize(nnz);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = h.rp[i]; e < h.rp[i + 1]; ++e) {
      const int32_t p = cur[h.col[e]]++;
      h.colt[p] = (int32_t)i;
      h.valt[p] = h.val[e];
    }
}

}  // namespace

extern "C" {

int bicgstab_host_create(const bicgstab_host_csr* A, int32_t k, int32_t variant, int32_t formulation,
                         int32_t precond, int32_t threads, bicgstab_host_t* out) {
  if (!A || !out) return fail(BICGSTAB_EINVAL, "null argument");
  *out = nullptr;
  if (A->n < 0 || A->n > INT32_MAX || A->nnz < 0 || A->nnz > INT32_MAX)
    return fail(BICGSTAB_EINVAL, "matrix size out of range");
  if (k < 1 || k > kMaxK) return fail(BICGSTAB_EINVAL, "k must be in [1, 64]");
  if (threads < 1 || threads > 1024) return fail(BICGSTAB_EINVAL, "threads must be in [1, 1024]");
  if (A->n > 0 && (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->values))))
    return fail(BICGSTAB_EINVAL, "null matrix array");
  if (formulation == BICGSTAB_FUSED && variant == BICGSTAB_IMPROVED)
    return fail(BICGSTAB_EUNSUPPORTED, "the fused formulation is not built for Improved BiCGStab");
  if (variant == BICGSTAB_IMPROVED && precond != BICGSTAB_PRECOND_NONE)
    return fail(BICGSTAB_EUNSUPPORTED, "Improved BiCGStab has no preconditioned form");
  std::unique_ptr<Ctx> h(new Ctx);
  std::string err;
  if (!build_plan(variant, formulation, precond, k, &h->plan, &err)) return fail(BICGSTAB_EINVAL, err);
  h->n = A->n;
  h->k = k;
  h->variant = variant;
  h->formulation = formulation;
  h->precond = precond;
  h->threads = threads;
  const int64_t n = A->n;
  h->rp.assign(n + 1, 0);
  if (n > 0) memcpy(h->rp.data(), A->row_ptr, (size_t)(n + 1) * 4);
  if (h->rp[0] != 0 || h->rp[n] != A->nnz) return fail(BICGSTAB_EINVAL, "row_ptr must run from 0 to nnz");
  for (int64_t i = 0; i < n; ++i)
    if (h->rp[i + 1] < h->rp[i]) return fail(BICGSTAB_EINVAL, "row_ptr must be non-decreasing");
  h->col.assign(A->col_idx, A->col_idx + A->nnz);
  h->val.assign(A->values, A->values + A->nnz);
  for (int32_t c : h->col)
    if (c < 0 || c >= n) return fail(BICGSTAB_EINVAL, "column index out of range");
  if (precond == BICGSTAB_PRECOND_JACOBI) {
    h->diag.assign(n, 0.0);
    int64_t zero = 0;
    for (int64_t i = 0; i < n; ++i) {
      double d = 0.0;
      for (int32_t e = h->rp[i]; e < h->rp[i + 1]; ++e)
        if (h->col[e] == i) d += h->val[e];
      h->diag[i] = d;
      zero += d == 0.0;
    }
    if (precond == BICGSTAB_PRECOND_JACOBI && zero > 0)
      return fail(BICGSTAB_EINVAL, "Jacobi preconditioner: " + std::to_string(zero) + " zero diagonal entries");
  }
  bool need_t = false, need_fold = false;
  for (const auto* list : {&h->plan.init, &h->plan.iter})
    for (const Step& s : *list) {
      need_t |= s.kind == K_SPMM_T;
      need_fold |= s.fold != 0;
    }
  if (need_fold) {
    // A M^{-1}: entry (i, j) is a_ij / a_jj
    h->val_fold.resize(h->val.size());
    for (size_t e = 0; e < h->val.size(); ++e) h->val_fold[e] = h->val[e] / h->diag[h->col[e]];
  }
  if (need_t) build_transpose(*h);
  const size_t nk = (size_t)n * k;
  for (int v : h->plan.vecs) {
    h->store.emplace_back(std::max<size_t>(nk, 1), 0.0);
    h->vec[v] = h->store.back().data();
  }
  for (int v = 0; v < V_NUM; ++v)
    if (h->plan.alias_from[v] >= 0) h->vec[v] = h->vec[h->plan.alias_from[v]];
  if (!h->vec[V_V]) {
    h->store.emplace_back(std::max<size_t>(nk, 1), 0.0);  // the exit product's output
    h->vec[V_V] = h->store.back().data();
  }
  h->sc.assign((size_t)S_NSCAL * kMaxK, 0.0);
  h->ist.assign((size_t)I_NINT * kMaxK, 0);
  h->red.assign((size_t)threads * 7 * k, 0.0);
  h->ctl.sc = h->sc.data();
  h->ctl.ist = h->ist.data();
  h->ctl.glob = &h->glob;
  h->ctl.partials = nullptr;
  h->ctl.hist = nullptr;
  h->ctl.k = k;
  *out = h.release();
  return BICGSTAB_OK;
}

int bicgstab_host_solve(bicgstab_host_t h, const double* b, double* x, double tol, int32_t maxit,
                        bicgstab_info* info) {
  if (!h) return fail(BICGSTAB_EINVAL, "null handle");
  if (h->n > 0 && (!b || !x)) return fail(BICGSTAB_EINVAL, "null b or x");
  if (!(tol >= 0.0)) return fail(BICGSTAB_EINVAL, "tol must be >= 0");
  const int k = h->k;
  double* vp[V_NUM];
  for (int v = 0; v < V_NUM; ++v) vp[v] = h->vec[v];
  vp[V_X] = x;
  vp[V_B] = const_cast<double*>(b);
  // per-solve state, as the GPU's set-up kernel writes it
  for (int c = 0; c < k; ++c) {
    ISh(*h, I_STATUS, c) = ST_RUNNING;
    ISh(*h, I_PEND, c) = -1;
    ISh(*h, I_ITERS, c) = 0;
    ISh(*h, I_ZEROB, c) = 0;
  }
  h->glob = Globals{};
  h->glob.nrun = k;
  h->glob.maxit = maxit;
  h->glob.tol = tol;
  int rc = BICGSTAB_OK;
  h->loop_seconds = 0.0;
  h->loop_passes = 0;
  if (h->n > 0) {
    for (const Step& st : h->plan.init)
      if ((rc = run_step(*h, st, vp))) return rc;
    if (maxit <= 0) {
      for (int c = 0; c < k; ++c)
        if (ISh(*h, I_STATUS, c) == ST_RUNNING) {
          ISh(*h, I_STATUS, c) = ST_MAXIT;
          ISh(*h, I_ITERS, c) = 0;
        }
      h->glob.nrun = 0;
    } else {
      const auto t0 = std::chrono::steady_clock::now();
      int64_t pass = 0;
      for (; h->glob.nrun > 0; ++pass) {
        if (pass > (int64_t)maxit + 2) return fail(BICGSTAB_EINVAL, "iteration counter did not reach maxit");
        for (const Step& st : h->plan.iter)
          if ((rc = run_step(*h, st, vp))) return rc;
      }
      h->loop_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
      h->loop_passes = (int)pass;
    }
    // exit: true residual b - A x and ||r|| for every column
    spmm(*h, h->rp, h->col, h->val, x, vp[V_V]);
    Step ex{};
    ex.kind = K_GROUP;
    ex.op = OP_EXIT;
    ex.in[0] = V_B;
    ex.in[1] = V_V;
    ex.in[2] = V_R;
    ex.nin = 3;
    ex.slot = 0;
    ex.fin = F_EXIT;
    if ((rc = run_group(*h, ex, vp))) return rc;
  } else {
    for (int c = 0; c < k; ++c) ISh(*h, I_STATUS, c) = ST_CONVERGED;
  }
  if (info)
    for (int c = 0; c < k; ++c) {
      if (info->iters) info->iters[c] = ISh(*h, I_ITERS, c);
      if (info->status) info->status[c] = ISh(*h, I_STATUS, c);
      if (info->relres_true) info->relres_true[c] = h->n > 0 ? SCh(*h, S_RELRES_TRUE, c) : 0.0;
      if (info->relres_recursive) info->relres_recursive[c] = h->n > 0 ? SCh(*h, S_RELRES_REC, c) : 0.0;
    }
  return BICGSTAB_OK;
}

int bicgstab_host_axpby_tab1(int32_t run, int64_t n, double a, double b, double c, const double* x, double* y,
                             double* z, int32_t threads) {
  if (run < 1 || run > 3) return fail(BICGSTAB_EINVAL, "run must be 1, 2 or 3");
  if (n < 0) return fail(BICGSTAB_EINVAL, "n must be >= 0");
  if (n > 0 && (!x || !y || !z)) return fail(BICGSTAB_EINVAL, "null vector");
  if (threads < 1 || threads > 1024) return fail(BICGSTAB_EINVAL, "threads must be in [1, 1024]");
  const int T = threads;
  auto pass = [&](auto body) {
#pragma omp parallel num_threads(T)
    {
      const int nth = omp_get_num_threads(), tid = omp_get_thread_num();
      for (int t = tid; t < T; t += nth)
        for (int64_t i = range_begin(n, t, T); i < range_begin(n, t + 1, T); ++i) body(i);
    }
  };
  if (run == 1) {
    pass([&](int64_t i) { y[i] = a * x[i] + b * y[i]; });
    pass([&](int64_t i) { z[i] = b * x[i] + a * z[i]; });
    pass([&](int64_t i) { z[i] = b * y[i] + c * z[i]; });
  } else if (run == 2) {
    pass([&](int64_t i) {
      y[i] = a * x[i] + b * y[i];
      z[i] = b * x[i] + a * z[i];
    });
  } else {
    pass([&](int64_t i) {
      const double yi = a * x[i] + b * y[i];
      const double zi = b * x[i] + a * z[i];
      y[i] = yi;
      z[i] = b * yi + c * zi;
    });
  }
  return BICGSTAB_OK;
}

int bicgstab_host_loop_time(bicgstab_host_t h, double* seconds, int32_t* passes) {
  if (!h) return fail(BICGSTAB_EINVAL, "null handle");
  if (seconds) *seconds = h->loop_seconds;
  if (passes) *passes = h->loop_passes;
  return BICGSTAB_OK;
}

int bicgstab_host_destroy(bicgstab_host_t h) {
  delete h;
  return BICGSTAB_OK;
}

const char* bicgstab_host_last_error(void) { return g_err.c_str(); }

}  // extern "C"
