// Launch plans: the sequence of kernels that makes up the start and one
// iteration of every method, in basic and merged form (and, for the classical
// method, a fused form).
//
// Merged plans give one streaming pass per line of the paper's merged
// listings (Appendix B: Alg. 2 and 5 classical, Alg. 6 Reordered, Alg. 4 and 7
// Pipelined). Basic plans give one pass per statement: a three-vector update
// is one pass, a four-vector update w = y - omega (t - alpha v) is two, and a
// dot product is its own pass reading each distinct vector once (the counting
// rule of Table 2 and its footnotes). Sparse products and preconditioner
// applications are separate launches in both forms (Section 2.3 counts them
// apart from Table 2).
#include <cstdlib>
#include <cstring>

#include "plan.hpp"

namespace bcg {

namespace {

const OpInfo kOps[OP_NUM] = {
    {2, 2, 2, "init"},        // OP_INIT
    {2, 3, 2, "init_p"},      // OP_INIT_P
    {0, 1, 0, "zerob"},       // OP_ZEROB
    {1, 1, 0, "copy"},        // OP_COPY
    {0, 1, 0, "fill0"},       // OP_FILL0
    {3, 0, 2, "exit"},        // OP_EXIT
    {2, 0, 1, "dot"},         // OP_DOT
    {1, 0, 1, "dotself"},     // OP_DOTSELF
    {2, 1, 0, "sub_alpha"},   // OP_SUB_ALPHA
    {2, 1, 0, "sub_omega"},   // OP_SUB_OMEGA
    {3, 1, 0, "xupd"},        // OP_XUPD
    {3, 1, 0, "pupd"},        // OP_PUPD
    {2, 0, 3, "c_ppt"},       // OP_C_PPT
    {5, 2, 1, "c_xr_rho"},    // OP_C_XR_RHO
    {3, 1, 1, "c_r_rho"},     // OP_C_R_RHO
    {4, 1, 4, "r_g3"},        // OP_R_G3
    {5, 3, 0, "r_xzv"},       // OP_R_XZV
    {7, 5, 3, "p_g1"},        // OP_P_G1
    {4, 2, 0, "p_g2"},        // OP_P_G2
    {7, 1, 4, "p_g3"},        // OP_P_G3
    {11, 7, 3, "pp_g12"},     // OP_PP_G12
    {12, 4, 4, "pp_g34"},     // OP_PP_G34
    {2, 1, 2, "ref_resid"},   // OP_REF_RESID
    {1, 2, 0, "ref_scale"},   // OP_REF_SCALE
    {2, 1, 0, "ref_update"},  // OP_REF_UPDATE
    {2, 2, 0, "f_sub_alpha_h"},  // OP_F_SUB_ALPHA_H (+ the diagonal)
    {3, 2, 0, "f_pupd_h"},       // OP_F_PUPD_H (+ the diagonal)
    {6, 2, 1, "f_xr_rho_h"},     // OP_F_XR_RHO_H
    {2, 0, 2, "ib_init"},        // OP_IB_INIT
    {5, 3, 0, "ib_g1"},          // OP_IB_G1
    {5, 1, 7, "ib_g2"},          // OP_IB_G2
    {4, 2, 0, "ib_g3"},          // OP_IB_G3
    {3, 1, 0, "ib_z"},           // OP_IB_Z
    {3, 1, 0, "ib_v"},           // OP_IB_V
    {3, 1, 0, "ib_x"},           // OP_IB_X
    {2, 2, 0, "re_r", 1},        // OP_RE_R (r0 written on a restart only)
    {5, 2, 1, "f_xr_rho_d"},     // OP_F_XR_RHO_D (+ the diagonal)
    {9, 3, 4, "f_p_g23"},        // OP_F_P_G23
    {9, 3, 4, "f_p_g23d"},       // OP_F_P_G23D (+ the diagonal)
    {5, 4, 0, "f_re_xvd", 1},    // OP_F_RE_XVD (+ the diagonal; r0 written on a restart only)
    {5, 4, 0, "f_re_xv", 1},     // OP_F_RE_XV (r0 written on a restart only)
    {3, 0, 4, "r_dots"},         // OP_R_DOTS
};

Step G(int op, std::initializer_list<int> in, std::initializer_list<int> out, int slot = 0, int fin = F_NONE) {
  Step s;
  std::memset(&s, 0, sizeof(s));
  s.kind = K_GROUP;
  s.op = op;
  for (int i = 0; i < kMaxPassIn; ++i) s.in[i] = V_NONE;
  for (int i = 0; i < kMaxPassOut; ++i) s.out[i] = V_NONE;
  if (in.size() > (size_t)kMaxPassIn || out.size() > (size_t)kMaxPassOut) std::abort();  // a plan bug
  int i = 0;
  for (int v : in) s.in[i++] = v;
  int o = 0;
  for (int v : out) s.out[o++] = v;
  s.nin = i;
  s.nout = o;
  s.slot = slot;
  s.fin = fin;
  return s;
}

Step SPMM(int in, int out) {
  Step s = G(OP_COPY, {in}, {out});
  s.kind = K_SPMM;
  s.op = -1;
  return s;
}

// The same with the Jacobi-folded matrix: y = (A M^{-1}) x.
Step SPMM_FOLD(int in, int out) {
  Step s = SPMM(in, out);
  s.fold = 1;
  return s;
}

// Sparse product y = A x with a dot epilogue against w (SpmmEpilogue epi).
Step SPMM_DOT(int x, int y, int epi, int w, int slot, int fin) {
  Step s = G(OP_COPY, {x, w}, {y}, slot, fin);
  s.kind = K_SPMM_DOT;
  s.op = epi;
  return s;
}

// The same with the Jacobi-folded matrix: y = (A M^{-1}) x.
Step SPMM_DOT_FOLD(int x, int y, int epi, int w, int slot, int fin) {
  Step s = SPMM_DOT(x, y, epi, w, slot, fin);
  s.fold = 1;
  return s;
}

// Sparse product y = A x that also writes yh = y / a_ii, with the dot
// (y, w) in its epilogue when w is given.
Step SPMM_PREC(int x, int y, int yh, int w = V_NONE, int slot = 0, int fin = F_NONE) {
  Step s = w == V_NONE ? G(OP_COPY, {x}, {y, yh}, slot, fin) : G(OP_COPY, {x, w}, {y, yh}, slot, fin);
  s.kind = K_SPMM_DOT;
  s.op = w == V_NONE ? E_PREC : E_DOT_W_PREC;
  return s;
}

// y = A^T x (the transposed matrix).
Step SPMM_T(int in, int out) {
  Step s = G(OP_COPY, {in}, {out});
  s.kind = K_SPMM_T;
  s.op = -1;
  return s;
}

Step PREC(int in, int out) {
  Step s = G(OP_COPY, {in}, {out});
  s.kind = K_PREC;
  s.op = -1;
  return s;
}

// ------------------------------------------------------------- classical ---
// Fused form (one device, beyond the paper's grouping): the same statements as
// Alg. 2 / Alg. 5 in five launches and their finalize kernels:
//   v = A ph with delta = (v, r0) in the product's epilogue;
//   s = r - alpha v;
//   t = A sh with phi = (t, s), psi = (t, t), theta = (s, s) in the epilogue;
//   x += alpha ph + omega sh, r = s - omega t, rho' = (r, r0);
//   p = r + beta (p - omega v).
// With Jacobi the preconditioner is folded into the products: Alg. 5
// preconditions from the right, so v = A (M^{-1} p) = (A M^{-1}) p, and with a
// diagonal M the matrix A M^{-1} (entries a_ij / a_jj) is formed once. The
// products then read p and s themselves, ph = p / a_ii and sh = s / a_ii are
// formed inside the solution-update pass, and no ph or sh block is written
// or read back.
void classical_fused(int precond, Plan* P) {
  const bool jac = precond == 1;
  P->init = {SPMM(V_X, V_V), G(OP_INIT_P, {V_B, V_V}, {V_R, V_R0, V_P}, 0, F_INIT), G(OP_ZEROB, {}, {V_X})};
  auto& it = P->iter;
  if (jac)
    it.push_back(SPMM_DOT_FOLD(V_P, V_V, E_DOT_W, V_R0, 0, F_ALPHA));
  else
    it.push_back(SPMM_DOT(V_P, V_V, E_DOT_W, V_R0, 0, F_ALPHA));
  it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_S}));
  if (jac) {
    it.push_back(SPMM_DOT_FOLD(V_S, V_T, E_PPT, V_S, 0, F_OMEGA_MERGED));
    it.push_back(G(OP_F_XR_RHO_D, {V_X, V_P, V_S, V_T, V_R0}, {V_X, V_R}, 3, F_BETA_END));
  } else {
    it.push_back(SPMM_DOT(V_S, V_T, E_PPT, V_S, 0, F_OMEGA_MERGED));
    it.push_back(G(OP_C_XR_RHO, {V_X, V_P, V_S, V_T, V_R0}, {V_X, V_R}, 3, F_BETA_END));
  }
  it.push_back(G(OP_PUPD, {V_R, V_P, V_V}, {V_P}));
  P->vecs = {V_R, V_R0, V_P, V_V, V_S, V_T};
}

void classical(int formulation, int precond, Plan* P) {
  if (formulation == 2) {
    classical_fused(precond, P);
    return;
  }
  const bool jac = precond == 1;
  const int ph = jac ? V_PH : V_P;  // p-hat (= p without preconditioner)
  const int sh = jac ? V_SH : V_S;  // s-hat
  P->init = {SPMM(V_X, V_V), G(OP_INIT_P, {V_B, V_V}, {V_R, V_R0, V_P}, 0, F_INIT), G(OP_ZEROB, {}, {V_X})};
  auto& it = P->iter;
  if (jac) it.push_back(PREC(V_P, V_PH));
  it.push_back(SPMM(ph, V_V));
  it.push_back(G(OP_DOT, {V_V, V_R0}, {}, 0, F_ALPHA));           // delta = (v, r0)
  it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_S}));                // s = r - alpha v
  if (jac) it.push_back(PREC(V_S, V_SH));
  it.push_back(SPMM(sh, V_T));
  if (formulation == 0) {
    // Alg. 2 / Alg. 5 merged lines
    it.push_back(G(OP_C_PPT, {V_T, V_S}, {}, 0, F_OMEGA_MERGED));  // phi, psi, theta
    if (!jac) {
      it.push_back(G(OP_C_XR_RHO, {V_X, V_P, V_S, V_T, V_R0}, {V_X, V_R}, 3, F_BETA_END));
    } else {
      // Alg. 5 keeps x += alpha ph + omega sh apart from {r, rho}; it does not
      // depend on beta, so it runs first and the rho pass closes the iteration.
      it.push_back(G(OP_XUPD, {V_X, V_PH, V_SH}, {V_X}));
      it.push_back(G(OP_C_R_RHO, {V_S, V_T, V_R0}, {V_R}, 3, F_BETA_END));
    }
  } else {
    // Alg. 1 one statement per pass; explicit (r, r) stop test
    it.push_back(G(OP_DOT, {V_T, V_S}, {}, 0, F_NONE));             // phi
    it.push_back(G(OP_DOTSELF, {V_T}, {}, 1, F_OMEGA_BASIC));      // psi -> omega
    it.push_back(G(OP_XUPD, {V_X, ph, sh}, {V_X}));
    it.push_back(G(OP_SUB_OMEGA, {V_S, V_T}, {V_R}));               // r = s - omega t
    it.push_back(G(OP_DOTSELF, {V_R}, {}, 2, F_CONV_BASIC));       // (r, r)
    it.push_back(G(OP_DOT, {V_R, V_R0}, {}, 3, F_BETA_END));        // rho'
  }
  it.push_back(G(OP_PUPD, {V_R, V_P, V_V}, {V_P}));                 // p = r + beta (p - omega v)
  P->vecs = {V_R, V_R0, V_P, V_V, V_S, V_T};
  if (jac) {
    P->vecs.push_back(V_PH);
    P->vecs.push_back(V_SH);
  }
}

// ------------------------------------------------------------- reordered ---
// Fused form of Alg. 6 (one device, beyond the paper's grouping). Without a
// preconditioner Alg. 6's z is r, s is v and t-hat is r-tilde (bit for bit:
// the same updates of the same operands), and with Jacobi, Alg. 6
// preconditions from the right, so with v-hat = M^{-1} p it is the listing
// run on the folded matrix A M^{-1} with no preconditioner, carrying p and
// r-tilde where it carried v-hat and t-hat. Either way: v = A p with delta in
// the product's epilogue; rt = r - alpha v; t = A rt with the four dots (t,
// rt), (t, t), (t, r0), (rt, rt) in its epilogue; then one pass {r = rt -
// omega t (r0 = r on a restart), x += alpha p + omega rt (with Jacobi p / a_ii
// and rt / a_ii), p = r + beta (p - omega v)}, the scalar step having formed
// beta with omega (A being A M^{-1} with Jacobi). 10 block reads and 4 writes
// per iteration, no z, s, t-hat or q block. Below k = 4 the blocks stay in
// the caches and the epilogue's run-sum kernel costs more than it saves: the
// four dots then take a pass of their own after a plain product (11 / 4).
void reordered_fused(int precond, int k, Plan* P) {
  const bool jac = precond == 1;
  P->init = {SPMM(V_X, V_V), G(OP_INIT, {V_B, V_V}, {V_R, V_R0}, 0, F_INIT), G(OP_ZEROB, {}, {V_X}),
             G(OP_COPY, {V_R}, {V_VH})};  // p_0 = r_0 (held in the v-hat block)
  auto& it = P->iter;
  const bool epi4 = k >= 4;
  if (jac) {
    it.push_back(SPMM_DOT_FOLD(V_VH, V_V, E_DOT_W, V_R0, 0, F_ALPHA));  // v = A M^{-1} p, delta
    it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_RT}));                  // rt = r - alpha v
    if (epi4)
      it.push_back(SPMM_DOT_FOLD(V_RT, V_T, E_RE4, V_R0, 0, F_RE_OMEGA));  // t = A M^{-1} rt, four dots
    else
      it.push_back(SPMM_FOLD(V_RT, V_T));
  } else {
    it.push_back(SPMM_DOT(V_VH, V_V, E_DOT_W, V_R0, 0, F_ALPHA));
    it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_RT}));
    if (epi4)
      it.push_back(SPMM_DOT(V_RT, V_T, E_RE4, V_R0, 0, F_RE_OMEGA));
    else
      it.push_back(SPMM(V_RT, V_T));
  }
  if (!epi4) it.push_back(G(OP_R_DOTS, {V_T, V_RT, V_R0}, {}, 0, F_RE_OMEGA));
  it.push_back(G(jac ? OP_F_RE_XVD : OP_F_RE_XV, {V_RT, V_T, V_X, V_VH, V_V}, {V_R, V_X, V_VH, V_R0}, 0, F_END));
  P->vecs = {V_R, V_R0, V_V, V_T, V_RT, V_VH};
}

void reordered(int formulation, int precond, int k, Plan* P) {
  const bool jac = precond == 1;
  if (formulation == 2) {
    reordered_fused(precond, k, P);
    return;
  }
  P->init = {SPMM(V_X, V_V), G(OP_INIT, {V_B, V_V}, {V_R, V_R0}, 0, F_INIT), G(OP_ZEROB, {}, {V_X})};
  if (jac)
    P->init.push_back(PREC(V_R, V_Z));
  else
    P->init.push_back(G(OP_COPY, {V_R}, {V_Z}));
  P->init.push_back(G(OP_COPY, {V_Z}, {V_VH}));  // v-hat_0 = z_0
  auto& it = P->iter;
  it.push_back(SPMM(V_VH, V_V));
  it.push_back(G(OP_DOT, {V_V, V_R0}, {}, 0, F_ALPHA));  // delta
  if (jac) it.push_back(PREC(V_V, V_S));                 // s = M^{-1} v (alias of v when M = I)
  it.push_back(G(OP_SUB_ALPHA, {V_Z, V_S}, {V_TH}));     // t-hat = z - alpha s
  it.push_back(SPMM(V_TH, V_T));
  if (formulation == 0) {
    it.push_back(G(OP_R_G3, {V_R, V_V, V_T, V_R0}, {V_RT}, 0, F_RE_OMEGA));
    if (jac) it.push_back(PREC(V_T, V_Q));
    it.push_back(G(OP_RE_R, {V_RT, V_T}, {V_R, V_R0}));   // r = rt - omega t
    it.push_back(G(OP_R_XZV, {V_X, V_VH, V_TH, V_Q, V_S}, {V_X, V_Z, V_VH}, 0, F_END));
  } else {
    it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_RT}));   // rt = r - alpha v
    it.push_back(G(OP_DOT, {V_T, V_RT}, {}, 0));         // theta
    it.push_back(G(OP_DOTSELF, {V_T}, {}, 1));           // phi
    it.push_back(G(OP_DOT, {V_T, V_R0}, {}, 2));         // psi
    it.push_back(G(OP_DOTSELF, {V_RT}, {}, 3, F_RE_OMEGA));  // eta
    if (jac) it.push_back(PREC(V_T, V_Q));
    it.push_back(G(OP_RE_R, {V_RT, V_T}, {V_R, V_R0}));
    it.push_back(G(OP_XUPD, {V_X, V_VH, V_TH}, {V_X}));
    it.push_back(G(OP_SUB_OMEGA, {V_TH, V_Q}, {V_Z}));   // z = th - omega q
    Step s = G(OP_PUPD, {V_Z, V_VH, V_S}, {V_VH}, 0, F_END);  // vh = z + beta (vh - omega s)
    it.push_back(s);
  }
  P->vecs = {V_R, V_R0, V_V, V_T, V_Z, V_TH, V_RT, V_VH};
  if (jac) {
    P->vecs.push_back(V_S);
    P->vecs.push_back(V_Q);
  } else {
    P->alias_from[V_S] = V_V;
    P->alias_from[V_Q] = V_T;
  }
}

// ------------------------------------------------------------- pipelined ---
// Fused form (one device, beyond the paper's grouping): Alg. 4's lines
// {x, r} and {w and the four dots} in one pass that keeps r in registers
// (16 block reads per iteration instead of 18). With Jacobi, Alg. 7 is Alg. 4
// on the operator A M^{-1}: its plain vectors obey Alg. 4's recurrences with
// that operator and each hat vector is M^{-1} times its plain one. So the
// products read the folded matrix (entries a_ij / a_jj), no hat block exists
// (10 blocks instead of 15, 24 block passes per iteration instead of 38) and
// the solution update divides p and q by a_ii itself.
void pipelined_fused(int precond, Plan* P) {
  const bool jac = precond == 1;
  auto prod = [jac](int in, int out) { return jac ? SPMM_FOLD(in, out) : SPMM(in, out); };
  P->init = {SPMM(V_X, V_V), G(OP_INIT, {V_B, V_V}, {V_R, V_R0}, 0, F_INIT), G(OP_ZEROB, {}, {V_X}), prod(V_R, V_W),
             prod(V_W, V_T), G(OP_DOT, {V_R, V_W}, {}, 0, F_PIPE_INIT)};
  for (int v : {V_S, V_Z, V_V, V_P}) P->init.push_back(G(OP_FILL0, {}, {v}));
  auto& it = P->iter;
  it.push_back(G(OP_P_G1, {V_R, V_P, V_S, V_W, V_Z, V_T, V_V}, {V_P, V_S, V_Z, V_Q, V_Y}, 0, F_PIPE_OMEGA));
  it.push_back(prod(V_Z, V_V));
  it.push_back(G(jac ? OP_F_P_G23D : OP_F_P_G23, {V_X, V_P, V_Q, V_Y, V_T, V_V, V_R0, V_Z, V_S}, {V_X, V_R, V_W}, 3,
                 F_PIPE_BETA_END));
  it.push_back(prod(V_W, V_T));
  P->vecs = {V_R, V_R0, V_P, V_V, V_S, V_T, V_Z, V_Q, V_W, V_Y};
}

void pipelined(int formulation, int precond, Plan* P) {
  if (formulation == 2) {
    pipelined_fused(precond, P);
    return;
  }
  const bool jac = precond == 1;
  auto& in = P->init;
  in = {SPMM(V_X, V_V), G(OP_INIT, {V_B, V_V}, {V_R, V_R0}, 0, F_INIT), G(OP_ZEROB, {}, {V_X})};
  if (!jac) {
    in.push_back(SPMM(V_R, V_W));
    in.push_back(SPMM(V_W, V_T));
  } else {
    in.push_back(PREC(V_R, V_RH));
    in.push_back(SPMM(V_RH, V_W));
    in.push_back(PREC(V_W, V_WH));
    in.push_back(SPMM(V_WH, V_T));
  }
  in.push_back(G(OP_DOT, {V_R, V_W}, {}, 0, F_PIPE_INIT));
  // previous-iteration vectors start at zero (beta_{-1} = 0)
  for (int v : {V_S, V_Z, V_V}) in.push_back(G(OP_FILL0, {}, {v}));
  if (!jac)
    in.push_back(G(OP_FILL0, {}, {V_P}));
  else
    for (int v : {V_PH, V_SH, V_ZH}) in.push_back(G(OP_FILL0, {}, {v}));

  auto& it = P->iter;
  if (!jac) {
    if (formulation == 0) {
      it.push_back(G(OP_P_G1, {V_R, V_P, V_S, V_W, V_Z, V_T, V_V}, {V_P, V_S, V_Z, V_Q, V_Y}, 0, F_PIPE_OMEGA));
      it.push_back(SPMM(V_Z, V_V));
      it.push_back(G(OP_P_G2, {V_X, V_P, V_Q, V_Y}, {V_X, V_R}));
      it.push_back(G(OP_P_G3, {V_Y, V_T, V_V, V_R0, V_R, V_Z, V_S}, {V_W}, 3, F_PIPE_BETA_END));
      it.push_back(SPMM(V_W, V_T));
    } else {
      it.push_back(G(OP_PUPD, {V_R, V_P, V_S}, {V_P}));     // p = r + beta (p - omega s)
      it.push_back(G(OP_PUPD, {V_W, V_S, V_Z}, {V_S}));     // s = w + beta (s - omega z)
      it.push_back(G(OP_PUPD, {V_T, V_Z, V_V}, {V_Z}));     // z = t + beta (z - omega v)
      it.push_back(G(OP_SUB_ALPHA, {V_R, V_S}, {V_Q}));     // q = r - alpha s
      it.push_back(G(OP_SUB_ALPHA, {V_W, V_Z}, {V_Y}));     // y = w - alpha z
      it.push_back(G(OP_DOT, {V_Q, V_Y}, {}, 0));           // theta
      it.push_back(G(OP_DOTSELF, {V_Y}, {}, 1));            // phi
      it.push_back(G(OP_DOTSELF, {V_Q}, {}, 2, F_PIPE_OMEGA));  // pi
      it.push_back(SPMM(V_Z, V_V));
      it.push_back(G(OP_XUPD, {V_X, V_P, V_Q}, {V_X}));
      it.push_back(G(OP_SUB_OMEGA, {V_Q, V_Y}, {V_R}));     // r = q - omega y
      it.push_back(G(OP_SUB_ALPHA, {V_T, V_V}, {V_W}));     // w = t - alpha v
      it.push_back(G(OP_SUB_OMEGA, {V_Y, V_W}, {V_W}));     // w = y - omega w
      it.push_back(G(OP_DOT, {V_R0, V_R}, {}, 3));          // rho'
      it.push_back(G(OP_DOT, {V_R0, V_Z}, {}, 4));          // psi
      it.push_back(G(OP_DOT, {V_R0, V_W}, {}, 5));          // sigma
      it.push_back(G(OP_DOT, {V_R0, V_S}, {}, 6, F_PIPE_BETA_END));  // delta
      it.push_back(SPMM(V_W, V_T));
    }
    P->vecs = {V_R, V_R0, V_P, V_V, V_S, V_T, V_Z, V_Q, V_W, V_Y};
  } else {
    if (formulation == 0) {
      // each line of Alg. 7 updates its hat (preconditioned) and plain blocks
      // in one pass: {ph, sh, qh, s, z, q, y; theta, phi, pi} and
      // {x, rh, r, w; the four dots}
      it.push_back(G(OP_PP_G12, {V_RH, V_PH, V_SH, V_WH, V_ZH, V_W, V_S, V_Z, V_T, V_V, V_R},
                     {V_PH, V_SH, V_QH, V_S, V_Z, V_Q, V_Y}, 0, F_PIPE_OMEGA));
      it.push_back(PREC(V_Z, V_ZH));
      it.push_back(SPMM(V_ZH, V_V));
      it.push_back(G(OP_PP_G34, {V_X, V_PH, V_QH, V_WH, V_ZH, V_Q, V_Y, V_T, V_V, V_R0, V_Z, V_S},
                     {V_X, V_RH, V_R, V_W}, 3, F_PIPE_BETA_END));
      it.push_back(PREC(V_W, V_WH));
      it.push_back(SPMM(V_WH, V_T));
    } else {
      it.push_back(G(OP_PUPD, {V_RH, V_PH, V_SH}, {V_PH}));  // ph = rh + beta (ph - omega sh)
      it.push_back(G(OP_PUPD, {V_WH, V_SH, V_ZH}, {V_SH}));  // sh = wh + beta (sh - omega zh)
      it.push_back(G(OP_SUB_ALPHA, {V_RH, V_SH}, {V_QH}));   // qh = rh - alpha sh
      it.push_back(G(OP_PUPD, {V_W, V_S, V_Z}, {V_S}));
      it.push_back(G(OP_PUPD, {V_T, V_Z, V_V}, {V_Z}));
      it.push_back(G(OP_SUB_ALPHA, {V_R, V_S}, {V_Q}));
      it.push_back(G(OP_SUB_ALPHA, {V_W, V_Z}, {V_Y}));
      it.push_back(G(OP_DOT, {V_Q, V_Y}, {}, 0));
      it.push_back(G(OP_DOTSELF, {V_Y}, {}, 1));
      it.push_back(G(OP_DOTSELF, {V_Q}, {}, 2, F_PIPE_OMEGA));
      it.push_back(PREC(V_Z, V_ZH));
      it.push_back(SPMM(V_ZH, V_V));
      it.push_back(G(OP_XUPD, {V_X, V_PH, V_QH}, {V_X}));
      it.push_back(G(OP_SUB_ALPHA, {V_WH, V_ZH}, {V_RH}));   // rh = wh - alpha zh
      it.push_back(G(OP_SUB_OMEGA, {V_QH, V_RH}, {V_RH}));   // rh = qh - omega rh
      it.push_back(G(OP_SUB_OMEGA, {V_Q, V_Y}, {V_R}));
      it.push_back(G(OP_SUB_ALPHA, {V_T, V_V}, {V_W}));
      it.push_back(G(OP_SUB_OMEGA, {V_Y, V_W}, {V_W}));
      it.push_back(G(OP_DOT, {V_R0, V_R}, {}, 3));
      it.push_back(G(OP_DOT, {V_R0, V_Z}, {}, 4));
      it.push_back(G(OP_DOT, {V_R0, V_W}, {}, 5));
      it.push_back(G(OP_DOT, {V_R0, V_S}, {}, 6, F_PIPE_BETA_END));
      it.push_back(PREC(V_W, V_WH));
      it.push_back(SPMM(V_WH, V_T));
    }
    P->vecs = {V_R, V_R0, V_V, V_S, V_T, V_Z, V_Q, V_W, V_Y, V_PH, V_SH, V_QH, V_RH, V_WH, V_ZH};
  }
}

// -------------------------------------------------------------- improved ---
// Alg. 3. Vectors: u -> V_W, f0 -> V_Y, q -> V_Q, plus r, r0, v, z, s, t.
// Merged: one pass per grouped line ({z, v, s}, {t and the seven dots},
// {r, x}); basic: one pass per statement, each dot its own pass (Tab. 2:
// 14 / 6 and 27 / 6 block reads / writes).
void improved(int formulation, Plan* P) {
  auto& in = P->init;
  in = {SPMM(V_X, V_V), G(OP_INIT, {V_B, V_V}, {V_R, V_R0}, 0, F_INIT), G(OP_ZEROB, {}, {V_X}),
        SPMM(V_R, V_W),                                   // u0 = A r0
        SPMM_T(V_R0, V_Y),                                // f0 = A^T r0
        G(OP_IB_INIT, {V_R0, V_W}, {}, 0, F_IB_INIT)};    // sigma_0, phi_0
  for (int v : {V_Q, V_V, V_Z}) in.push_back(G(OP_FILL0, {}, {v}));
  auto& it = P->iter;
  if (formulation == 0) {
    it.push_back(G(OP_IB_G1, {V_R, V_Z, V_V, V_W, V_Q}, {V_Z, V_V, V_S}));
    it.push_back(SPMM(V_V, V_Q));
    it.push_back(G(OP_IB_G2, {V_W, V_Q, V_R0, V_S, V_Y}, {V_T}, 0, F_IB_OMEGA));
    it.push_back(G(OP_IB_G3, {V_S, V_T, V_X, V_Z}, {V_R, V_X}, 0, F_IB_END));
  } else {
    it.push_back(G(OP_IB_Z, {V_R, V_Z, V_V}, {V_Z}));
    it.push_back(G(OP_IB_V, {V_W, V_V, V_Q}, {V_V}));
    it.push_back(G(OP_SUB_ALPHA, {V_R, V_V}, {V_S}));   // s = r - alpha v
    it.push_back(SPMM(V_V, V_Q));
    it.push_back(G(OP_SUB_ALPHA, {V_W, V_Q}, {V_T}));   // t = u - alpha q
    it.push_back(G(OP_DOT, {V_R0, V_S}, {}, 0));        // phi
    it.push_back(G(OP_DOT, {V_R0, V_Q}, {}, 1));        // pi
    it.push_back(G(OP_DOT, {V_Y, V_S}, {}, 2));         // gamma
    it.push_back(G(OP_DOT, {V_Y, V_T}, {}, 3));         // eta
    it.push_back(G(OP_DOT, {V_S, V_T}, {}, 4));         // theta
    it.push_back(G(OP_DOTSELF, {V_T}, {}, 5));          // kappa
    it.push_back(G(OP_DOTSELF, {V_S}, {}, 6, F_IB_OMEGA));  // nu
    it.push_back(G(OP_SUB_OMEGA, {V_S, V_T}, {V_R}));   // r = s - omega t
    it.push_back(G(OP_IB_X, {V_X, V_Z, V_S}, {V_X}, 0, F_IB_END));
  }
  it.push_back(SPMM(V_R, V_W));  // u = A r
  P->vecs = {V_R, V_R0, V_W, V_Y, V_Q, V_V, V_Z, V_S, V_T};
}

}  // namespace

const OpInfo& op_info(int op) { return kOps[op]; }

bool build_plan(int variant, int formulation, int precond, int k, Plan* P, std::string* err) {
  P->init.clear();
  P->iter.clear();
  P->vecs.clear();
  for (int v = 0; v < V_NUM; ++v) P->alias_from[v] = -1;
  if (precond != 0 && precond != 1) {
    *err = "unknown preconditioner";
    return false;
  }
  if (formulation != 0 && formulation != 1 && formulation != 2) {
    *err = "unknown formulation";
    return false;
  }
  if (formulation == 2 && variant == 3) {
    *err = "the fused formulation is not built for Improved BiCGStab";
    return false;
  }
  if (variant == 3 && precond != 0) {
    *err = "Improved BiCGStab has no preconditioned form";
    return false;
  }
  switch (variant) {
    case 0: classical(formulation, precond, P); break;
    case 1: reordered(formulation, precond, k, P); break;
    case 2: pipelined(formulation, precond, P); break;
    case 3: improved(formulation, P); break;
    default: *err = "unknown variant"; return false;
  }
  // Every operand must be a vector the plan allocates (or x, b, or an alias),
  // and every vector pass must get exactly the operands its kernel reads and
  // writes: a plan error is caught here, on the host, never on the device.
  bool have[V_NUM] = {};
  have[V_X] = have[V_B] = true;
  for (int v : P->vecs) have[v] = true;
  for (int v = 0; v < V_NUM; ++v)
    if (P->alias_from[v] >= 0) have[v] = have[P->alias_from[v]];
  for (const auto* list : {&P->init, &P->iter}) {
    for (const Step& s : *list) {
      if (s.kind == K_GROUP) {
        const OpInfo& oi = op_info(s.op);
        if (s.nin != oi.nin || s.nout != oi.nout) {
          *err = std::string("plan step ") + oi.name + ": operand count mismatch";
          return false;
        }
        if (oi.ndot > 0 && s.slot + oi.ndot > 7) {
          *err = std::string("plan step ") + oi.name + ": dot slots out of range";
          return false;
        }
      } else if (s.kind == K_SPMM_DOT) {
        const bool known = s.op >= 0 && s.op < E_NUM;
        if (!known || s.nin != 1 + (epilogue_dots(s.op) > 0 ? 1 : 0) || s.nout != 1 + (epilogue_prec(s.op) ? 1 : 0) ||
            s.slot + epilogue_dots(s.op) > 7) {
          *err = "plan step: product with an epilogue needs x, y, the epilogue's operands and a known epilogue";
          return false;
        }
      } else if (s.nin != 1 || s.nout != 1) {
        *err = "plan step: product/preconditioner needs one input and one output";
        return false;
      }
      for (int i = 0; i < s.nin; ++i)
        if (s.in[i] < 0 || s.in[i] >= V_NUM || !have[s.in[i]]) {
          *err = "plan step reads a vector the plan does not allocate";
          return false;
        }
      for (int i = 0; i < s.nout; ++i)
        if (s.out[i] < 0 || s.out[i] >= V_NUM || !have[s.out[i]] || s.out[i] == V_B) {
          *err = "plan step writes a vector the plan does not allocate";
          return false;
        }
    }
  }
  return true;
}

}  // namespace bcg
