// Launch plans, per-solve state layout and the method's ids: plain C++ shared
// by the HIP library and the host executor (no HIP types here).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace bcg {

constexpr int kBlock = 256;       // threads per workgroup for every kernel
constexpr int kMaxK = 64;         // columns per handle (one wavefront of lanes)
constexpr int kSpmmNnzMax = 4096; // CSR entries staged in LDS per SpMM row block
constexpr int kSpmmRowsMax = 1024; // rows per SpMM row block

// ---- per-column device state: scalars sc[slot * kMaxK + c] -----------------
enum ScalarSlot {
  S_RHO = 0,
  S_ALPHA,
  S_OMEGA,
  S_BETA,
  S_EPS2,
  S_BB,
  S_EST,
  S_RELRES_TRUE,
  S_RELRES_REC,
  S_RHONEXT,
  S_SCALE,  // refinement: ||r_c|| of the outer residual
  S_DELTA,       // Improved BiCGStab (Alg. 3): delta_{j+1}
  S_TAU,         //   tau_{j+1}
  S_SIGMA,       //   sigma_j
  S_SIGMA_PREV,  //   sigma_{j-1}
  S_C1,          //   beta_{j+1} alpha_{j+1} / alpha_j (z update)
  S_C2,          //   alpha_{j+1} delta_{j+1} (z update)
  S_RE_ERR,      // Reordered BiCGStab (Alg. 6): running bound E of the rho recurrence's rounding
  S_RE_SH,       //   (r0, r0) of the current shadow vector
  S_D0,  // dot results D0..D6 follow
  S_NSCAL = S_D0 + 7
};
// ---- per-column ints ist[slot * kMaxK + c] ------------------------------------
// I_PEND_NEXT: a stop found while forming the next pass's scalars (Alg. 3),
// taken when that pass would start. I_RESTART: the Reordered method restarts
// this column in the current pass (its r pass also writes the new shadow r0).
enum IntSlot { I_STATUS = 0, I_PEND, I_ITERS, I_ZEROB, I_PEND_NEXT, I_RESTART, I_NINT };
// ---- globals -----------------------------------------------------------------
struct Globals {
  int nrun;      // columns with status RUNNING; every iteration kernel exits at once when 0
  int it;        // passes completed
  int maxit;
  int hist_cap;  // history rows available
  double tol;
  int zero_diag; // Jacobi setup: number of zero diagonal entries
  int pad;
};

constexpr int ST_RUNNING = -1;
constexpr int ST_CONVERGED = 0;
constexpr int ST_MAXIT = 1;
constexpr int ST_BREAKDOWN = 2;
constexpr int ST_NONFINITE = 3;

// Finalize steps: the scalar recurrence run by the one-workgroup finalize
// kernel that follows a reduction pass (or a dot-free pass that closes an
// iteration).
enum FinStep {
  F_NONE = 0,
  F_INIT,           // D0=(r,r) D1=(b,b): eps^2, rho_0, early stops
  F_ALPHA,          // D0=delta: alpha = rho/delta
  F_OMEGA_MERGED,   // D0=phi D1=psi D2=theta: omega, theta-omega*phi stop test
  F_OMEGA_BASIC,    // D0=phi D1=psi: omega
  F_CONV_BASIC,     // D2=(r,r): explicit stop test
  F_BETA_END,       // D3=rho': beta, then close the iteration
  F_RE_OMEGA,       // D0=theta D1=phi D2=psi D3=eta: omega, stop, rho'=-omega psi, beta, restart test
  F_END,            // close the iteration
  F_PIPE_INIT,      // D0=(r0,w0): alpha_0
  F_PIPE_OMEGA,     // D0=theta D1=phi D2=pi: omega, pi-omega*theta stop test
  F_PIPE_BETA_END,  // D3=rho' D4=psi D5=sigma D6=delta: beta, alpha_{j+1}, close
  F_EXIT,           // D0=||b-Ax||^2 D1=||r||^2: relative residuals
  F_REFINE_NORM,    // refinement: D0=||r||^2, D1=||b||^2 of the outer residual
  F_IB_INIT,        // Alg. 3: D0=sigma_0=(r0,u0) D1=phi_0=(r0,r0): the first pass's scalars
  F_IB_OMEGA,       // Alg. 3: D0..D6 = phi, pi, gamma, eta, theta, kappa, nu: omega, sigma,
                    //   stop test, then the next pass's rho, delta, beta, tau, alpha
  F_IB_END,         // Alg. 3: close the iteration (a pending stop, or the next pass's)
};

// Pointers to the per-solve device state, passed by value to kernels.
struct Ctl {
  double* sc;
  int* ist;
  Globals* glob;
  double* partials;
  double* hist;
  int k;
};

// ---- vector-operation kernels ("groups") ---------------------------------------
// Every group is one streaming pass over n x k blocks. Ops are named after the
// statement(s) they perform; see kernels.hip for their bodies.
enum OpId {
  OP_INIT = 0,     // r = b - z; r0 = r; dots (r,r), (b,b)
  OP_INIT_P,       // same, plus p = r
  OP_ZEROB,        // x_c = 0 for columns whose b_c = 0
  OP_COPY,         // out = in
  OP_FILL0,        // out = 0
  OP_EXIT,         // dots (b - z, b - z), (r, r)
  OP_DOT,          // dot (u, w)
  OP_DOTSELF,      // dot (u, u)
  OP_SUB_ALPHA,    // out = a - alpha * b
  OP_SUB_OMEGA,    // out = a - omega * b
  OP_XUPD,         // x = x + alpha * a + omega * b
  OP_PUPD,         // out = a + beta * (out - omega * b)   (p-type three-vector update)
  OP_C_PPT,        // dots (t,s), (t,t), (s,s)
  OP_C_XR_RHO,     // x += alpha p + omega s; r = s - omega t; dot (r, r0)
  OP_C_R_RHO,      // r = s - omega t; dot (r, r0)
  OP_R_G3,         // rt = r - alpha v; dots (t,rt), (t,t), (t,r0), (rt,rt)
  OP_R_XZV,        // x += alpha vh + omega th; z = th - omega q; vh = z + beta (vh - omega s)
  OP_P_G1,         // Alg. 4 first group (p, s, z, q, y; theta, phi, pi)
  OP_P_G2,         // x += alpha p + omega q; r = q - omega y
  OP_P_G3,         // w = y - omega (t - alpha v); dots (r0,r), (r0,z), (r0,w), (r0,s)
  OP_PP_G12,       // Alg. 7, first line: ph, sh, qh and s, z, q, y; theta, phi, pi
  OP_PP_G34,       // Alg. 7, second line: x += alpha ph + omega qh, rh = qh - omega (wh - alpha zh)
                   // and r = q - omega y, w = y - omega (t - alpha v); 4 dots
  OP_REF_RESID,    // refinement: r = b - z (FP64); dots (r,r), (b,b)
  OP_REF_SCALE,    // refinement: r32 = r / ||r_c|| (to FP32), d = 0
  OP_REF_UPDATE,   // refinement: x = x + ||r_c|| * d
  OP_F_SUB_ALPHA_H,  // fused Jacobi: s = r - alpha v; sh = s / a_ii
  OP_F_PUPD_H,       // fused Jacobi: p = r + beta (p - omega v); ph = p / a_ii
  OP_F_XR_RHO_H,     // fused Jacobi: x += alpha ph + omega sh; r = s - omega t; dot (r, r0)
  OP_IB_INIT,        // Alg. 3 start: dots (r0, u), (r0, r0)
  OP_IB_G1,          // Alg. 3: z, v, s updates
  OP_IB_G2,          // Alg. 3: t = u - alpha q and the seven dots
  OP_IB_G3,          // Alg. 3: r = s - omega t; x = x + z + omega s
  OP_IB_Z,           // Alg. 3 basic: z = alpha r + c1 z - c2 v
  OP_IB_V,           // Alg. 3 basic: v = u + beta v - delta q
  OP_IB_X,           // Alg. 3 basic: x = x + z + omega s
  OP_RE_R,           // Alg. 6: r = rt - omega t; r0 = r for a column that restarts
  OP_F_XR_RHO_D,     // folded Jacobi, Alg. 5: x += alpha p / a_ii + omega s / a_ii; r = s - omega t; dot (r, r0)
  OP_F_P_G23,        // fused Alg. 4: OP_P_G2 and OP_P_G3 in one pass (r kept in registers); 4 dots
  OP_F_P_G23D,       // folded Jacobi, Alg. 7 as Alg. 4 on A M^{-1}: the same with x += (alpha p + omega q) / a_ii
  OP_F_RE_XVD,       // folded Jacobi, Alg. 6 on A M^{-1}: r = rt - omega t (r0 = r on a restart);
                     //   x += alpha p / a_ii + omega rt / a_ii; p = r + beta (p - omega v)
  OP_F_RE_XV,        // fused Alg. 6 without a preconditioner: the same with x += alpha p + omega rt
  OP_R_DOTS,         // Alg. 6: (t, rt), (t, t), (t, r0), (rt, rt)
  OP_NUM
};

// Blocks a vector pass reads and writes at most (Alg. 7's passes, which
// update the preconditioned and the plain blocks of a line together).
constexpr int kMaxPassIn = 12, kMaxPassOut = 8;

// Vector names used by the launch plans (indices into the handle's table).
enum VecId {
  V_NONE = -1,
  V_X = 0,  // user solution / initial guess
  V_B,      // user right-hand side
  V_R, V_R0, V_P, V_V, V_S, V_T, V_Z, V_PH, V_SH, V_TH, V_RT, V_Q, V_VH, V_W, V_WH, V_Y, V_QH, V_RH, V_ZH,
  V_NUM
};

// K_SPMM_DOT: a sparse product with an epilogue on the rows it writes
// (op = SpmmEpilogue): dot products against a second operand (in[1]) and/or
// the Jacobi-scaled copy y / a_ii (out[1]).
// K_SPMM_T: the product with the transposed matrix (Alg. 3's f0 = A^T r0).
enum StepKind { K_SPMM = 0, K_PREC, K_GROUP, K_SPMM_DOT, K_SPMM_T };

enum SpmmEpilogue {
  E_DOT_W = 0,   // y = A x; dot (y, w)
  E_PPT,         // y = A x; dots (y, w), (y, y), (w, w)
  E_PREC,        // y = A x; yh = y / a_ii
  E_DOT_W_PREC,  // y = A x; yh = y / a_ii; dot (y, w)
  E_RE4,         // y = A x; dots (y, x), (y, y), (y, w), (x, x) with x read at the row itself (Alg. 6)
  E_NUM
};
// Dot products and scaled-copy output of an epilogue.
constexpr int epilogue_dots(int epi) {
  return epi == E_RE4 ? 4 : epi == E_PPT ? 3 : (epi == E_DOT_W || epi == E_DOT_W_PREC) ? 1 : 0;
}
constexpr int kMaxEpilogueDots = 4;
// the epilogue also reads the product's own input row (not only gathers it)
constexpr bool epilogue_reads_x(int epi) { return epi == E_RE4; }
constexpr bool epilogue_prec(int epi) { return epi == E_PREC || epi == E_DOT_W_PREC; }

struct Step {
  StepKind kind;
  int op;        // OpId for K_GROUP
  int in[kMaxPassIn];    // VecIds of the blocks a vector pass reads
  int out[kMaxPassOut];  // and writes
  int slot;      // first dot slot written
  int fin;       // FinStep
  int nin, nout; // vector reads / writes of the pass (traffic accounting)
  int fold;      // products: 1 = with A M^{-1} (Jacobi folded into the values), 0 = with A
};

struct Plan {
  std::vector<Step> init;  // before the loop
  std::vector<Step> iter;  // one iteration
  std::vector<int> vecs;   // VecIds the plan touches (beside x and b)
  int alias_from[V_NUM];   // alias_from[v] = u: vector v is the same storage as u
};

// Builds the launch plan of (variant, formulation, precond). Returns false on
// an unknown combination.
// k: the right-hand sides (from k = 4 on the fused Reordered form takes its
// four dots in a product's epilogue; below, in a pass of their own).
bool build_plan(int variant, int formulation, int precond, int k, Plan* plan, std::string* err);

// Static description of every op (for traffic accounting and validation).
// The last ncond outputs are written only for a column that restarts (a rare
// event, left out of the per-iteration traffic).
struct OpInfo {
  int nin, nout, ndot;
  const char* name;
  int ncond;
};
const OpInfo& op_info(int op);

}  // namespace bcg
