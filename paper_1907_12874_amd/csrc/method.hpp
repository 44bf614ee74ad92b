// The method's arithmetic, shared by the GPU kernels and the host executor:
// the per-element bodies of the vector passes (one per op id) and the
// per-column scalar steps that follow each reduction (the recurrences of
// Alg. 2-7 with the stop tests and breakdown rules). Compiled as host and
// device code by hipcc and as plain C++ by the host build.
#pragma once

#include <math.h>

#include "plan.hpp"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define BCG_HD __host__ __device__
#else
#define BCG_HD
#endif
#define BCG_INLINE inline __attribute__((always_inline))

namespace bcg {

struct Coef {
  double alpha, omega, beta, scale;
  double delta, c1, c2;  // Alg. 3 updates
};

// ------------------------------------------------------------ op bodies ---
// Each op: NIN inputs, NOUT outputs, NDOT dot products per column. XIN / XOUT
// are bitmasks of inputs / outputs that are always FP64 (the solution block);
// the others have the Krylov type T. PART says which columns take part:
// running columns, every column, or the columns whose right-hand side is zero.
enum Part { PART_RUN = 0, PART_ALL = 1, PART_ZEROB = 2 };

// COUT: bitmask of outputs written only for a column that restarts in this
// pass (I_RESTART set by the scalar step before it).
#define OP_HEAD_C(NI, NO, ND, XI, XO, PT, EARLY_, USED, CO) \
  static constexpr int NIN = NI, NOUT = NO, NDOT = ND;      \
  static constexpr unsigned XIN = XI, XOUT = XO, COUT = CO; \
  static constexpr int PART = PT;                           \
  static constexpr bool EARLY = EARLY_;                     \
  static constexpr bool USE_D = USED;
#define OP_HEAD_(NI, NO, ND, XI, XO, PT, EARLY_, USED) OP_HEAD_C(NI, NO, ND, XI, XO, PT, EARLY_, USED, 0u)
#define OP_HEAD(NI, NO, ND, XI, XO, PT, EARLY_) OP_HEAD_(NI, NO, ND, XI, XO, PT, EARLY_, false)
// USE_D: the op also reads the row's diagonal entry a_ii, passed as v[NIN].
#define OP_HEAD_D(NI, NO, ND, XI, XO, PT, EARLY_) OP_HEAD_(NI, NO, ND, XI, XO, PT, EARLY_, true)
// Op bodies compute in FP64 from operands of storage type T; a value that is
// both stored and used again in the same op is first rounded to T (R(.)), so
// dots and later terms see exactly the stored vector (a no-op when T is FP64).
#define OP_F                                                                                  \
  template <class T>                                                                          \
  BCG_HD BCG_INLINE static void f(const double* v, const Coef& c, double* o, double* a)
#define R(x) ((double)(T)(x))

struct KInit {  // r = b - z; r0 = r; (r, r), (b, b)
  OP_HEAD(2, 2, 2, 0, 0, PART_RUN, true)
  OP_F {
    double r = R(v[0] - v[1]);
    o[0] = r;
    o[1] = r;
    a[0] += r * r;
    a[1] += v[0] * v[0];
  }
};
struct KInitP {  // r = b - z; r0 = r; p = r; (r, r), (b, b)
  OP_HEAD(2, 3, 2, 0, 0, PART_RUN, true)
  OP_F {
    double r = v[0] - v[1];
    o[0] = r;
    o[1] = r;
    o[2] = r;
    a[0] += r * r;
    a[1] += v[0] * v[0];
  }
};
struct KZeroB {  // x = 0 where b = 0
  OP_HEAD(0, 1, 0, 0, 1, PART_ZEROB, false)
  OP_F { o[0] = 0.0; }
};
struct KCopy {
  OP_HEAD(1, 1, 0, 0, 0, PART_ALL, true)
  OP_F { o[0] = v[0]; }
};
struct KFill0 {
  OP_HEAD(0, 1, 0, 0, 0, PART_ALL, true)
  OP_F { o[0] = 0.0; }
};
struct KExit {  // in: b, z = A x, r ; dots (b - z, b - z), (r, r)
  OP_HEAD(3, 0, 2, 0, 0, PART_ALL, false)
  OP_F {
    double d = v[0] - v[1];
    a[0] += d * d;
    a[1] += v[2] * v[2];
  }
};
struct KDot {
  OP_HEAD(2, 0, 1, 0, 0, PART_RUN, true)
  OP_F { a[0] += v[0] * v[1]; }
};
struct KDotSelf {
  OP_HEAD(1, 0, 1, 0, 0, PART_RUN, true)
  OP_F { a[0] += v[0] * v[0]; }
};
struct KSubAlpha {  // out = a - alpha b
  OP_HEAD(2, 1, 0, 0, 0, PART_RUN, true)
  OP_F { o[0] = v[0] - c.alpha * v[1]; }
};
struct KSubOmega {  // out = a - omega b
  OP_HEAD(2, 1, 0, 0, 0, PART_RUN, true)
  OP_F { o[0] = v[0] - c.omega * v[1]; }
};
struct KXUpd {  // x = x + alpha a + omega b
  OP_HEAD(3, 1, 0, 1, 1, PART_RUN, true)
  OP_F { o[0] = v[0] + c.alpha * v[1] + c.omega * v[2]; }
};
struct KPUpd {  // in: a, u, b ; out = a + beta (u - omega b)
  OP_HEAD(3, 1, 0, 0, 0, PART_RUN, true)
  OP_F { o[0] = v[0] + c.beta * (v[1] - c.omega * v[2]); }
};
struct KCPpt {  // in: t, s ; (t, s), (t, t), (s, s)
  OP_HEAD(2, 0, 3, 0, 0, PART_RUN, true)
  OP_F {
    a[0] += v[0] * v[1];
    a[1] += v[0] * v[0];
    a[2] += v[1] * v[1];
  }
};
struct KCXrRho {  // in: x, p, s, t, r0 ; out: x, r
  OP_HEAD(5, 2, 1, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    double r = R(v[2] - c.omega * v[3]);
    o[1] = r;
    a[0] += r * v[4];
  }
};
struct KFXrRhoD {  // folded Jacobi: in: x, p, s, t, r0 (+ a_ii) ; out: x, r ; dot (r, r0)
  OP_HEAD_D(5, 2, 1, 1, 1, PART_RUN, true)
  OP_F {
    const double ph = R(v[1] / v[5]);
    const double sh = R(v[2] / v[5]);
    o[0] = v[0] + c.alpha * ph + c.omega * sh;
    const double r = R(v[2] - c.omega * v[3]);
    o[1] = r;
    a[0] += r * v[4];
  }
};
struct KReR {  // Alg. 6: in: rt, t ; out: r = rt - omega t, and r0 = r where the column restarts
  OP_HEAD_C(2, 2, 0, 0, 0, PART_RUN, true, false, 2u)
  OP_F {
    const double r = R(v[0] - c.omega * v[1]);
    o[0] = r;
    o[1] = r;
  }
};
struct KCRRho {  // in: s, t, r0 ; out: r
  OP_HEAD(3, 1, 1, 0, 0, PART_RUN, true)
  OP_F {
    double r = R(v[0] - c.omega * v[1]);
    o[0] = r;
    a[0] += r * v[2];
  }
};
struct KRG3 {  // in: r, v, t, r0 ; out: rt ; (t, rt), (t, t), (t, r0), (rt, rt)
  OP_HEAD(4, 1, 4, 0, 0, PART_RUN, true)
  OP_F {
    double rt = R(v[0] - c.alpha * v[1]);
    o[0] = rt;
    a[0] += v[2] * rt;
    a[1] += v[2] * v[2];
    a[2] += v[2] * v[3];
    a[3] += rt * rt;
  }
};
// Alg. 6 on A M^{-1} (Jacobi folded into the products): in: rt, t, x, p, v
// (+ a_ii) ; out: r, x, p, and r0 = r where the column restarts. Alg. 6's
// z_{j+1} is r_{j+1} here, and its v-hat and t-hat are p / a_ii and rt / a_ii,
// formed for the solution update alone (rounded to the storage type as a
// stored copy would be).
struct KFReXvD {
  OP_HEAD_C(5, 4, 0, 4, 2, PART_RUN, true, true, 8u)
  OP_F {
    const double r = R(v[0] - c.omega * v[1]);
    const double ph = R(v[3] / v[5]);
    const double th = R(v[0] / v[5]);
    o[0] = r;
    o[1] = v[2] + c.alpha * ph + c.omega * th;
    o[2] = r + c.beta * (v[3] - c.omega * v[4]);
    o[3] = r;
  }
};
struct KRDots {  // in: t, rt, r0 ; (t, rt), (t, t), (t, r0), (rt, rt)
  OP_HEAD(3, 0, 4, 0, 0, PART_RUN, true)
  OP_F {
    a[0] += v[0] * v[1];
    a[1] += v[0] * v[0];
    a[2] += v[0] * v[2];
    a[3] += v[1] * v[1];
  }
};
// Fused Alg. 6 without a preconditioner (z = r, s = v, t-hat = r-tilde): in:
// rt, t, x, p, v ; out: r, x, p, and r0 = r where the column restarts.
struct KFReXv {
  OP_HEAD_C(5, 4, 0, 4, 2, PART_RUN, true, false, 8u)
  OP_F {
    const double r = R(v[0] - c.omega * v[1]);
    o[0] = r;
    o[1] = v[2] + c.alpha * v[3] + c.omega * v[0];
    o[2] = r + c.beta * (v[3] - c.omega * v[4]);
    o[3] = r;
  }
};
struct KRXzv {  // in: x, vh, th, q, s ; out: x, z, vh
  OP_HEAD(5, 3, 0, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    double z = R(v[2] - c.omega * v[3]);
    o[1] = z;
    o[2] = z + c.beta * (v[1] - c.omega * v[4]);
  }
};
struct KPG1 {  // in: r, p, s, w, z, t, v ; out: p, s, z, q, y ; (q, y), (y, y), (q, q)
  OP_HEAD(7, 5, 3, 0, 0, PART_RUN, true)
  OP_F {
    double p = R(v[0] + c.beta * (v[1] - c.omega * v[2]));
    double s = R(v[3] + c.beta * (v[2] - c.omega * v[4]));
    double z = R(v[5] + c.beta * (v[4] - c.omega * v[6]));
    double q = R(v[0] - c.alpha * s);
    double y = R(v[3] - c.alpha * z);
    o[0] = p;
    o[1] = s;
    o[2] = z;
    o[3] = q;
    o[4] = y;
    a[0] += q * y;
    a[1] += y * y;
    a[2] += q * q;
  }
};
struct KPG2 {  // in: x, p, q, y ; out: x, r
  OP_HEAD(4, 2, 0, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    o[1] = v[2] - c.omega * v[3];
  }
};
struct KPG3 {  // in: y, t, v, r0, r, z, s ; out: w ; (r0,r), (r0,z), (r0,w), (r0,s)
  OP_HEAD(7, 1, 4, 0, 0, PART_RUN, true)
  OP_F {
    double w = R(v[0] - c.omega * (v[1] - c.alpha * v[2]));
    o[0] = w;
    a[0] += v[3] * v[4];
    a[1] += v[3] * v[5];
    a[2] += v[3] * w;
    a[3] += v[3] * v[6];
  }
};
// Fused Alg. 4: {x, r} and {w and the four dots} in one pass; r is rounded to
// the storage type as if stored and read back.
struct KFPG23 {  // in: x, p, q, y, t, v, r0, z, s ; out: x, r, w ; (r0,r), (r0,z), (r0,w), (r0,s)
  OP_HEAD(9, 3, 4, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    const double r = R(v[2] - c.omega * v[3]);
    const double w = R(v[3] - c.omega * (v[4] - c.alpha * v[5]));
    o[1] = r;
    o[2] = w;
    a[0] += v[6] * r;
    a[1] += v[6] * v[7];
    a[2] += v[6] * w;
    a[3] += v[6] * v[8];
  }
};
// Alg. 7 as Alg. 4 on A M^{-1} (Jacobi folded into the products): the hat
// vectors p-hat = p / a_ii and q-hat = q / a_ii are formed here for the
// solution update alone (rounded to the storage type as a stored copy would
// be).
struct KFPG23D {  // in: x, p, q, y, t, v, r0, z, s (+ a_ii) ; out: x, r, w ; the same dots
  OP_HEAD_D(9, 3, 4, 1, 1, PART_RUN, true)
  OP_F {
    const double ph = R(v[1] / v[9]);
    const double qh = R(v[2] / v[9]);
    o[0] = v[0] + c.alpha * ph + c.omega * qh;
    const double r = R(v[2] - c.omega * v[3]);
    const double w = R(v[3] - c.omega * (v[4] - c.alpha * v[5]));
    o[1] = r;
    o[2] = w;
    a[0] += v[6] * r;
    a[1] += v[6] * v[7];
    a[2] += v[6] * w;
    a[3] += v[6] * v[8];
  }
};
// Alg. 7 in four groups: the preconditioned (hat) blocks of the first line
// (KPPG1) and its plain blocks (KPPG2), then those of the second line (KPPG3,
// KPPG4). The passes run a line's two groups together (KPPG12, KPPG34): the
// groups read and write disjoint blocks, so joining them changes no value.
struct KPPG1 {  // in: rh, ph, sh, wh, zh ; out: ph, sh, qh
  OP_HEAD(5, 3, 0, 0, 0, PART_RUN, true)
  OP_F {
    double ph = R(v[0] + c.beta * (v[1] - c.omega * v[2]));
    double sh = R(v[3] + c.beta * (v[2] - c.omega * v[4]));
    o[0] = ph;
    o[1] = sh;
    o[2] = v[0] - c.alpha * sh;
  }
};
struct KPPG2 {  // in: w, s, z, t, v, r ; out: s, z, q, y ; (q, y), (y, y), (q, q)
  OP_HEAD(6, 4, 3, 0, 0, PART_RUN, true)
  OP_F {
    double s = R(v[0] + c.beta * (v[1] - c.omega * v[2]));
    double z = R(v[3] + c.beta * (v[2] - c.omega * v[4]));
    double q = R(v[5] - c.alpha * s);
    double y = R(v[0] - c.alpha * z);
    o[0] = s;
    o[1] = z;
    o[2] = q;
    o[3] = y;
    a[0] += q * y;
    a[1] += y * y;
    a[2] += q * q;
  }
};
struct KPPG3 {  // in: x, ph, qh, wh, zh ; out: x, rh
  OP_HEAD(5, 2, 0, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    o[1] = v[2] - c.omega * (v[3] - c.alpha * v[4]);
  }
};
struct KPPG4 {  // in: q, y, t, v, r0, z, s ; out: r, w ; (r0,r), (r0,z), (r0,w), (r0,s)
  OP_HEAD(7, 2, 4, 0, 0, PART_RUN, true)
  OP_F {
    double r = R(v[0] - c.omega * v[1]);
    double w = R(v[1] - c.omega * (v[2] - c.alpha * v[3]));
    o[0] = r;
    o[1] = w;
    a[0] += v[4] * r;
    a[1] += v[4] * v[5];
    a[2] += v[4] * w;
    a[3] += v[4] * v[6];
  }
};
// in: rh, ph, sh, wh, zh, w, s, z, t, v, r ; out: ph, sh, qh, s, z, q, y ; (q, y), (y, y), (q, q)
struct KPPG12 {
  OP_HEAD(11, 7, 3, 0, 0, PART_RUN, true)
  OP_F {
    KPPG1::f<T>(v, c, o, a);
    KPPG2::f<T>(v + KPPG1::NIN, c, o + KPPG1::NOUT, a);
  }
};
// in: x, ph, qh, wh, zh, q, y, t, v, r0, z, s ; out: x, rh, r, w ; (r0,r), (r0,z), (r0,w), (r0,s)
struct KPPG34 {
  OP_HEAD(12, 4, 4, 1, 1, PART_RUN, true)
  OP_F {
    KPPG3::f<T>(v, c, o, a);
    KPPG4::f<T>(v + KPPG3::NIN, c, o + KPPG3::NOUT, a);
  }
};
static_assert(KPPG12::NIN == KPPG1::NIN + KPPG2::NIN && KPPG12::NOUT == KPPG1::NOUT + KPPG2::NOUT, "");
static_assert(KPPG34::NIN == KPPG3::NIN + KPPG4::NIN && KPPG34::NOUT == KPPG3::NOUT + KPPG4::NOUT, "");
// Refinement passes (outer loop of the FP32 tier). Inputs/outputs marked in
// XIN/XOUT are FP64; the rest are the inner (FP32) Krylov type.
struct KRefResid {  // in: b, z (FP64) ; out: r (FP64) ; (r, r), (b, b)
  OP_HEAD(2, 1, 2, 3, 1, PART_ALL, false)
  OP_F {
    double r = v[0] - v[1];
    o[0] = r;
    a[0] += r * r;
    a[1] += v[0] * v[0];
  }
};
struct KRefScale {  // in: r (FP64) ; out: rs = r / ||r_c|| (T), d = 0 (FP64)
  OP_HEAD(1, 2, 0, 1, 2, PART_ALL, false)
  OP_F {
    o[0] = c.scale > 0.0 ? v[0] / c.scale : 0.0;
    o[1] = 0.0;
  }
};
struct KRefUpdate {  // in: x, d (FP64) ; out: x = x + ||r_c|| d
  OP_HEAD(2, 1, 0, 3, 1, PART_ALL, false)
  OP_F { o[0] = v[0] + c.scale * v[1]; }
};

// Fused Jacobi: the pass that produces s or p also writes the preconditioned
// copy (the same division by a_ii as the preconditioner pass, so the values
// are those of the merged form), and the solution update joins {r, rho'}.
struct KFSubAlphaH {  // in: r, v (+ a_ii) ; out: s, sh
  OP_HEAD_D(2, 2, 0, 0, 0, PART_RUN, true)
  OP_F {
    const double sv = R(v[0] - c.alpha * v[1]);
    o[0] = sv;
    o[1] = sv / v[2];
  }
};
struct KFPUpdH {  // in: r, p, v (+ a_ii) ; out: p, ph
  OP_HEAD_D(3, 2, 0, 0, 0, PART_RUN, true)
  OP_F {
    const double pv = R(v[0] + c.beta * (v[1] - c.omega * v[2]));
    o[0] = pv;
    o[1] = pv / v[3];
  }
};
struct KFXrRhoH {  // in: x, ph, sh, s, t, r0 ; out: x, r ; (r, r0)
  OP_HEAD(6, 2, 1, 1, 1, PART_RUN, true)
  OP_F {
    o[0] = v[0] + c.alpha * v[1] + c.omega * v[2];
    const double r = R(v[3] - c.omega * v[4]);
    o[1] = r;
    a[0] += r * v[5];
  }
};

// Improved BiCGStab (Alg. 3). Coefficients: alpha = alpha_{j+1}, beta, delta,
// c1 = beta alpha_{j+1} / alpha_j, c2 = alpha_{j+1} delta, omega = omega_{j+1}.
struct KIbInit {  // in: r0, u ; (r0, u), (r0, r0)
  OP_HEAD(2, 0, 2, 0, 0, PART_RUN, true)
  OP_F {
    a[0] += v[0] * v[1];
    a[1] += v[0] * v[0];
  }
};
struct KIbG1 {  // in: r, z, v, u, q ; out: z, v, s
  OP_HEAD(5, 3, 0, 0, 0, PART_RUN, true)
  OP_F {
    o[0] = c.alpha * v[0] + c.c1 * v[1] - c.c2 * v[2];  // z = alpha r + c1 z - c2 v
    const double vn = R(v[3] + c.beta * v[2] - c.delta * v[4]);  // v = u + beta v - delta q
    o[1] = vn;
    o[2] = v[0] - c.alpha * vn;  // s = r - alpha v
  }
};
struct KIbG2 {  // in: u, q, r0, s, f0 ; out: t ; phi, pi, gamma, eta, theta, kappa, nu
  OP_HEAD(5, 1, 7, 0, 0, PART_RUN, true)
  OP_F {
    const double t = R(v[0] - c.alpha * v[1]);
    o[0] = t;
    a[0] += v[2] * v[3];  // (r0, s)
    a[1] += v[2] * v[1];  // (r0, q)
    a[2] += v[4] * v[3];  // (f0, s)
    a[3] += v[4] * t;     // (f0, t)
    a[4] += v[3] * t;     // (s, t)
    a[5] += t * t;        // (t, t)
    a[6] += v[3] * v[3];  // (s, s)
  }
};
struct KIbG3 {  // in: s, t, x, z ; out: r, x
  OP_HEAD(4, 2, 0, 4, 2, PART_RUN, true)
  OP_F {
    o[0] = v[0] - c.omega * v[1];         // r = s - omega t
    o[1] = v[2] + v[3] + c.omega * v[0];  // x = x + z + omega s
  }
};
struct KIbZ {  // in: r, z, v ; out: z
  OP_HEAD(3, 1, 0, 0, 0, PART_RUN, true)
  OP_F { o[0] = c.alpha * v[0] + c.c1 * v[1] - c.c2 * v[2]; }
};
struct KIbV {  // in: u, v, q ; out: v
  OP_HEAD(3, 1, 0, 0, 0, PART_RUN, true)
  OP_F { o[0] = v[0] + c.beta * v[1] - c.delta * v[2]; }
};
struct KIbX {  // in: x, z, s ; out: x
  OP_HEAD(3, 1, 0, 1, 1, PART_RUN, true)
  OP_F { o[0] = v[0] + v[1] + c.omega * v[2]; }
};

// ------------------------------------------------------- scalar recurrence ---

// FP64 unit roundoff and the factor of the Reordered method's restart test.
constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53
constexpr double kRestartKappa = 16.0;

BCG_HD BCG_INLINE double& SC(const Ctl& C, int slot, int c) { return C.sc[slot * kMaxK + c]; }
BCG_HD BCG_INLINE int& IS(const Ctl& C, int slot, int c) { return C.ist[slot * kMaxK + c]; }

BCG_HD inline void record_history(const Ctl& C, int c, double alpha, double omega, double rho, double est) {
  const int it = C.glob->it;
  if (C.hist && it < C.glob->hist_cap) {
    double* h = C.hist + ((size_t)it * C.k + c) * 4;
    h[0] = alpha;
    h[1] = omega;
    h[2] = rho;
    h[3] = est;
  }
}

// Close an iteration for column c: a pending stop takes effect, or maxit.
BCG_HD inline void end_column(const Ctl& C, int c) {
  const int it1 = C.glob->it + 1;
  int& st = IS(C, I_STATUS, c);
  int& pend = IS(C, I_PEND, c);
  if (pend >= 0) {
    st = pend;
    IS(C, I_ITERS, c) = it1;
  } else if (it1 >= C.glob->maxit) {
    st = ST_MAXIT;
    IS(C, I_ITERS, c) = it1;
  }
}

// Alg. 3: the scalars that open a pass, from phi, pi, omega of the pass before
// and sigma_{j-1}, sigma_j, rho_j, alpha_j, tau_j; stored for the pass's
// updates. Returns -1, or the stop the pass would take (BREAKDOWN on a zero
// rho_{j+1} or tau_{j+1}, NONFINITE on a non-finite scalar).
BCG_HD inline int ib_open_pass(const Ctl& C, int c, double phi, double pi, double omega, double sigma_prev,
                            double sigma, double rho, double alpha, double tau) {
  const double rho1 = phi - omega * sigma_prev + omega * alpha * pi;
  const double delta = (rho1 / rho) * alpha;
  const double beta = delta / omega;
  const double tau1 = sigma + beta * tau - delta * pi;
  if (rho1 == 0.0 || tau1 == 0.0) return ST_BREAKDOWN;
  const double alpha1 = rho1 / tau1;
  if (!(isfinite(delta) && isfinite(beta) && isfinite(tau1) && isfinite(alpha1))) return ST_NONFINITE;
  SC(C, S_RHO, c) = rho1;
  SC(C, S_DELTA, c) = delta;
  SC(C, S_BETA, c) = beta;
  SC(C, S_TAU, c) = tau1;
  SC(C, S_C1, c) = beta * (alpha1 / alpha);
  SC(C, S_C2, c) = alpha1 * delta;
  SC(C, S_ALPHA, c) = alpha1;
  return -1;
}

// Per-column scalar work of a finalize step (see the FinStep list).
BCG_HD inline void finalize_column(int step, int c, const Ctl& C) {
  int& st = IS(C, I_STATUS, c);
  const double D0 = SC(C, S_D0 + 0, c), D1 = SC(C, S_D0 + 1, c), D2 = SC(C, S_D0 + 2, c);
  const double D3 = SC(C, S_D0 + 3, c);
  if (step == F_INIT) {
    const double rr = D0, bb = D1;
    SC(C, S_BB, c) = bb;
    IS(C, I_PEND, c) = -1;
    IS(C, I_PEND_NEXT, c) = -1;
    IS(C, I_ITERS, c) = 0;
    IS(C, I_ZEROB, c) = 0;
    SC(C, S_ALPHA, c) = 0.0;
    SC(C, S_OMEGA, c) = 1.0;
    SC(C, S_BETA, c) = 0.0;
    SC(C, S_EST, c) = rr;
    SC(C, S_RE_ERR, c) = rr;
    SC(C, S_RE_SH, c) = rr;
    IS(C, I_RESTART, c) = 0;
    if (!isfinite(bb)) {
      st = ST_NONFINITE;
      return;
    }
    if (bb == 0.0) {
      st = ST_CONVERGED;
      IS(C, I_ZEROB, c) = 1;
      return;
    }
    const double tol = C.glob->tol;
    const double eps2 = tol > 0.0 ? tol * tol * bb : -INFINITY;
    SC(C, S_EPS2, c) = eps2;
    if (!isfinite(rr)) {
      st = ST_NONFINITE;
      return;
    }
    if (rr < eps2) {
      st = ST_CONVERGED;
      return;
    }
    SC(C, S_RHO, c) = rr;
    return;
  }
  if (step == F_EXIT) {
    const double bb = SC(C, S_BB, c);
    if (bb == 0.0) {
      SC(C, S_RELRES_TRUE, c) = 0.0;
      SC(C, S_RELRES_REC, c) = 0.0;
    } else {
      SC(C, S_RELRES_TRUE, c) = sqrt(D0) / sqrt(bb);
      SC(C, S_RELRES_REC, c) = sqrt(D1) / sqrt(bb);
    }
    return;
  }
  if (step == F_REFINE_NORM) {
    // outer residual of the refinement loop: D0 = ||r||^2, D1 = ||b||^2
    SC(C, S_EST, c) = D0;
    SC(C, S_SCALE, c) = sqrt(D0);
    return;
  }
  if (st != ST_RUNNING) return;
  const int it1 = C.glob->it + 1;
  int& pend = IS(C, I_PEND, c);
  auto stop = [&](int s) {
    st = s;
    IS(C, I_ITERS, c) = it1;
  };
  const double eps2 = SC(C, S_EPS2, c);
  switch (step) {
    case F_ALPHA: {
      const double delta = D0;
      if (delta == 0.0) {
        stop(ST_BREAKDOWN);
        return;
      }
      const double alpha = SC(C, S_RHO, c) / delta;
      if (!isfinite(alpha)) {
        stop(ST_NONFINITE);
        return;
      }
      SC(C, S_ALPHA, c) = alpha;
      return;
    }
    case F_OMEGA_MERGED: {
      const double phi = D0, psi = D1, theta = D2;
      const double omega = psi != 0.0 ? phi / psi : 0.0;
      const double est = theta - omega * phi;
      if (!(isfinite(omega) && isfinite(est))) {
        stop(ST_NONFINITE);
        return;
      }
      SC(C, S_OMEGA, c) = omega;
      SC(C, S_EST, c) = est;
      if (est < eps2)
        pend = ST_CONVERGED;
      else if (omega == 0.0)
        pend = ST_BREAKDOWN;
      return;
    }
    case F_OMEGA_BASIC: {
      const double phi = D0, psi = D1;
      const double omega = psi != 0.0 ? phi / psi : 0.0;
      if (!isfinite(omega)) {
        stop(ST_NONFINITE);
        return;
      }
      SC(C, S_OMEGA, c) = omega;
      return;
    }
    case F_CONV_BASIC: {
      const double rr = D2;
      SC(C, S_EST, c) = rr;
      if (!isfinite(rr)) {
        stop(ST_NONFINITE);
        return;
      }
      if (rr < eps2) {
        record_history(C, c, SC(C, S_ALPHA, c), SC(C, S_OMEGA, c), SC(C, S_RHO, c), rr);
        stop(ST_CONVERGED);
        return;
      }
      if (SC(C, S_OMEGA, c) == 0.0) stop(ST_BREAKDOWN);
      return;
    }
    case F_BETA_END: {
      const double alpha = SC(C, S_ALPHA, c), omega = SC(C, S_OMEGA, c), rho = SC(C, S_RHO, c);
      if (pend < 0) {
        const double rho1 = D3;
        if (rho1 == 0.0) {
          stop(ST_BREAKDOWN);
          return;
        }
        const double beta = (rho1 / rho) * (alpha / omega);
        if (!isfinite(beta)) {
          stop(ST_NONFINITE);
          return;
        }
        SC(C, S_BETA, c) = beta;
        SC(C, S_RHO, c) = rho1;
      }
      record_history(C, c, alpha, omega, rho, SC(C, S_EST, c));
      end_column(C, c);
      return;
    }
    case F_RE_OMEGA: {
      const double theta = D0, phi = D1, psi = D2, eta = D3;
      const double omega = phi != 0.0 ? theta / phi : 0.0;
      const double est = eta - omega * theta;
      if (!(isfinite(omega) && isfinite(est))) {
        stop(ST_NONFINITE);
        return;
      }
      const double est_prev = SC(C, S_EST, c);  // ||r_j||^2 as the previous pass estimated it
      SC(C, S_OMEGA, c) = omega;
      SC(C, S_EST, c) = est;
      IS(C, I_RESTART, c) = 0;
      if (est < eps2) {
        pend = ST_CONVERGED;
        return;
      }
      if (omega == 0.0) {
        pend = ST_BREAKDOWN;
        return;
      }
      // rho_{j+1} = -omega psi rests on (rt, r0) = 0, which rounding meets
      // only up to an error that adds up pass by pass; E bounds it. Once
      // |rho_{j+1}| is down to u E the recurrence carries no information:
      // restart with the shadow vector r0 = r_{j+1} and rho_{j+1} = the stop
      // estimate of (r_{j+1}, r_{j+1}), beta = 0.
      const double rn = est_prev > 0.0 ? sqrt(est_prev) : 0.0;
      double err = SC(C, S_RE_ERR, c) + sqrt(SC(C, S_RE_SH, c)) * (rn + 2.0 * sqrt(eta) + 2.0 * fabs(omega) * sqrt(phi));
      double rho1 = -omega * psi;
      double beta;
      if (fabs(rho1) <= kRestartKappa * kU64 * err) {
        if (!(est > 0.0)) {
          pend = ST_BREAKDOWN;
          return;
        }
        rho1 = est;
        beta = 0.0;
        SC(C, S_RE_SH, c) = est;
        err = eta;
        IS(C, I_RESTART, c) = 1;
      } else {
        beta = (rho1 / SC(C, S_RHO, c)) * (SC(C, S_ALPHA, c) / omega);
        if (!isfinite(beta)) {
          stop(ST_NONFINITE);
          return;
        }
      }
      SC(C, S_RE_ERR, c) = err;
      SC(C, S_BETA, c) = beta;
      SC(C, S_RHONEXT, c) = rho1;
      return;
    }
    case F_IB_INIT: {
      // sigma_{-1} = pi_0 = tau_0 = 0, rho_0 = alpha_0 = omega_0 = 1
      const double sigma0 = D0, phi0 = D1;
      SC(C, S_SIGMA_PREV, c) = 0.0;
      SC(C, S_SIGMA, c) = sigma0;
      SC(C, S_OMEGA, c) = 1.0;
      const int bad = ib_open_pass(C, c, phi0, 0.0, 1.0, 0.0, sigma0, 1.0, 1.0, 0.0);
      // the first pass is entered and stops before its updates (unless maxit = 0)
      if (bad >= 0 && C.glob->maxit > 0) stop(bad);
      return;
    }
    case F_IB_OMEGA: {
      const double phi = D0, pi = D1, gamma = D2, eta = D3;
      const double theta = SC(C, S_D0 + 4, c), kappa = SC(C, S_D0 + 5, c), nu = SC(C, S_D0 + 6, c);
      const double omega = kappa != 0.0 ? theta / kappa : 0.0;
      const double sigma1 = gamma - omega * eta;
      const double est = nu - omega * theta;
      if (!(isfinite(omega) && isfinite(sigma1) && isfinite(est))) {
        stop(ST_NONFINITE);
        return;
      }
      SC(C, S_OMEGA, c) = omega;
      SC(C, S_EST, c) = est;
      record_history(C, c, SC(C, S_ALPHA, c), omega, SC(C, S_RHO, c), est);
      if (est < eps2)
        pend = ST_CONVERGED;
      else if (omega == 0.0)
        pend = ST_BREAKDOWN;
      const double sigma = SC(C, S_SIGMA, c);
      if (pend < 0)
        IS(C, I_PEND_NEXT, c) = ib_open_pass(C, c, phi, pi, omega, sigma, sigma1, SC(C, S_RHO, c),
                                             SC(C, S_ALPHA, c), SC(C, S_TAU, c));
      SC(C, S_SIGMA_PREV, c) = sigma;
      SC(C, S_SIGMA, c) = sigma1;
      return;
    }
    case F_IB_END: {
      // a stop found when forming the next pass's scalars is taken as that
      // pass starts (it counts as entered), unless maxit ends the solve first
      const int nx = IS(C, I_PEND_NEXT, c);
      if (pend < 0 && nx >= 0 && it1 < C.glob->maxit) {
        st = nx;
        IS(C, I_ITERS, c) = it1 + 1;
        return;
      }
      end_column(C, c);
      return;
    }
    case F_END: {
      record_history(C, c, SC(C, S_ALPHA, c), SC(C, S_OMEGA, c), SC(C, S_RHO, c), SC(C, S_EST, c));
      if (pend < 0) SC(C, S_RHO, c) = SC(C, S_RHONEXT, c);
      end_column(C, c);
      return;
    }
    case F_PIPE_INIT: {
      const double rw = D0;
      if (rw == 0.0) {
        st = ST_BREAKDOWN;
        IS(C, I_ITERS, c) = 0;
        return;
      }
      const double alpha = SC(C, S_RHO, c) / rw;
      if (!isfinite(alpha)) {
        st = ST_NONFINITE;
        IS(C, I_ITERS, c) = 0;
        return;
      }
      SC(C, S_ALPHA, c) = alpha;
      return;
    }
    case F_PIPE_OMEGA: {
      const double theta = D0, phi = D1, pi = D2;
      const double omega = phi != 0.0 ? theta / phi : 0.0;
      const double est = pi - omega * theta;
      if (!(isfinite(omega) && isfinite(est))) {
        stop(ST_NONFINITE);
        return;
      }
      SC(C, S_OMEGA, c) = omega;
      SC(C, S_EST, c) = est;
      if (est < eps2)
        pend = ST_CONVERGED;
      else if (omega == 0.0)
        pend = ST_BREAKDOWN;
      return;
    }
    case F_PIPE_BETA_END: {
      const double alpha = SC(C, S_ALPHA, c), omega = SC(C, S_OMEGA, c), rho = SC(C, S_RHO, c);
      if (pend < 0) {
        const double rho1 = D3, psi = SC(C, S_D0 + 4, c), sigma = SC(C, S_D0 + 5, c), delta = SC(C, S_D0 + 6, c);
        if (rho1 == 0.0) {
          stop(ST_BREAKDOWN);
          return;
        }
        const double beta = (alpha / omega) * (rho1 / rho);
        const double denom = sigma + beta * delta - beta * omega * psi;
        if (denom == 0.0) {
          stop(ST_BREAKDOWN);
          return;
        }
        const double alpha1 = rho1 / denom;
        if (!(isfinite(beta) && isfinite(alpha1))) {
          stop(ST_NONFINITE);
          return;
        }
        SC(C, S_BETA, c) = beta;
        SC(C, S_ALPHA, c) = alpha1;
        SC(C, S_RHO, c) = rho1;
      }
      record_history(C, c, alpha, omega, rho, SC(C, S_EST, c));
      end_column(C, c);
      return;
    }
    default:
      return;
  }
}

BCG_HD BCG_INLINE bool closes_iteration(int step) {
  return step == F_BETA_END || step == F_END || step == F_PIPE_BETA_END || step == F_IB_END;
}

// Run by thread 0 of the last workgroup after finalize_column.
BCG_HD inline void finalize_global(int step, const Ctl& C) {
  if (closes_iteration(step)) C.glob->it += 1;
  int nrun = 0;
  for (int c = 0; c < C.k; ++c) nrun += IS(C, I_STATUS, c) == ST_RUNNING;
  C.glob->nrun = nrun;
}

}  // namespace bcg
