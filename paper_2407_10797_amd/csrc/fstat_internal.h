// fstat_internal.h -- device-side building blocks shared by the libfstat kernels.
//
// Physics (Fu, Wang & Mohanty, arXiv:2407.10797):
//   * template phase Psi(f) of App. A (TaylorF2 up to alpha_6 plus the
//     leading eccentric term), evaluated in cycles with double-double
//     arithmetic for every term that reaches 10^2..10^7 cycles, so that the
//     fractional cycle is exact to ~1e-14;
//   * SPA time t_f = (1/2pi) dPsi/df (Sec. IV) from the analytic derivative;
//   * zeroth-order TDI-X response at t_f (Sec. IV, Eq. freDres with N = 0) on
//     a rigid-arm, first-order analytic orbit.
// The template-independent factor of the TDI-X transfer, the f^{-7/6}
// amplitude, 1/S_n and 4 df are folded into per-bin data at plan time, so a
// bin needs only the particle-dependent part T'_{+,x} (see prep kernel).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fstat {

// ---- physical constants (SI; light-seconds for lengths) -------------------
constexpr double kMsunS = 4.925490947641267e-6;  // G Msun / c^3
constexpr double kYear = 31557600.0;             // Julian year
constexpr double kC = 299792458.0;
constexpr double kAU = 1.495978707e11;
constexpr double kArm = 2.5e9;
constexpr double kF0Ecc = 0.01;                  // e0 reference GW frequency
constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kLs = kArm / kC;                // arm light time [s]
constexpr double kRs = kAU / kC;                 // orbit radius [s]
constexpr double kSqrt3 = 1.7320508075688772935;
constexpr double kRankCut = 1e-12;               // singular-M eigenvalue ratio
constexpr int kSurMinNp = 16;                    // surrogate only in stages with Np >= 16

// ---- double-double helpers ---------------------------------------------------
// Error-free transformations must not be contracted: with fp-contract=fast the
// compiler may fuse an addition that consumes a rounded product into an FMA on
// the exact product, double-counting the product's error term.  Every function
// that builds or consumes double-double values switches contraction off.
#define FSTAT_NO_CONTRACT _Pragma("clang fp contract(off)")

struct dd {
  double hi, lo;
};

__host__ __device__ __forceinline__ dd two_prod(double a, double b) {
  FSTAT_NO_CONTRACT
  double p = a * b;
  return {p, __builtin_fma(a, b, -p)};
}
__host__ __device__ __forceinline__ dd two_sum(double a, double b) {
  FSTAT_NO_CONTRACT
  double s = a + b;
  double bb = s - a;
  return {s, (a - (s - bb)) + (b - bb)};
}
__host__ __device__ __forceinline__ dd quick_two_sum(double a, double b) {
  FSTAT_NO_CONTRACT
  double s = a + b;
  return {s, b - (s - a)};
}
__host__ __device__ __forceinline__ dd dd_add(dd a, dd b) {
  FSTAT_NO_CONTRACT
  dd s = two_sum(a.hi, b.hi);
  s.lo += a.lo + b.lo;
  return quick_two_sum(s.hi, s.lo);
}
__host__ __device__ __forceinline__ dd dd_mul(dd a, dd b) {
  FSTAT_NO_CONTRACT
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  FSTAT_NO_CONTRACT
  dd p = two_prod(a.hi, b);
  p.lo += a.lo * b;
  return quick_two_sum(p.hi, p.lo);
}
__host__ __device__ __forceinline__ dd dd_div(dd a, dd b) {
  FSTAT_NO_CONTRACT
  double q1 = a.hi / b.hi;
  dd r = dd_add(a, dd_mul_d(b, -q1));
  double q2 = r.hi / b.hi;
  return quick_two_sum(q1, q2);
}
// rational p/q as double-double
__host__ __device__ __forceinline__ dd dd_ratio(double p, double q) {
  FSTAT_NO_CONTRACT
  return dd_div(dd{p, 0.0}, dd{q, 0.0});
}
// x^(1/n), x > 0, as double-double: a double estimate w0 and one Newton step
// on w^n = x (quadratic convergence from ~1 ulp).
__host__ __device__ __forceinline__ dd dd_root(dd x, int n, double w0) {
  FSTAT_NO_CONTRACT
  dd wn = dd{w0, 0.0};
  for (int i = 1; i < n; ++i) wn = dd_mul_d(wn, w0);
  double r = ((x.hi - wn.hi) + (x.lo - wn.lo)) / x.hi;   // 1 - w0^n / x
  return quick_two_sum(w0, w0 * r / (double)n);
}
__host__ __device__ __forceinline__ double dd_frac(dd a) {
  FSTAT_NO_CONTRACT
  return (a.hi - floor(a.hi)) + a.lo;
}

// ---- per-particle constants (filled by the setup kernel) -------------------
// Phase in cycles, with x = Mc f, y = x^{-1/3}, v = (pi M f)^{1/3} = vfac / y
// (App. A; (3/128)(pi Mc f)^{-5/3} v^k / (2 pi) = cN vfac^k y^{5-k}):
//   Psi/(2 pi) = f t_c + cN y^5 + c1 y^3 + c15 y^2 + ce y^{34/3}     (double-double)
//              + c2 y + c5 ln v + (c6 / y)(a6k + b6 ln v) + const    (double)
// cN = 3/(256 pi^{8/3}); c1 = cN alpha_2 vfac^2; c15 = cN alpha_3 vfac^3;
// ce = cN (-2355/1462) e0^2 (f0 Mc)^{19/9}; c2 = cN alpha_4 vfac^4;
// c5 = 3 cN c5' vfac^5 with alpha_5 = c5'(1 + 3 ln(v sqrt 6)); c6 = cN vfac^6;
// alpha_6 = a6k + b6 ln v.  The terms that reach 10^2..10^7 cycles are
// carried as double-double, so the fractional cycle is exact to ~1e-14.
// Numerical orbit: nseg segments of length dt from t0, each a degree-9
// Chebyshev series per spacecraft and coordinate (positions in seconds of
// light travel), coef [nseg][3][3][10]; coef == nullptr: analytic orbit.
// Read-only device memory addressed through the constant address space, so
// that wave-uniform reads become scalar loads.
typedef __attribute__((address_space(4))) double kconst_double;
struct OrbitTable {
  const double* coef = nullptr;
  int32_t nseg = 0;
  double t0 = 0.0;
  double dt = 1.0;
};

struct PartConst {
  double tc;
  double mc_hi, mc_lo;     // Mc [s]
  double cN_hi, cN_lo, c1_hi, c1_lo, c15_hi, c15_lo, ce_hi, ce_lo;
  double c2, c5, c6, a6k, b6, ln_vfac;
  double c5v5;             // cN c5' vfac^5 (enters t_f)
  double ecc_k;            // -(2355/1462) e0^2: Psi_e = ecc_k (f0/f)^{19/9} Psi_N
  double nn_mc, nn_e0;     // surrogate inputs for Mc and e0, mapped to [-1, 1]
  double k[3], u[3], v[3];
  double flo, fhi;
  int32_t j_lo, j_hi;      // support bins (inclusive); j_lo > j_hi when empty
  int32_t np;
  int32_t status;          // 0 ok, 1 empty support, 2 invalid parameters
  int32_t sur;             // 1: eccentric term from the surrogate knots
  int32_t pad_;
};

enum { kStatusOk = 0, kStatusEmpty = 1, kStatusInvalid = 2 };

// ---- phase and SPA time -------------------------------------------------------
// Fractional cycle of Psi(f)/(2 pi) (constant phase offsets dropped: the
// F-statistic absorbs them) and the SPA time t_f = (1/2 pi) dPsi/df.
// Cubic Lagrange interpolation through four knots x_a (ek[0..3]) with
// coefficients c_a = value_a / prod_{b != a}(x_a - x_b) (ek[4..7]):
// I(f) = sum_a c_a prod_{b != a} (f - x_b).
__host__ __device__ __forceinline__ double knot_interp(const double* ek, double f) {
  double d0 = f - ek[0], d1 = f - ek[1], d2 = f - ek[2], d3 = f - ek[3];
  double d01 = d0 * d1, d23 = d2 * d3;
  return ek[4] * (d1 * d23) + ek[5] * (d0 * d23) + ek[6] * (d01 * d3) + ek[7] * (d01 * d2);
}

// ek == nullptr: analytic eccentric term; otherwise the eccentric term (cycles)
// is interpolated from the surrogate's knot values of the current partition.
__host__ __device__ __forceinline__ void phase_and_tf(const PartConst& P, double f, double& frac,
                                             double& tf, const double* ek = nullptr) {
  FSTAT_NO_CONTRACT
  dd ft = two_prod(f, P.tc);
  double c_ft = (ft.hi - floor(ft.hi)) + ft.lo;
  dd x = dd_mul_d(dd{P.mc_hi, P.mc_lo}, f);
  double lx = log(x.hi);
  // y = x^{-1/3}: y0 within a few ulp (the cube of w0 = x^{-1/9}, which the
  // eccentric term needs anyway), then one Newton step on x y^3 = 1
  const double w0 = ek ? 0.0 : exp(lx * (-1.0 / 9.0));
  double y0 = ek ? exp(lx * (-1.0 / 3.0)) : w0 * w0 * w0;
  dd b = dd_mul(dd_mul_d(two_prod(y0, y0), y0), x);
  double r = (1.0 - b.hi) - b.lo;
  dd y = quick_two_sum(y0, y0 * r * (1.0 / 3.0));
  dd y2 = dd_mul(y, y);
  dd y3 = dd_mul(y2, y);
  dd y5 = dd_mul(y3, y2);
  double xy2 = x.hi * y2.hi;                         // x^{1/3} = 1 / y
  dd tN = dd_mul(dd{P.cN_hi, P.cN_lo}, y5);
  dd t1 = dd_mul(dd{P.c1_hi, P.c1_lo}, y3);
  dd t15 = dd_mul(dd{P.c15_hi, P.c15_lo}, y2);
  dd te;
  if (ek) {
    te = dd{knot_interp(ek, f), 0.0};
  } else {
    // w = y^{1/3}: estimate w0, then one Newton step on w^3 = y
    dd w3 = dd_mul_d(two_prod(w0, w0), w0);
    double rw = ((y.hi - w3.hi) + (y.lo - w3.lo)) * xy2;
    dd w = quick_two_sum(w0, w0 * rw * (1.0 / 3.0));
    te = dd_mul(dd_mul(dd{P.ce_hi, P.ce_lo}, dd_mul(dd_mul(y5, y5), y)), w);
  }
  double lnv = P.ln_vfac + lx * (1.0 / 3.0);
  double t2 = P.c2 * y.hi;
  double t6 = P.c6 * xy2;
  double small = t2 + P.c5 * lnv + t6 * (P.a6k + P.b6 * lnv);
  double ph = c_ft + dd_frac(tN) + dd_frac(t1) + dd_frac(t15) + dd_frac(te) + small;
  frac = ph - floor(ph);
  // t_f: a term c y^m = c x^{-m/3} contributes -(m/3) c y^m / f to dPsi/df/(2 pi);
  // 1/f = Mc / x = Mc y^3
  double D = (-5.0 / 3.0) * tN.hi - t1.hi - (2.0 / 3.0) * t15.hi - (1.0 / 3.0) * t2 + P.c5v5 +
             t6 * (P.a6k + P.b6 + P.b6 * lnv) * (1.0 / 3.0) - (34.0 / 9.0) * te.hi;
  tf = P.tc + D * (P.mc_hi * y3.hi);
}

// The same phase unreduced (whole cycles kept, double-double) and t_f, at a
// frequency given as double-double: the interpolating bin loop takes phase
// differences across a work item from it, at node positions between bins,
// where rounding f to a double would move the phase by t_f * 1e-16 f
// (~1e-9 cycles at t_f ~ 1e8 s).
__host__ __device__ __forceinline__ dd phase_full(const PartConst& P, dd f, dd& tf,
                                                  const double* ek = nullptr) {
  FSTAT_NO_CONTRACT
  dd ft = dd_mul_d(f, P.tc);
  dd x = dd_mul(dd{P.mc_hi, P.mc_lo}, f);
  double lx = log(x.hi);
  const double w0 = ek ? 0.0 : exp(lx * (-1.0 / 9.0));   // as in phase_and_tf
  double y0 = ek ? exp(lx * (-1.0 / 3.0)) : w0 * w0 * w0;
  dd b = dd_mul(dd_mul_d(two_prod(y0, y0), y0), x);
  double r = (1.0 - b.hi) - b.lo;
  dd y = quick_two_sum(y0, y0 * r * (1.0 / 3.0));
  dd y2 = dd_mul(y, y);
  dd y3 = dd_mul(y2, y);
  dd y5 = dd_mul(y3, y2);
  double xy2 = x.hi * y2.hi;
  dd tN = dd_mul(dd{P.cN_hi, P.cN_lo}, y5);
  dd t1 = dd_mul(dd{P.c1_hi, P.c1_lo}, y3);
  dd t15 = dd_mul(dd{P.c15_hi, P.c15_lo}, y2);
  dd te;
  if (ek) {
    te = dd{knot_interp(ek, f.hi), 0.0};
  } else {
    dd w3 = dd_mul_d(two_prod(w0, w0), w0);
    double rw = ((y.hi - w3.hi) + (y.lo - w3.lo)) * xy2;
    dd w = quick_two_sum(w0, w0 * rw * (1.0 / 3.0));
    te = dd_mul(dd_mul(dd{P.ce_hi, P.ce_lo}, dd_mul(dd_mul(y5, y5), y)), w);
  }
  double lnv = P.ln_vfac + lx * (1.0 / 3.0);
  // the alpha_4 term reaches ~1e2 cycles: double-double too, so that its
  // rounding does not add ~1e-14-cycle noise between interpolation nodes
  dd t2d = dd_mul_d(y, P.c2);
  double t2 = t2d.hi;
  double t6 = P.c6 * xy2;
  double small = P.c5 * lnv + t6 * (P.a6k + P.b6 * lnv);
  dd ph = dd_add(dd_add(dd_add(ft, tN), dd_add(t1, t15)),
                 dd_add(te, dd_add(t2d, dd{small, 0.0})));
  // t_f in double-double as well: its rounding (1e-8 s at 1e8 s) would turn
  // the orbit angle and the 1000-s Doppler term into ~1e-13-cycle noise
  dd D = dd_add(dd_add(dd_mul_d(tN, -5.0 / 3.0), dd{-t1.hi, -t1.lo}),
                dd_add(dd_mul_d(t15, -2.0 / 3.0), dd_mul_d(te, -34.0 / 9.0)));
  D = dd_add(D, dd{-(1.0 / 3.0) * t2 + P.c5v5 + t6 * (P.a6k + P.b6 + P.b6 * lnv) * (1.0 / 3.0), 0.0});
  tf = dd_add(dd{P.tc, 0.0}, dd_mul(D, dd_mul(dd{P.mc_hi, P.mc_lo}, y3)));
  return ph;
}

// The same phase and t_f in plain FP64 (whole cycles kept): at ~1e7 cycles
// the phase rounds to ~2e-9 cycles, enough where the sine is taken in FP32
// (~6e-8 turns).  y = x^{-1/3} from w0^3 with one Newton step, as above.
__host__ __device__ __forceinline__ double phase_full_fp64(const PartConst& P, double f,
                                                           double& tf,
                                                           const double* ek = nullptr) {
  const double x = P.mc_hi * f;
  const double lx = log(x);
  const double w0 = ek ? 0.0 : exp(lx * (-1.0 / 9.0));
  const double y0 = ek ? exp(lx * (-1.0 / 3.0)) : w0 * w0 * w0;
  const double r = fma(-(y0 * y0) * y0, x, 1.0);
  const double y = fma(y0 * r, 1.0 / 3.0, y0);
  const double y2 = y * y, y3 = y2 * y, y5 = y3 * y2;
  const double xy2 = x * y2;
  const double tN = P.cN_hi * y5, t1 = P.c1_hi * y3, t15 = P.c15_hi * y2;
  const double te = ek ? knot_interp(ek, f) : P.ce_hi * (y5 * y5 * y) * w0;
  const double lnv = P.ln_vfac + lx * (1.0 / 3.0);
  const double t2 = P.c2 * y;
  const double t6 = P.c6 * xy2;
  const double small = P.c5 * lnv + t6 * (P.a6k + P.b6 * lnv);
  const double D = (-5.0 / 3.0) * tN - t1 - (2.0 / 3.0) * t15 - (1.0 / 3.0) * t2 + P.c5v5 +
                   t6 * (P.a6k + P.b6 + P.b6 * lnv) * (1.0 / 3.0) - (34.0 / 9.0) * te;
  tf = P.tc + D * (P.mc_hi * y3);
  return f * P.tc + (tN + ((t1 + t15) + (te + (t2 + small))));
}

// Per-particle phase coefficients (see PartConst), double-double where the
// term they multiply reaches 10^2..10^7 cycles.
__host__ __device__ inline void fill_constants(PartConst& P, const double* th) {
  FSTAT_NO_CONTRACT
  double tc = th[0], mc = th[1], dmu = th[2], theta = th[3], phi = th[4], e0 = th[5];
  P.tc = tc;
  dd m = two_prod(mc, kMsunS);                       // Mc [s], exact
  P.mc_hi = m.hi; P.mc_lo = m.lo;
  dd d2 = two_prod(dmu, dmu);
  dd one_m = dd_add(dd{1.0, 0.0}, dd{-d2.hi, -d2.lo});
  dd eta = dd{one_m.hi * 0.25, one_m.lo * 0.25};      // (1 - dmu^2)/4
  const dd pi = {3.141592653589793116e+00, 1.2246467991473532e-16};
  dd pi13 = dd_root(pi, 3, cbrt(pi.hi));
  dd ie5 = dd_root(dd_div(dd{1.0, 0.0}, eta), 5, pow(eta.hi, -0.2));   // eta^{-1/5}
  dd vfac = dd_mul(pi13, ie5);                        // v = vfac (Mc f)^{1/3}
  dd vf2 = dd_mul(vfac, vfac), vf3 = dd_mul(vf2, vfac);
  dd pi2 = dd_mul(pi, pi);
  dd cN = dd_div(dd{3.0, 0.0}, dd_mul_d(dd_mul(pi2, dd_mul(pi13, pi13)), 256.0));
  dd a2 = dd_add(dd_ratio(3715.0, 756.0), dd_mul(dd_ratio(55.0, 9.0), eta));
  dd c1 = dd_mul(dd_mul(cN, a2), vf2);
  dd c15 = dd_mul(dd_mul(cN, dd_mul_d(pi, -16.0)), vf3);
  dd z = dd_mul_d(m, kF0Ecc);                         // f0 Mc
  dd z19 = dd_mul(dd_mul(z, z), dd_root(z, 9, pow(z.hi, 1.0 / 9.0)));   // (f0 Mc)^{19/9}
  dd ce = dd_mul(dd_mul(cN, dd_ratio(-2355.0, 1462.0)), dd_mul(two_prod(e0, e0), z19));
  P.cN_hi = cN.hi; P.cN_lo = cN.lo;
  P.c1_hi = c1.hi; P.c1_lo = c1.lo;
  P.c15_hi = c15.hi; P.c15_lo = c15.lo;
  P.ce_hi = ce.hi; P.ce_lo = ce.lo;
  double et = eta.hi, vf = vfac.hi, K = cN.hi;
  const double pisq = kPi * kPi;
  double a4 = 15293365.0 / 508032.0 + 27145.0 * et / 504.0 + 3085.0 * et * et / 72.0;
  double c5p = kPi * (38645.0 / 756.0 - 65.0 * et / 9.0);
  const double euler = 0.57721566490153286061;
  double a6c = 11583231236531.0 / 4694215680.0 - 640.0 * pisq / 3.0 - 6848.0 * euler / 21.0 +
               (-15737765635.0 / 3048192.0 + 2255.0 * pisq / 12.0) * et +
               76055.0 * et * et / 1728.0 - 127825.0 * et * et * et / 1296.0;
  double vf4 = vf * vf * vf * vf, vf5 = vf4 * vf, vf6 = vf5 * vf;
  P.c2 = K * a4 * vf4;
  P.c5v5 = K * c5p * vf5;
  P.c5 = 3.0 * P.c5v5;
  P.c6 = K * vf6;
  P.b6 = -6848.0 / 21.0;
  P.a6k = a6c + P.b6 * log(4.0);
  P.ln_vfac = log(vf);
  P.ecc_k = -(2355.0 / 1462.0) * e0 * e0;
  P.nn_mc = (mc - 30.0) / 20.0;
  P.nn_e0 = e0 / 0.075 - 1.0;
  P.sur = 0;
  P.pad_ = 0;
  double st, ct, sp, cp;
  sincos(theta, &st, &ct);
  sincos(phi, &sp, &cp);
  P.k[0] = -st * cp; P.k[1] = -st * sp; P.k[2] = -ct;
  P.u[0] = ct * cp;  P.u[1] = ct * sp;  P.u[2] = -st;
  P.v[0] = sp;       P.v[1] = -cp;      P.v[2] = 0.0;
}

// Newtonian and eccentric phase terms (cycles) of the plain template at f:
// tN = cN y^5 and te = ce y^{34/3} (App. A), in double precision; used to
// build the surrogate's training targets and to check its knot values.
__host__ __device__ __forceinline__ void newton_and_ecc(const PartConst& P, double f, double& tN,
                                                       double& te) {
  FSTAT_NO_CONTRACT
  dd x = dd_mul_d(dd{P.mc_hi, P.mc_lo}, f);
  double lx = log(x.hi);
  double y = exp(lx * (-1.0 / 3.0));
  double y5 = y * y * y * y * y;
  tN = (P.cN_hi + P.cN_lo) * y5;
  te = (P.ce_hi + P.ce_lo) * y5 * y5 * y * exp(lx * (-1.0 / 9.0));
}

// ---- per-bin template (particle-dependent part) -------------------------------
// Full basis template (Sec. II.A, Eq. response; Sec. IV, Eq. freDres, N = 0):
//   A^1 = C(f) f^{-7/6} e^{-i Phi} T''_+,  Phi = Psi + 2 pi f k.p_1,
// with C(f) = (1 - z^2)(-i pi f L) e^{-i pi f L} folded into the per-bin data,
// and for a rigid constellation (arms of length L along the orbit's arm
// directions n_a = 1->2, n_b = 1->3) the link propagation phase
// e^{-i pi f k.(p_s + p_r)} = e^{-2 pi i f k.p_1} e^{-i pi f L k.n}: the common
// factor joins the template phase, the arm factor reuses the sincos of the
// link sinc argument.  Per arm
//   S = e^{-i x0 kn} [sinc(x0 (1 + kn)) + z sinc(x0 (1 - kn))],  x0 = pi f L,
//   T''_P = F^P_b S_b - F^P_a S_a,  F^+ = (u.n)^2 - (v.n)^2,  F^x = 2 (u.n)(v.n).
__host__ __device__ __forceinline__ double sinc_from(double num, double den) {
  // num = sin(den) computed by angle addition; series near den = 0
  return (fabs(den) < 1e-6) ? 1.0 - den * den * (1.0 / 6.0) : num / den;
}

// a * b + c as one three-operand FMA into a fresh register, a wave-uniform
// (a scalar register: constants cost scalar moves, not vector ones)
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "s"(a), "v"(b), "v"(c));
  return d;
}

// sin(2 pi r), cos(2 pi r) for |r| < 2^22 turns: r = n / kSinTab + x with x
// exact and |x| <= 1 / (2 kSinTab); the coarse factor from the LDS table, the
// fine one from short Taylor series (sin to theta^5, cos to theta^6:
// remainders below 1e-19 for |theta| <= pi / kSinTab), combined by the
// angle-addition formulas.  In the bin loop |r| stays below ~1e4 turns (the
// item's start phase is below one turn, the linear term below half a turn
// per bin, the residual a few hundred turns at most).
constexpr int kSinTab = 512;
__device__ __forceinline__ void sincos_tab(double r, const double2* tab, double& s, double& c) {
  const double n = rint(r * (double)kSinTab);
  const double x = fma(-1.0 / (double)kSinTab, n, r);
  const double2 e = tab[(int)n & (kSinTab - 1)];
  const double th = x * 6.283185307179586477;
  const double z = th * th;
  const double ps = fma3(1.0 / 120.0, z, -1.0 / 6.0);
  const double pc = fma(fma3(-1.0 / 720.0, z, 1.0 / 24.0), z, -0.5);
  const double sl = fma(th * z, ps, th);
  const double cl = fma(z, pc, 1.0);
  s = fma(e.x, cl, e.y * sl);
  c = fma(e.y, cl, -(e.x * sl));
}

// (sin, cos)(2 pi k / kSinTab) into a block's LDS table; every thread of the
// block calls it (it ends with a block barrier).
__device__ __forceinline__ void fill_sincos_table(double2* tab) {
  for (int k = threadIdx.x; k < kSinTab; k += blockDim.x) {
    double sv, cv;
    sincospi(2.0 * (double)k / (double)kSinTab, &sv, &cv);
    tab[k] = make_double2(sv, cv);
  }
  __syncthreads();
}

// sin(pi x), cos(pi x): from the table when one is given, else the library.
__device__ __forceinline__ void sincospi_t(double x, const double2* tab, double* s, double* c) {
  if (tab) sincos_tab(0.5 * x, tab, *s, *c);
  else sincospi(x, s, c);
}

// hardware reciprocal / reciprocal square root seeds refined by two Newton
// steps (accurate to about one ulp)
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  r = r * __builtin_fma(-h * r, r, 1.5);
  return r * __builtin_fma(-h * r, r, 1.5);
}

// spacecraft offsets from the guiding centre R (cos a, sin a, 0) for the
// first-order analytic orbit: beta_i = 2 pi i / 3, e R / 2 = L / (4 sqrt 3),
// sqrt(3) e R = L / 2
template <typename T>
__device__ __forceinline__ void orbit_offsets(T ca, T sa, T d[3][3]) {
  const T q = (T)(kLs / (4.0 * kSqrt3));
  const T hz = (T)(0.5 * kLs);
  const T cb[3] = {(T)1.0, (T)-0.5, (T)-0.5};
  const T sb[3] = {(T)0.0, (T)(0.5 * kSqrt3), (T)(-0.5 * kSqrt3)};
  T c2a = ca * ca - sa * sa, s2a = (T)2.0 * sa * ca;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    d[i][0] = q * (c2a * cb[i] + s2a * sb[i] - (T)3.0 * cb[i]);
    d[i][1] = q * (s2a * cb[i] - c2a * sb[i] - (T)3.0 * sb[i]);
    d[i][2] = -hz * (ca * cb[i] + sa * sb[i]);
  }
}

// Channel codes (Grid::chan): weights of M_0 = X, M_1 = Y, M_2 = Z in a channel
__device__ __forceinline__ void channel_weights(int code, double w[3]) {
  const double r2 = 0.70710678118654752440, r6 = 0.40824829046386301637,
               r3 = 0.57735026918962576451;
  w[0] = w[1] = w[2] = 0.0;
  if (code <= 2) w[code] = 1.0;
  else if (code == 3) { w[0] = -r2; w[2] = r2; }
  else if (code == 4) { w[0] = r6; w[1] = -2.0 * r6; w[2] = r6; }
  else { w[0] = w[1] = w[2] = r3; }
}

// TDI transfer (T''_+, T''_x) at f of the Michelson combination at spacecraft
// a (a = 0: X) relative to the phase reference p_1: arms from p_a to p_{a+1},
// p_{a+2}, and the factor exp(-2 pi i f k.(p_a - p_1)) of the vertex's offset.
// d are the spacecraft offsets, s0, c0 = sin, cos(pi f L).  Delays and sinc
// arguments take the nominal arm length L.  The link phase pi f k.(p_s + p_r)
// takes L n for the arm vector on the analytic (rigid) constellation, the arm
// vector itself when `table` (a numerical orbit, whose arms need not have
// length L).
__device__ __forceinline__ void michelson_fp64(const PartConst& P, double f, double s0, double c0,
                                               const double d[3][3], int a, double& tpr,
                                               double& tpi, double& txr, double& txi,
                                               bool table = false, const double2* tab = nullptr) {
  const double kx = P.k[0], ky = P.k[1], kz = P.k[2];
  const double x0 = kPi * kLs * f;
  const double zr = c0 * c0 - s0 * s0, zi = -2.0 * s0 * c0;   // z = e^{-2 i x0}
  double out[2][4];
#pragma unroll
  for (int arm = 0; arm < 2; ++arm) {
    const int w = (a + 1 + arm) % 3;
    double ax = d[w][0] - d[a][0], ay = d[w][1] - d[a][1], az = d[w][2] - d[a][2];
    const double r2 = ax * ax + ay * ay + az * az;
    double inv = rsq_nr(r2);
    ax *= inv; ay *= inv; az *= inv;
    double kn = kx * ax + ky * ay + kz * az;
    double un = P.u[0] * ax + P.u[1] * ay + P.u[2] * az;
    double vn = P.v[0] * ax + P.v[1] * ay + P.v[2] * az;
    double sq, cq;
    sincospi_t(kLs * f * kn, tab, &sq, &cq);
    double np_ = s0 * cq + c0 * sq, nm = s0 * cq - c0 * sq;   // sin(x0 (1 +- kn))
    double dp = x0 * (1.0 + kn), dm = x0 * (1.0 - kn);
    double sp, sm;
    if (fabs(dp) > 1e-6 && fabs(dm) > 1e-6) {
      double r = rcp_nr(dp * dm);
      sp = np_ * dm * r;
      sm = nm * dp * r;
    } else {
      sp = sinc_from(np_, dp);
      sm = sinc_from(nm, dm);
    }
    double Sr = sp + zr * sm, Si = zi * sm;
    if (table) {   // link phase from the arm vector: rotate by exp(-i pi f kn (|d| - L))
      double se, ce;
      sincospi_t(f * kn * (r2 * inv - kLs), tab, &se, &ce);
      const double tr = sq * ce + cq * se, tc = cq * ce - sq * se;
      sq = tr;
      cq = tc;
    }
    out[arm][0] = cq * Sr + sq * Si;      // e^{-i x0 kn} S
    out[arm][1] = cq * Si - sq * Sr;
    out[arm][2] = un * un - vn * vn;
    out[arm][3] = 2.0 * un * vn;
  }
  double pr = out[1][2] * out[1][0] - out[0][2] * out[0][0];
  double pi = out[1][2] * out[1][1] - out[0][2] * out[0][1];
  double xr = out[1][3] * out[1][0] - out[0][3] * out[0][0];
  double xi = out[1][3] * out[1][1] - out[0][3] * out[0][1];
  if (a != 0) {
    const double kd = kx * (d[a][0] - d[0][0]) + ky * (d[a][1] - d[0][1]) + kz * (d[a][2] - d[0][2]);
    double sv, cv;
    sincospi_t(2.0 * f * kd, tab, &sv, &cv);   // e^{-i 2 pi f kd} = cv - i sv
    const double r0 = pr * cv + pi * sv, i0 = pi * cv - pr * sv;
    const double r1 = xr * cv + xi * sv, i1 = xi * cv - xr * sv;
    pr = r0; pi = i0; xr = r1; xi = i1;
  }
  tpr = pr; tpi = pi; txr = xr; txi = xi;
}

// Transfer of channel `code` (relative to the phase reference p_1).
__device__ __forceinline__ void response_ch_fp64(const PartConst& P, double f, double s0, double c0,
                                                 const double d[3][3], int code, double& tpr,
                                                 double& tpi, double& txr, double& txi,
                                                 bool table = false, const double2* tab = nullptr) {
  double w[3];
  channel_weights(code, w);
  tpr = tpi = txr = txi = 0.0;
  // one copy of the Michelson code in a rolled loop: unrolled, the three
  // copies raise the kernels' register use above the occupancy limit
#pragma unroll 1
  for (int a = 0; a < 3; ++a) {
    if (w[a] == 0.0) continue;
    double pr, pi, xr, xi;
    michelson_fp64(P, f, s0, c0, d, a, pr, pi, xr, xi, table, tab);
    tpr = fma(w[a], pr, tpr); tpi = fma(w[a], pi, tpi);
    txr = fma(w[a], xr, txr); txi = fma(w[a], xi, txi);
  }
}

// The nine degree-9 Chebyshev series of one table segment at x in [-1, 1]
// (Clenshaw's recurrence), coefficients c[9][10].
template <typename C>
__device__ __forceinline__ void clenshaw_positions(const C* c, double x, double p[3][3]) {
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const C* cq = c + 10 * q;
    double b1 = 0.0, b2 = 0.0;
#pragma unroll
    for (int k = 9; k >= 1; --k) {
      const double b0 = fma(2.0 * x, b1, cq[k] - b2);
      b2 = b1;
      b1 = b0;
    }
    p[q / 3][q % 3] = fma(x, b1, cq[0] - b2);
  }
}

// Spacecraft positions [s] at time t = th + tl (tl = 0 for a plain double)
// from an orbit table: Clenshaw on the segment that holds t (the first or last
// segment outside the table).  The offset from the segment's start is formed
// without rounding t itself (whose ulp at 1e8 s, 1.5e-8 s, would move the
// positions by ~1e-12 s and the Doppler phase by ~1e-13 cycles).
__device__ __forceinline__ void table_positions(const OrbitTable& o, double th, double tl,
                                                double p[3][3]) {
  int seg;
  double x;
  {
    FSTAT_NO_CONTRACT
    const dd a = two_sum(th, -o.t0);                      // t - t0
    seg = (int)floor(a.hi / o.dt);
    seg = min(max(seg, 0), o.nseg - 1);
    const dd s0 = two_prod(o.dt, (double)seg);            // segment start - t0
    // a.hi - s0.hi is exact inside the table (the two are within a factor 2)
    const double loc = (a.hi - s0.hi) + ((a.lo - s0.lo) + tl);
    x = 2.0 * loc / o.dt - 1.0;
  }
  // All active lanes in one segment (the usual case): its coefficients are
  // read through the scalar cache (wave-uniform address, read only);
  // otherwise each lane reads its own segment's.
  const int s = __builtin_amdgcn_readfirstlane(seg);
  if (__builtin_amdgcn_ballot_w64(seg != s) == 0)
    clenshaw_positions((const kconst_double*)(o.coef + (int64_t)s * 90), x, p);
  else
    clenshaw_positions(o.coef + (int64_t)seg * 90, x, p);
}

// k . p_1 from the table, with d[i] = p_i - p_1 (the response uses only
// differences of the d and k . (d_a - d_0)).
__device__ __forceinline__ double k_dot_p1_table(const PartConst& P, const OrbitTable& o, double th,
                                                 double tl, double d[3][3]) {
  double p[3][3];
  table_positions(o, th, tl, p);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) d[i][c] = p[i][c] - p[0][c];
  return P.k[0] * p[0][0] + P.k[1] * p[0][1] + P.k[2] * p[0][2];
}

// k . p_1 [s] of spacecraft 1 at orbit angle (ca, sa); fills the offsets d
__device__ __forceinline__ double k_dot_p1(const PartConst& P, double ca, double sa, double d[3][3]) {
  orbit_offsets<double>(ca, sa, d);
  const double kx = P.k[0], ky = P.k[1], kz = P.k[2];
  return kRs * (kx * ca + ky * sa) + (kx * d[0][0] + ky * d[0][1] + kz * d[0][2]);
}

__device__ __forceinline__ void template_fp64(const PartConst& P, double f, double s0, double c0,
                                              double& cph, double& sph, double& tpr,
                                              double& tpi, double& txr, double& txi,
                                              const double* ek = nullptr, int code = 0,
                                              const OrbitTable* orb = nullptr,
                                              const double2* tab = nullptr) {
  double fr, tf;
  phase_and_tf(P, f, fr, tf, ek);
  double d[3][3];
  double kp1;
  if (orb && orb->coef) {
    kp1 = k_dot_p1_table(P, *orb, tf, 0.0, d);
  } else {
    double sa, ca;
    sincospi_t(2.0 * tf * (1.0 / kYear), tab, &sa, &ca);
    kp1 = k_dot_p1(P, ca, sa, d);
  }
  double ph = fr + f * kp1;               // Phi / (2 pi) in cycles
  ph -= rint(ph);
  sincospi_t(2.0 * ph, tab, &sph, &cph);
  response_ch_fp64(P, f, s0, c0, d, code, tpr, tpi, txr, txi, orb && orb->coef, tab);
}

// The template at an arbitrary frequency fd (double-double; an interpolation
// node): the whole phase Phi / (2 pi) = Psi / (2 pi) + f k.p_1 in cycles
// (double-double, not reduced) and the transfer without the Doppler factor.
__device__ __forceinline__ dd template_node(const PartConst& P, dd fd, const double* ek,
                                            double& tpr, double& tpi, double& txr, double& txi,
                                            int code = 0, const OrbitTable* orb = nullptr,
                                            const double2* tab = nullptr) {
  dd tf;
  dd ph = phase_full(P, fd, tf, ek);
  const double f = fd.hi;
  double d[3][3];
  double kp1;
  if (orb && orb->coef) {
    kp1 = k_dot_p1_table(P, *orb, tf.hi, tf.lo, d);
  } else {
    double sa, ca;
    {
      FSTAT_NO_CONTRACT
      const dd turns = dd_mul_d(tf, 1.0 / kYear);     // orbit angle in turns, reduced exactly
      sincospi_t(2.0 * ((turns.hi - floor(turns.hi)) + turns.lo), tab, &sa, &ca);
    }
    kp1 = k_dot_p1(P, ca, sa, d);
  }
  double s0, c0;
  sincospi_t(kLs * f, tab, &s0, &c0);
  response_ch_fp64(P, f, s0, c0, d, code, tpr, tpi, txr, txi, orb && orb->coef, tab);
  return dd_add(ph, dd_mul_d(fd, kp1));
}

// The same node template in plain FP64 (the mixed path's interpolation nodes).
__device__ __forceinline__ double template_node_fp64(const PartConst& P, double f, const double* ek,
                                                     double& tpr, double& tpi, double& txr,
                                                     double& txi, int code = 0,
                                                     const OrbitTable* orb = nullptr,
                                                     const double2* tab = nullptr) {
  double tf;
  const double ph = phase_full_fp64(P, f, tf, ek);
  double d[3][3];
  double kp1;
  if (orb && orb->coef) {
    kp1 = k_dot_p1_table(P, *orb, tf, 0.0, d);
  } else {
    double sa, ca;
    sincospi_t(2.0 * tf * (1.0 / kYear), tab, &sa, &ca);
    kp1 = k_dot_p1(P, ca, sa, d);
  }
  double s0, c0;
  sincospi_t(kLs * f, tab, &s0, &c0);
  response_ch_fp64(P, f, s0, c0, d, code, tpr, tpi, txr, txi, orb && orb->coef, tab);
  return fma(f, kp1, ph);
}

// ---- per-partition solve (2x2 Hermitian closed form) --------------------------
// acc = {Re Z+, Im Z+, Re Zx, Im Zx, P, Q, Re R, Im R};  F = 1/2 z^H H^{-1} z,
// H = [[P, conj R], [R, Q]] is the complex form of the real 4x4 M of
// Eq. coherent_F_stat; rank-deficient H uses the pseudo-inverse.
__host__ __device__ __forceinline__ double solve_partition(const double* a) {
  double zpr = a[0], zpi = a[1], zxr = a[2], zxi = a[3];
  double P = a[4], Q = a[5], rr = a[6], ri = a[7];
  double hs = 0.5 * (P + Q), hd = 0.5 * (P - Q);
  double rad = sqrt(hd * hd + rr * rr + ri * ri);
  double lp = hs + rad;
  if (!(lp > 0.0)) return 0.0;
  double det = P * Q - (rr * rr + ri * ri);
  double lm = det / lp;
  double zp2 = zpr * zpr + zpi * zpi, zx2 = zxr * zxr + zxi * zxi;
  if (lm > kRankCut * lp) {
    double cross = (rr * zpr - ri * zpi) * zxr + (rr * zpi + ri * zpr) * zxi;
    return (Q * zp2 + P * zx2 - 2.0 * cross) / (2.0 * det);
  }
  // rank one: eigenvector of lambda_+ ; pick the better-conditioned form
  double v1r, v1i, v2r, v2i;
  if (P >= Q) { v1r = lp - Q; v1i = 0.0; v2r = rr; v2i = ri; }      // (lp - Q, R)
  else        { v1r = rr; v1i = -ri; v2r = lp - P; v2i = 0.0; }     // (conj R, lp - P)
  double n2 = v1r * v1r + v1i * v1i + v2r * v2r + v2i * v2i;
  if (!(n2 > 0.0)) return 0.0;
  // v^H z
  double pr = v1r * zpr + v1i * zpi + v2r * zxr + v2i * zxi;
  double pi = v1r * zpi - v1i * zpr + v2r * zxi - v2i * zxr;
  return 0.5 * (pr * pr + pi * pi) / (lp * n2);
}

// ---- maximum-likelihood amplitudes of a partition (Eq. aandMN3) -------------
// The log-likelihood over the complex pair beta = (beta_+, beta_x) of the
// templates (T+ g, Tx g) is Re(beta^H z) - 1/2 beta^H H beta (up to the bin
// weighting), maximised by beta = H^{-1} z; when H is rank deficient the
// pseudo-inverse keeps the lambda_+ eigendirection only (the minimum-norm
// maximiser).  acc as for solve_partition; out {Re, Im} beta_+, {Re, Im} beta_x.
__host__ __device__ __forceinline__ void solve_beta(const double* a, double* out) {
  double zpr = a[0], zpi = a[1], zxr = a[2], zxi = a[3];
  double P = a[4], Q = a[5], rr = a[6], ri = a[7];
  for (int k = 0; k < 4; ++k) out[k] = 0.0;
  double hs = 0.5 * (P + Q), hd = 0.5 * (P - Q);
  double rad = sqrt(hd * hd + rr * rr + ri * ri);
  double lp = hs + rad;
  if (!(lp > 0.0)) return;
  double det = P * Q - (rr * rr + ri * ri);
  double lm = det / lp;
  if (lm > kRankCut * lp) {
    // H^{-1} = [[Q, -conj R], [-R, P]] / det
    double cxr = rr * zxr + ri * zxi, cxi = rr * zxi - ri * zxr;   // conj(R) z_x
    double rpr = rr * zpr - ri * zpi, rpi = rr * zpi + ri * zpr;   // R z_+
    out[0] = (Q * zpr - cxr) / det;
    out[1] = (Q * zpi - cxi) / det;
    out[2] = (P * zxr - rpr) / det;
    out[3] = (P * zxi - rpi) / det;
    return;
  }
  double v1r, v1i, v2r, v2i;
  if (P >= Q) { v1r = lp - Q; v1i = 0.0; v2r = rr; v2i = ri; }
  else        { v1r = rr; v1i = -ri; v2r = lp - P; v2i = 0.0; }
  double n2 = v1r * v1r + v1i * v1i + v2r * v2r + v2i * v2i;
  if (!(n2 > 0.0)) return;
  double pr = v1r * zpr + v1i * zpi + v2r * zxr + v2i * zxi;     // v^H z
  double pi = v1r * zpi - v1i * zpr + v2r * zxi - v2i * zxr;
  double sr = pr / (lp * n2), si = pi / (lp * n2);
  out[0] = v1r * sr - v1i * si;
  out[1] = v1r * si + v1i * sr;
  out[2] = v2r * sr - v2i * si;
  out[3] = v2r * si + v2i * sr;
}

}  // namespace fstat
