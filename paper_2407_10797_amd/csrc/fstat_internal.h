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
struct PartConst {
  double tc;
  double mc_hi, mc_lo;     // Mc [s]
  double cN_hi, cN_lo, c1_hi, c1_lo, c15_hi, c15_lo, ce_hi, ce_lo;
  double c2, c5, c6, a6k, b6, ln_vfac;
  double c5v5;             // cN c5' vfac^5 (enters t_f)
  double k[3], u[3], v[3];
  double flo, fhi;
  int32_t j_lo, j_hi;      // support bins (inclusive); j_lo > j_hi when empty
  int32_t np;
  int32_t status;          // 0 ok, 1 empty support, 2 invalid parameters
};

enum { kStatusOk = 0, kStatusEmpty = 1, kStatusInvalid = 2 };

// ---- phase and SPA time -------------------------------------------------------
// Fractional cycle of Psi(f)/(2 pi) (constant phase offsets dropped: the
// F-statistic absorbs them) and the SPA time t_f = (1/2 pi) dPsi/df.
__host__ __device__ __forceinline__ void phase_and_tf(const PartConst& P, double f, double& frac,
                                             double& tf) {
  FSTAT_NO_CONTRACT
  dd ft = two_prod(f, P.tc);
  double c_ft = (ft.hi - floor(ft.hi)) + ft.lo;
  dd x = dd_mul_d(dd{P.mc_hi, P.mc_lo}, f);
  double lx = log(x.hi);
  // y = x^{-1/3}: y0 ~ 1 ulp, then one Newton step on x y^3 = 1
  double y0 = exp(lx * (-1.0 / 3.0));
  dd b = dd_mul(dd_mul_d(two_prod(y0, y0), y0), x);
  double r = (1.0 - b.hi) - b.lo;
  dd y = quick_two_sum(y0, y0 * r * (1.0 / 3.0));
  dd y2 = dd_mul(y, y);
  dd y3 = dd_mul(y2, y);
  dd y5 = dd_mul(y3, y2);
  dd y11 = dd_mul(dd_mul(y5, y5), y);
  dd w = dd_root(y, 3, exp(lx * (-1.0 / 9.0)));     // y^{1/3}
  dd tN = dd_mul(dd{P.cN_hi, P.cN_lo}, y5);
  dd t1 = dd_mul(dd{P.c1_hi, P.c1_lo}, y3);
  dd t15 = dd_mul(dd{P.c15_hi, P.c15_lo}, y2);
  dd te = dd_mul(dd_mul(dd{P.ce_hi, P.ce_lo}, y11), w);
  double lnv = P.ln_vfac + lx * (1.0 / 3.0);
  double t2 = P.c2 * y.hi;
  double t6 = P.c6 / y.hi;
  double small = t2 + P.c5 * lnv + t6 * (P.a6k + P.b6 * lnv);
  double ph = c_ft + dd_frac(tN) + dd_frac(t1) + dd_frac(t15) + dd_frac(te) + small;
  frac = ph - floor(ph);
  // t_f: a term c y^m = c x^{-m/3} contributes -(m/3) c y^m / f to dPsi/df/(2 pi)
  double D = (-5.0 / 3.0) * tN.hi - t1.hi - (2.0 / 3.0) * t15.hi - (1.0 / 3.0) * t2 + P.c5v5 +
             t6 * (P.a6k + P.b6 + P.b6 * lnv) * (1.0 / 3.0) - (34.0 / 9.0) * te.hi;
  tf = P.tc + D / f;
}

// ---- TDI-X response (particle-dependent part) --------------------------------
// Returns T'_+ and T'_x such that the full transfer is C(f) T', with the
// template-independent C(f) = (1 - z^2)(-i pi f L) exp(-i pi f L) folded into
// the per-bin data.  s0, c0 = sin, cos(pi f L).
__host__ __device__ __forceinline__ double sinc_from(double num, double den) {
  // num = sin(den) computed by angle addition; series near den = 0
  return (fabs(den) < 1e-6) ? 1.0 - den * den * (1.0 / 6.0) : num / den;
}

__host__ __device__ __forceinline__ void response_fp64(const PartConst& P, double f, double tf, double s0,
                                              double c0, double& tpr, double& tpi, double& txr,
                                              double& txi) {
  // orbit at t_f: alpha = 2 pi t / yr; spacecraft i at beta_i = 2 pi i / 3
  double sa, ca;
  sincospi(2.0 * tf * (1.0 / kYear), &sa, &ca);
  double c2a = ca * ca - sa * sa, s2a = 2.0 * sa * ca;
  const double q = kLs / (4.0 * kSqrt3);   // e R / 2
  const double hz = 0.5 * kLs;             // sqrt(3) e R
  const double cb1 = -0.5, sb1 = 0.5 * kSqrt3, cb2 = -0.5, sb2 = -0.5 * kSqrt3;
  // offsets d_i of spacecraft i from the guiding centre R (cos a, sin a, 0)
  double d0x = q * (c2a - 3.0), d0y = q * s2a, d0z = -hz * ca;
  double d1x = q * (c2a * cb1 + s2a * sb1 - 3.0 * cb1);
  double d1y = q * (s2a * cb1 - c2a * sb1 - 3.0 * sb1);
  double d1z = -hz * (ca * cb1 + sa * sb1);
  double d2x = q * (c2a * cb2 + s2a * sb2 - 3.0 * cb2);
  double d2y = q * (s2a * cb2 - c2a * sb2 - 3.0 * sb2);
  double d2z = -hz * (ca * cb2 + sa * sb2);
  const double kx = P.k[0], ky = P.k[1], kz = P.k[2];
  double kP2 = 2.0 * kRs * (kx * ca + ky * sa);   // 2 k . (guiding centre)
  double kd0 = kx * d0x + ky * d0y + kz * d0z;
  double kd1 = kx * d1x + ky * d1y + kz * d1z;
  double kd2 = kx * d2x + ky * d2y + kz * d2z;
  double x0 = kPi * kLs * f;
  double zr = c0 * c0 - s0 * s0, zi = -2.0 * s0 * c0;   // z = exp(-2 i pi f L)
  double out[2][4];  // per arm: (re, im) of E S, and F+, Fx
#pragma unroll
  for (int arm = 0; arm < 2; ++arm) {
    double ax = (arm == 0 ? d1x : d2x) - d0x;
    double ay = (arm == 0 ? d1y : d2y) - d0y;
    double az = (arm == 0 ? d1z : d2z) - d0z;
    double inv = 1.0 / sqrt(ax * ax + ay * ay + az * az);
    ax *= inv; ay *= inv; az *= inv;
    double kn = kx * ax + ky * ay + kz * az;
    double un = P.u[0] * ax + P.u[1] * ay + P.u[2] * az;
    double vn = P.v[0] * ax + P.v[1] * ay + P.v[2] * az;
    // propagation phase exp(-i pi f k.(p_0 + p_arm))
    double kp = kP2 + kd0 + (arm == 0 ? kd1 : kd2);
    double se, ce;
    sincospi(-f * kp, &se, &ce);
    // sinc(x0 (1 + kn)) + z sinc(x0 (1 - kn))
    double sq, cq;
    sincospi(kLs * f * kn, &sq, &cq);
    double sp = sinc_from(s0 * cq + c0 * sq, x0 * (1.0 + kn));
    double sm = sinc_from(s0 * cq - c0 * sq, x0 * (1.0 - kn));
    double Sr = sp + zr * sm, Si = zi * sm;
    out[arm][0] = ce * Sr - se * Si;
    out[arm][1] = ce * Si + se * Sr;
    out[arm][2] = un * un - vn * vn;
    out[arm][3] = 2.0 * un * vn;
  }
  // T' = F_b (E_b S_b) - F_a (E_a S_a)   (arm 0 = a: 1-2, arm 1 = b: 1-3)
  tpr = out[1][2] * out[1][0] - out[0][2] * out[0][0];
  tpi = out[1][2] * out[1][1] - out[0][2] * out[0][1];
  txr = out[1][3] * out[1][0] - out[0][3] * out[0][0];
  txi = out[1][3] * out[1][1] - out[0][3] * out[0][1];
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

}  // namespace fstat
