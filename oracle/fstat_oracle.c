/*
 * fstat_oracle.c -- plain, slow, FP64 CPU reference for the semi-coherent
 * F-statistic of eccentric inspirals seen through one TDI-X channel.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path: every constant below is typed here independently.
 *
 * What it computes (Fu, Wang & Mohanty 2024, arXiv:2407.10797):
 *   - the noise-weighted inner product <a,b> = 4 Re sum_k a_k conj(b_k) / S_k df
 *     (Sec. II.A, Eq. "inner_product", discretised on the rFFT grid);
 *   - the restricted-PN frequency-domain waveform  f^{-7/6} exp(-i Psi(f)) with
 *     Psi = 2 pi f t_c - phi_c - pi/4 + (3/128)(pi Mc f)^{-5/3} sum_k alpha_k v^k
 *     + Psi_e(f)  (App. A);
 *   - the SPA time t_f = (1/2pi) dPsi/df (Sec. IV) and the zeroth-order
 *     frequency-domain TDI response  x(f) = T(f) h(f)  evaluated at t_f (Sec. IV,
 *     Eq. "freDres" with N = 0);
 *   - four explicit real-amplitude basis templates A^i (Sec. II.A, Eq.
 *     "response"; the amplitude map of App. B), N^i = <s|A^i>, M^ij = <A^i|A^j>
 *     and the coherent statistic F = 1/2 N^T M^{-1} N (Eq. "coherent_F_stat");
 *   - the semi-coherent mean over Np frequency partitions whose outer limits are
 *     the template's lowest and highest instantaneous frequency during the
 *     observation (Sec. II.B, Eq. "semi-cohF").
 *
 * Readings of points the paper leaves open (PN coefficients, eccentric phase,
 * orbit, TDI-X combination, partition widths, singular M) are listed with the
 * repository's design notes; each is marked where it is used below.
 *
 * Precision: the template phase reaches 10^7 cycles, so it is evaluated in
 * IEEE binary128 (__float128) and reduced modulo one cycle before the
 * trigonometric functions are taken in double; t_f uses x87 extended
 * precision.  All other arithmetic is plain double with compensated
 * (Neumaier) summation.
 *
 * Parity status of each function is stated in its header comment.
 */
#include <math.h>
#include <quadmath.h>
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- physical constants (SI) ------------------------------------------- */
static const double OR_MSUN_S = 4.925490947641267e-6; /* G Msun / c^3  [s]   */
static const double OR_YEAR_S = 31557600.0;           /* Julian year [s]     */
static const double OR_C = 299792458.0;               /* speed of light      */
static const double OR_AU_M = 1.495978707e11;         /* astronomical unit   */
static const double OR_ARM_M = 2.5e9;                 /* nominal arm length  */
static const double OR_F0_ECC = 0.01;                 /* e0 reference f_gw   */
static const long double OR_PI_L = 3.141592653589793238462643383279502884L;
static const long double OR_EULER_L = 0.577215664901532860606512090082402431L;
static const double OR_PI = 3.14159265358979323846;

/* PN order switch used only by the Newtonian-limit pin: 0 keeps alpha_0
 * alone, anything >= 6 keeps every term up to alpha_6 (the paper's k <= 6). */
static int g_pn_order = 6;
void or_set_pn_order(int order) { g_pn_order = order; }
int or_get_pn_order(void) { return g_pn_order; }

/* ---- intrinsic parameters --------------------------------------------- */
/* theta6 = {t_c [s], Mc [Msun], delta_mu, theta [rad], phi [rad], e0} (Sec. II.A) */
typedef struct {
  double tc, mc, dmu, theta, phi, e0;
} or_intr;

static or_intr unpack(const double *t6) {
  or_intr p;
  p.tc = t6[0]; p.mc = t6[1]; p.dmu = t6[2];
  p.theta = t6[3]; p.phi = t6[4]; p.e0 = t6[5];
  return p;
}

static int params_ok(const or_intr *p) {
  return isfinite(p->tc) && isfinite(p->mc) && isfinite(p->dmu) &&
         isfinite(p->theta) && isfinite(p->phi) && isfinite(p->e0) &&
         p->mc > 0.0 && fabs(p->dmu) < 1.0 && p->e0 >= 0.0;
}

/* ---- App. A: template phase ------------------------------------------- */
/* Symmetric mass ratio from the dimensionless mass difference
 * delta_mu = (m1 - m2)/M, so eta = m1 m2 / M^2 = (1 - delta_mu^2)/4. */
static long double eta_of(const or_intr *p) {
  long double d = (long double)p->dmu;
  return (1.0L - d * d) / 4.0L;
}

/* The phase reaches 10^7 cycles and the statistic is sensitive to phase
 * errors of order 1e-12 rad (amplified by the conditioning of M), so the
 * phase is evaluated in IEEE binary128 (__float128, 113-bit significand):
 * per-particle quantities once, then three quad transcendentals per bin.  */
typedef __float128 qd;
static const qd OR_PI_Q = 3.14159265358979323846264338327950288Q;
static const qd OR_EULER_Q = 0.57721566490153286060651209008240243Q;

typedef struct {
  qd tc, mc, eta, m;              /* t_c [s], Mc [s], eta, M = Mc eta^{-3/5} [s] */
  qd a2, a3, a4, c5, a6c, b6, e0sq;
} or_pq;

static or_pq phase_consts(const or_intr *p) {
  or_pq c;
  const qd pi = OR_PI_Q;
  qd d = (qd)p->dmu;
  c.tc = (qd)p->tc;
  c.mc = (qd)p->mc * (qd)OR_MSUN_S;
  c.eta = (1 - d * d) / 4;
  c.m = c.mc * powq(c.eta, -0.6Q);
  qd eta = c.eta;
  c.a2 = 3715.0Q / 756 + 55 * eta / 9;
  c.a3 = -16 * pi;
  c.a4 = 15293365.0Q / 508032 + 27145 * eta / 504 + 3085 * eta * eta / 72;
  c.c5 = pi * (38645.0Q / 756 - 65 * eta / 9);
  c.a6c = 11583231236531.0Q / 4694215680 - 640 * pi * pi / 3 - 6848 * OR_EULER_Q / 21 +
          (-15737765635.0Q / 3048192 + 2255 * pi * pi / 12) * eta + 76055 * eta * eta / 1728 -
          127825 * eta * eta * eta / 1296;
  c.b6 = -6848.0Q / 21;
  c.e0sq = (qd)p->e0 * (qd)p->e0;
  return c;
}

/* Psi(f)/(2 pi) in cycles (App. A with phi_p and phi_D carried by the
 * response instead of the phase, see response()):
 *   f t_c - phi_c/(2 pi) - 1/8 + (3/128)(pi Mc f)^{-5/3} [sum_k alpha_k v^k + Psi_e/Psi_N] / (2 pi)
 * v = (pi M f)^{1/3}; (3/128)(pi Mc f)^{-5/3} = 3 / (128 eta v^5).
 * alpha_k: non-spinning TaylorF2 coefficients of the literature the paper
 * cites (parity unpinned beyond the Newtonian term: the paper does not print
 * them).  Psi_e: leading-order eccentric correction -(2355/1462) e0^2
 * (f0/f)^{19/9} times the Newtonian term, e0 defined at the GW frequency
 * f0 = 10 mHz (Sec. II.A, Table I).                                        */
static qd phase_cycles_q(const or_pq *c, double f, double phic) {
  const qd pi = OR_PI_Q;
  qd F = (qd)f;
  qd v = cbrtq(pi * c->m * F);
  qd v2 = v * v, v5 = v2 * v2 * v;
  qd newt = 3 / (128 * c->eta * v5);
  qd s = 1;
  if (g_pn_order >= 2) {
    qd lv = logq(v);
    qd v3 = v2 * v, v4 = v2 * v2, v6 = v3 * v3;
    qd a5 = c->c5 * (1 + 3 * (lv + logq(sqrtq(6.0Q))));
    qd a6 = c->a6c + c->b6 * (lv + logq(4.0Q));
    s += c->a2 * v2 + c->a3 * v3 + c->a4 * v4 + a5 * v5 + a6 * v6;
  }
  qd ecc = 0;
  if (c->e0sq != 0) ecc = -(2355.0Q / 1462) * c->e0sq * powq((qd)OR_F0_ECC / F, 19.0Q / 9);
  return F * c->tc - (qd)phic / (2 * pi) - 0.125Q + newt * (s + ecc) / (2 * pi);
}

/* dPsi/df (radians per Hz): each term of the series differentiated by hand.
 * A term newt * v^k scales as f^{(k-5)/3}; the alpha_5 logarithm and the
 * alpha_6 logarithm contribute their own derivative; Psi_e scales as
 * f^{-34/9}. */
static long double dpsi_df(const or_intr *p, long double f) {
  const long double pi = OR_PI_L;
  long double eta = eta_of(p);
  long double mc = (long double)p->mc * (long double)OR_MSUN_S;
  long double m = mc * powl(eta, -0.6L);
  long double v = cbrtl(pi * m * f);
  long double newt = 3.0L / (128.0L * powl(pi * mc * f, 5.0L / 3.0L));
  long double d = -5.0L / 3.0L; /* k = 0 */
  if (g_pn_order >= 2) {
    long double v2 = v * v, v3 = v2 * v, v4 = v3 * v, v5 = v4 * v, v6 = v5 * v;
    long double a2 = 3715.0L / 756.0L + 55.0L * eta / 9.0L;
    long double a3 = -16.0L * pi;
    long double a4 = 15293365.0L / 508032.0L + 27145.0L * eta / 504.0L +
                     3085.0L * eta * eta / 72.0L;
    long double c5 = pi * (38645.0L / 756.0L - 65.0L * eta / 9.0L);
    long double a6c = 11583231236531.0L / 4694215680.0L - 640.0L * pi * pi / 3.0L -
                      6848.0L * OR_EULER_L / 21.0L +
                      (-15737765635.0L / 3048192.0L + 2255.0L * pi * pi / 12.0L) * eta +
                      76055.0L * eta * eta / 1728.0L - 127825.0L * eta * eta * eta / 1296.0L;
    long double b6 = -6848.0L / 21.0L;
    d += (-3.0L / 3.0L) * a2 * v2 + (-2.0L / 3.0L) * a3 * v3 + (-1.0L / 3.0L) * a4 * v4;
    d += c5 * v5;                                          /* d/df of the log */
    d += v6 * (a6c + b6 * logl(4.0L * v) + b6) / 3.0L;    /* f^{1/3} term    */
  }
  long double e0 = (long double)p->e0;
  long double ecc = -(2355.0L / 1462.0L) * e0 * e0 *
                    powl((long double)OR_F0_ECC / f, 19.0L / 9.0L);
  d += (-34.0L / 9.0L) * ecc;
  return 2.0L * pi * (long double)p->tc + newt * d / f;
}

/* Sec. IV: t_f = (1/2pi) dPsi/df. */
static double tf_of(const or_intr *p, double f) {
  return (double)(dpsi_df(p, (long double)f) / (2.0L * OR_PI_L));
}

/* ---- Sec. IV: detector orbit ------------------------------------------ */
/* Analytic rigid-triangle orbit, first order in the orbital eccentricity
 * e = L / (2 sqrt(3) R) (the paper states its result does not depend on the
 * orbit model).  Guiding centre on a circle of radius R = 1 AU, alpha =
 * 2 pi t / yr, spacecraft phases beta_i = 2 pi i / 3 (i = 0, 1, 2).
 * Positions in light-seconds.                                             */
static void orbit(double t, double pos[3][3]) {
  const double R = OR_AU_M / OR_C;
  const double L = OR_ARM_M / OR_C;
  const double e = L / (2.0 * sqrt(3.0) * R);
  const double a = 2.0 * OR_PI * t / OR_YEAR_S;
  for (int i = 0; i < 3; ++i) {
    double b = 2.0 * OR_PI * (double)i / 3.0;
    pos[i][0] = R * cos(a) + 0.5 * e * R * (cos(2.0 * a - b) - 3.0 * cos(b));
    pos[i][1] = R * sin(a) + 0.5 * e * R * (sin(2.0 * a - b) - 3.0 * sin(b));
    pos[i][2] = -sqrt(3.0) * e * R * cos(a - b);
  }
}

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Sky direction, propagation vector and polarisation basis for colatitude
 * theta and longitude phi (Sec. II.A: theta = pi/2 - beta, phi = lambda). */
static void sky_frame(double theta, double phi, double k[3], double u[3], double v[3]) {
  double st = sin(theta), ct = cos(theta), sp = sin(phi), cp = cos(phi);
  k[0] = -st * cp; k[1] = -st * sp; k[2] = -ct; /* k = -Omega (propagation) */
  u[0] = ct * cp;  u[1] = ct * sp;  u[2] = -st;
  v[0] = sp;       v[1] = -cp;      v[2] = 0.0;
}

/* Single-link Fourier-domain transfer at zeroth order of the Marsat-Baker
 * expansion (Sec. IV, Eq. "freDres" with N = 0): the time-domain link signal
 *   y_{r<-s}(t) = n.H.n / (2 (1 - k.n)) [h(t - L - k.p_s) - h(t - k.p_r)]
 * with positions frozen at t_f transforms (FT kernel exp(-2 pi i f t)) into
 *   -i pi f L sinc(pi f L (1 - k.n)) n.H.n exp(-i pi f (L + k.(p_s + p_r))) h(f).
 * Returned for unit polarisation amplitude; xp/xx carry n.e+.n and n.ex.n.  */
static void link_transfer(const double pos[3][3], int r, int s, const double k[3],
                          const double u[3], const double v[3], double f,
                          double complex *yp, double complex *yx) {
  const double L = OR_ARM_M / OR_C;
  double d[3], n[3];
  for (int c = 0; c < 3; ++c) d[c] = pos[r][c] - pos[s][c];
  double nrm = sqrt(dot3(d, d));
  for (int c = 0; c < 3; ++c) n[c] = d[c] / nrm;
  double kn = dot3(k, n);
  double x = OR_PI * f * L * (1.0 - kn);
  double sinc = (x == 0.0) ? 1.0 : sin(x) / x;
  double ps[3];
  for (int c = 0; c < 3; ++c) ps[c] = pos[s][c] + pos[r][c];
  double ph = -OR_PI * f * (L + dot3(k, ps));
  double complex g = -I * OR_PI * f * L * sinc * cexp(I * ph);
  double un = dot3(u, n), vn = dot3(v, n);
  *yp = g * (un * un - vn * vn);
  *yx = g * (2.0 * un * vn);
}

/* Rigid constellation (reading of Sec. IV's orbit, on which the paper says its
 * result does not depend): spacecraft 1 follows the analytic orbit and
 * spacecraft 2, 3 sit at p1 + L n, with the arm directions n of the analytic
 * orbit, so every arm has the nominal length L used for the delays. */
static void rigid_positions(double t, double pos[3][3]) {
  const double L = OR_ARM_M / OR_C;
  double orb[3][3];
  orbit(t, orb);
  for (int c = 0; c < 3; ++c) pos[0][c] = orb[0][c];
  for (int i = 1; i < 3; ++i) {
    double d[3];
    for (int c = 0; c < 3; ++c) d[c] = orb[i][c] - orb[0][c];
    double nrm = sqrt(dot3(d, d));
    for (int c = 0; c < 3; ++c) pos[i][c] = orb[0][c] + L * d[c] / nrm;
  }
}

/* Numerical orbit (Sec. IV allows one, interpolated with Chebyshev
 * polynomials): n_seg segments of length dt from t0, each given by the
 * spacecraft positions [3][3] at the 10 Chebyshev points
 * t = t0 + dt (seg + (1 + s_k)/2), s_k = cos(pi (k + 1/2) / 10); positions
 * between them are the degree-9 interpolant, evaluated here in barycentric
 * Lagrange form in long double.  With no table the rigid analytic
 * constellation above is used.                                              */
static struct {
  int nseg;
  double t0, dt;
  double *nodes;   /* [nseg][3][3][10] */
} g_orb = {0, 0.0, 0.0, NULL};

int or_set_orbit(double t0, double dt, int nseg, const double *nodes) {
  free(g_orb.nodes);
  g_orb.nodes = NULL;
  g_orb.nseg = 0;
  if (nseg <= 0) return 0;
  if (!(dt > 0.0) || !nodes) return -1;
  g_orb.nodes = malloc(sizeof(double) * 90 * (size_t)nseg);
  if (!g_orb.nodes) return -1;
  memcpy(g_orb.nodes, nodes, sizeof(double) * 90 * (size_t)nseg);
  g_orb.nseg = nseg;
  g_orb.t0 = t0;
  g_orb.dt = dt;
  return 0;
}

static void table_positions(double t, double pos[3][3]) {
  int seg = (int)floor((t - g_orb.t0) / g_orb.dt);
  if (seg < 0) seg = 0;
  if (seg > g_orb.nseg - 1) seg = g_orb.nseg - 1;
  const long double x = 2.0L * ((long double)t - g_orb.t0 - (long double)g_orb.dt * seg) / g_orb.dt - 1.0L;
  long double w[10], sk[10], den = 0.0L;
  int hit = -1;
  for (int k = 0; k < 10; ++k) {
    const long double th = (long double)OR_PI * (k + 0.5L) / 10.0L;
    sk[k] = cosl(th);
    /* barycentric weights of the first-kind Chebyshev points */
    w[k] = ((k & 1) ? -1.0L : 1.0L) * sinl(th);
    if (x == sk[k]) hit = k;
  }
  const double *nd = g_orb.nodes + 90 * (size_t)seg;
  for (int i = 0; i < 3; ++i)
    for (int c = 0; c < 3; ++c) {
      const double *v = nd + 30 * i + 10 * c;
      if (hit >= 0) { pos[i][c] = v[hit]; continue; }
      long double num = 0.0L;
      den = 0.0L;
      for (int k = 0; k < 10; ++k) {
        const long double q = w[k] / (x - sk[k]);
        num += q * v[k];
        den += q;
      }
      pos[i][c] = (double)(num / den);
    }
}

static void positions(double t, double pos[3][3]) {
  if (g_orb.nseg > 0) table_positions(t, pos);
  else rigid_positions(t, pos);
}

/* Spacecraft positions used by the response (the table when one is set). */
void or_positions(const double *t, int64_t n, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    double pos[3][3];
    positions(t[i], pos);
    memcpy(out + 9 * i, pos, sizeof(pos));
  }
}

/* First-generation Michelson combination at spacecraft a (index a) with equal
 * static delays L (reading of the TDI-X combination the paper cites); with
 * b = a + 1, c = a + 2 (mod 3):
 *   M_a = (1 - z^2) [ (y_{a<-c} + z y_{c<-a}) - (y_{a<-b} + z y_{b<-a}) ],
 *   z = exp(-2 pi i f L);  X = M_0, Y = M_1, Z = M_2 (cyclic relabelling).
 * Output: transfer for the + and x polarisation, constellation at t.      */
static void michelson(const or_intr *p, double f, double t, int a, double complex T[2]) {
  const double L = OR_ARM_M / OR_C;
  double pos[3][3], k[3], u[3], v[3];
  positions(t, pos);
  sky_frame(p->theta, p->phi, k, u, v);
  const int b = (a + 1) % 3, c = (a + 2) % 3;
  double complex yacp, yacx, ycap, ycax, yabp, yabx, ybap, ybax;
  link_transfer(pos, a, c, k, u, v, f, &yacp, &yacx);
  link_transfer(pos, c, a, k, u, v, f, &ycap, &ycax);
  link_transfer(pos, a, b, k, u, v, f, &yabp, &yabx);
  link_transfer(pos, b, a, k, u, v, f, &ybap, &ybax);
  double complex z = cexp(-2.0 * I * OR_PI * f * L);
  double complex pre = 1.0 - z * z;
  T[0] = pre * ((yacp + z * ycap) - (yabp + z * ybap));
  T[1] = pre * ((yacx + z * ycax) - (yabx + z * ybax));
}

static void response(const or_intr *p, double f, double t, double complex T[2]) {
  michelson(p, f, t, 0, T);
}

/* Channel codes: 0 X, 1 Y, 2 Z, and the noise-orthogonal combinations of the
 * equal-arm Michelson channels (Sec. II.A names them; the paper itself uses X
 * only): 3 A = (Z - X)/sqrt 2, 4 E = (X - 2Y + Z)/sqrt 6, 5 T = (X + Y + Z)/sqrt 3. */
static int channel_ok(int ch) { return ch >= 0 && ch <= 5; }
static void response_ch(const or_intr *p, double f, double t, int ch, double complex T[2]) {
  if (ch <= 2) {
    michelson(p, f, t, ch, T);
    return;
  }
  double complex X[2], Y[2], Z[2];
  michelson(p, f, t, 0, X);
  michelson(p, f, t, 1, Y);
  michelson(p, f, t, 2, Z);
  for (int q = 0; q < 2; ++q) {
    if (ch == 3) T[q] = (Z[q] - X[q]) / sqrt(2.0);
    else if (ch == 4) T[q] = (X[q] - 2.0 * Y[q] + Z[q]) / sqrt(6.0);
    else T[q] = (X[q] + Y[q] + Z[q]) / sqrt(3.0);
  }
}

/* Four real-amplitude basis templates at one frequency (Eq. "response"):
 *   A^1 = T+ g,  A^2 = -Tx g,  A^3 = -i T+ g,  A^4 = i Tx g,
 * g = f^{-7/6} exp(-i Psi(f)) with phi_c = 0.  With the App. B amplitudes
 * a_1..a_4 this reproduces h_X = T+ h+ + Tx hx for h+ = (1+cos^2 i)/2 ...,
 * hx = -i cos(i) ... rotated by psi (reading of the App. B conventions).    */
static void basis_at(const or_intr *p, const or_pq *pq, double f, int ch, double complex A[4]) {
  qd cyc = phase_cycles_q(pq, f, 0.0);
  double fr = (double)(cyc - floorq(cyc));
  double ph = 2.0 * OR_PI * fr;
  double complex g = pow(f, -7.0 / 6.0) * cexp(-I * ph);
  double complex T[2];
  response_ch(p, f, tf_of(p, f), ch, T);
  A[0] = T[0] * g;
  A[1] = -T[1] * g;
  A[2] = -I * T[0] * g;
  A[3] = I * T[1] * g;
}

/* ---- support and partitions (Sec. II.B) -------------------------------- */
/* Frequency at which t_f reaches `t`, by bisection on [fa, fb] (t_f is
 * increasing in f over the search ranges).                                 */
static double invert_tf(const or_intr *p, double t, double fa, double fb) {
  for (int it = 0; it < 200; ++it) {
    double fm = 0.5 * (fa + fb);
    if (fm <= fa || fm >= fb) break;
    if (tf_of(p, fm) < t) fa = fm; else fb = fm;
  }
  return fb;
}

/* Lowest and highest instantaneous frequency during [0, T_obs], clipped to
 * the data band [f_first, f_last].  Returns 0 when the support is empty.   */
static int support(const or_intr *p, double T_obs, double f_first, double f_last,
                   double *flo, double *fhi) {
  double t_first = tf_of(p, f_first), t_last = tf_of(p, f_last);
  if (t_last < 0.0 || t_first > T_obs) return 0;
  *flo = (t_first >= 0.0) ? f_first : invert_tf(p, 0.0, f_first, f_last);
  *fhi = (t_last <= T_obs) ? f_last : invert_tf(p, T_obs, f_first, f_last);
  return *flo <= *fhi;
}

/* ---- small dense linear algebra ---------------------------------------- */
/* Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix. */
static void jacobi4(const double Ain[4][4], double lam[4], double V[4][4]) {
  double A[4][4];
  memcpy(A, Ain, sizeof(A));
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < 4; ++i)
      for (int j = i + 1; j < 4; ++j) off += A[i][j] * A[i][j];
    if (off == 0.0) break;
    for (int pq = 0; pq < 6; ++pq) {
      static const int P[6] = {0, 0, 0, 1, 1, 2}, Q[6] = {1, 2, 3, 2, 3, 3};
      int p = P[pq], q = Q[pq];
      if (A[p][q] == 0.0) continue;
      double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
      double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
      double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int r = 0; r < 4; ++r) { /* A <- A J */
        double arp = A[r][p], arq = A[r][q];
        A[r][p] = c * arp - s * arq;
        A[r][q] = s * arp + c * arq;
      }
      for (int r = 0; r < 4; ++r) { /* A <- J^T A */
        double apr = A[p][r], aqr = A[q][r];
        A[p][r] = c * apr - s * aqr;
        A[q][r] = s * apr + c * aqr;
      }
      for (int r = 0; r < 4; ++r) {
        double vrp = V[r][p], vrq = V[r][q];
        V[r][p] = c * vrp - s * vrq;
        V[r][q] = s * vrp + c * vrq;
      }
    }
  }
  for (int i = 0; i < 4; ++i) lam[i] = A[i][i];
}

/* Solve M a = N by Gaussian elimination with partial pivoting. */
static void lu_solve4(const double Min[4][4], const double N[4], double a[4]) {
  double M[4][5];
  for (int i = 0; i < 4; ++i) {
    for (int j = 0; j < 4; ++j) M[i][j] = Min[i][j];
    M[i][4] = N[i];
  }
  for (int c = 0; c < 4; ++c) {
    int piv = c;
    for (int r = c + 1; r < 4; ++r)
      if (fabs(M[r][c]) > fabs(M[piv][c])) piv = r;
    if (piv != c)
      for (int j = 0; j < 5; ++j) { double t = M[c][j]; M[c][j] = M[piv][j]; M[piv][j] = t; }
    for (int r = c + 1; r < 4; ++r) {
      double m = M[r][c] / M[c][c];
      for (int j = c; j < 5; ++j) M[r][j] -= m * M[c][j];
    }
  }
  for (int r = 3; r >= 0; --r) {
    double s = M[r][4];
    for (int j = r + 1; j < 4; ++j) s -= M[r][j] * a[j];
    a[r] = s / M[r][r];
  }
}

/* Relative eigenvalue cut below which M is treated as singular and the
 * pseudo-inverse is used (the paper is silent on singular M; with N in the
 * range of M the pseudo-inverse still gives max_a Lambda).                 */
#define OR_RANK_CUT 1e-12

/* Eq. "coherent_F_stat": F = 1/2 N^T M^{-1} N, with a = M^{-1} N.
 * Returns F; writes lambda_max/lambda_min to *cond (inf when singular).   */
static double fstat_solve(const double M[4][4], const double N[4], double *cond, double a_out[4]) {
  double lam[4], V[4][4];
  jacobi4(M, lam, V);
  double lmax = lam[0], lmin = lam[0];
  for (int i = 1; i < 4; ++i) {
    if (lam[i] > lmax) lmax = lam[i];
    if (lam[i] < lmin) lmin = lam[i];
  }
  for (int r = 0; r < 4; ++r) a_out[r] = 0.0;
  if (!(lmax > 0.0)) { *cond = INFINITY; return 0.0; }
  *cond = (lmin > 0.0) ? lmax / lmin : INFINITY;
  if (lmin > OR_RANK_CUT * lmax) {
    lu_solve4(M, N, a_out);           /* the maximiser a = M^{-1} N (Eq. aandMN3) */
    return 0.5 * (N[0] * a_out[0] + N[1] * a_out[1] + N[2] * a_out[2] + N[3] * a_out[3]);
  }
  /* pseudo-inverse: the minimum-norm maximiser */
  double F = 0.0;
  for (int i = 0; i < 4; ++i) {
    if (lam[i] <= OR_RANK_CUT * lmax) continue;
    double proj = V[0][i] * N[0] + V[1][i] * N[1] + V[2][i] * N[2] + V[3][i] * N[3];
    F += 0.5 * proj * proj / lam[i];
    for (int r = 0; r < 4; ++r) a_out[r] += V[r][i] * proj / lam[i];
  }
  return F;
}

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } or_acc;
static void acc_add(or_acc *a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
  else a->c += (x - t) + a->s;
  a->s = t;
}
static double acc_val(const or_acc *a) { return a->s + a->c; }

/* ---- exported entry points -------------------------------------------- */

/* Phase Psi(f)/(2 pi) in cycles at each frequency, as hi + lo doubles. */
int or_phase(const double *theta6, double phic, const double *f, int64_t n, double *hi, double *lo) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    or_pq pq = phase_consts(&p);
    qd c = phase_cycles_q(&pq, f[i], phic);
    hi[i] = (double)c;
    lo[i] = (double)(c - (qd)hi[i]);
  }
  return 0;
}

/* SPA time t_f at each frequency. */
int or_tf(const double *theta6, const double *f, int64_t n, double *out) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p)) return -1;
  for (int64_t i = 0; i < n; ++i) out[i] = tf_of(&p, f[i]);
  return 0;
}

/* Spacecraft positions [n][3][3] (light-seconds) at times t: the analytic
 * orbit (rigid = 0) or the rigid constellation used by the response (1). */
void or_orbit(const double *t, int64_t n, int rigid, double *out) {
  for (int64_t i = 0; i < n; ++i) {
    double pos[3][3];
    if (rigid) rigid_positions(t[i], pos); else orbit(t[i], pos);
    memcpy(out + 9 * i, pos, sizeof(pos));
  }
}

/* TDI-X transfer T+, Tx (complex, interleaved re/im) at frequencies f and
 * explicit orbit times t (not necessarily t_f). Output [n][2][2].          */
int or_response(const double *theta6, const double *f, const double *t, int64_t n, double *out) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double complex T[2];
    response(&p, f[i], t[i], T);
    out[4 * i + 0] = creal(T[0]); out[4 * i + 1] = cimag(T[0]);
    out[4 * i + 2] = creal(T[1]); out[4 * i + 3] = cimag(T[1]);
  }
  return 0;
}

/* Transfer of channel `ch` (codes above) at frequencies f and orbit times t:
 * output [n][2][2].                                                         */
int or_response_ch(const double *theta6, const double *f, const double *t, int64_t n, int ch,
                   double *out) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p) || !channel_ok(ch)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    double complex T[2];
    response_ch(&p, f[i], t[i], ch, T);
    out[4 * i + 0] = creal(T[0]); out[4 * i + 1] = cimag(T[0]);
    out[4 * i + 2] = creal(T[1]); out[4 * i + 3] = cimag(T[1]);
  }
  return 0;
}

/* Single-link transfer y_{r<-s} for unit + and x amplitude at frequency f and
 * explicit spacecraft positions pos[3][3] (for the time-domain pin).        */
void or_link(const double *pos9, int r, int s, double theta, double phi, double f, double *out4) {
  double pos[3][3], k[3], u[3], v[3];
  memcpy(pos, pos9, sizeof(pos));
  sky_frame(theta, phi, k, u, v);
  double complex yp, yx;
  link_transfer(pos, r, s, k, u, v, f, &yp, &yx);
  out4[0] = creal(yp); out4[1] = cimag(yp); out4[2] = creal(yx); out4[3] = cimag(yx);
}

/* Basis templates A^1..A^4 of channel ch at frequencies f: output [n][4][2]. */
int or_basis(const double *theta6, const double *f, int64_t n, int ch, double *out) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p) || !channel_ok(ch)) return -1;
  or_pq pq = phase_consts(&p);
  for (int64_t i = 0; i < n; ++i) {
    double complex A[4];
    basis_at(&p, &pq, f[i], ch, A);
    for (int b = 0; b < 4; ++b) {
      out[8 * i + 2 * b] = creal(A[b]);
      out[8 * i + 2 * b + 1] = cimag(A[b]);
    }
  }
  return 0;
}

/* Support [f_lo, f_hi] on the band; returns 1 if non-empty, 0 if empty. */
int or_support(const double *theta6, double T_obs, double f_first, double f_last, double *out2) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p)) return -1;
  double lo = 0.0, hi = 0.0;
  int ok = support(&p, T_obs, f_first, f_last, &lo, &hi);
  out2[0] = lo; out2[1] = hi;
  return ok;
}

/* Injected signal sum_i a_i A^i on the grid f_j = (k_lo + j) df, set to zero
 * outside the template support during [0, T_obs].  Output [nbins][2].     */
int or_signal(const double *theta6, const double *amp4, double df, int64_t k_lo, int64_t nbins,
              double T_obs, int ch, double *out) {
  or_intr p = unpack(theta6);
  if (!params_ok(&p) || nbins <= 0 || !channel_ok(ch)) return -1;
  memset(out, 0, sizeof(double) * 2 * (size_t)nbins);
  double f_first = (double)k_lo * df, f_last = (double)(k_lo + nbins - 1) * df;
  double flo, fhi;
  if (!support(&p, T_obs, f_first, f_last, &flo, &fhi)) return 0;
  or_pq pq = phase_consts(&p);
#pragma omp parallel for schedule(static)
  for (int64_t j = 0; j < nbins; ++j) {
    double f = (double)(k_lo + j) * df;
    if (f < flo || f > fhi) continue;
    double complex A[4];
    basis_at(&p, &pq, f, ch, A);
    double complex h = amp4[0] * A[0] + amp4[1] * A[1] + amp4[2] * A[2] + amp4[3] * A[3];
    out[2 * j] = creal(h);
    out[2 * j + 1] = cimag(h);
  }
  return 0;
}

/* Semi-coherent F-statistic (Eq. "semi-cohF").
 *   data  [nch][nbins][2]  s_c(f_j), f_j = (k_lo + j) df, channel c = chans[c]
 *         (chans NULL, nch 1: TDI-X)
 *   psd   [nch][nbins]     one-sided S_c(f_j) > 0 (channel noises independent:
 *         N and M are sums over the channels)
 *   params[n][6], np[n] (or np == NULL and np_uniform)
 *   F_hat [n]; F_part [n][part_stride] (or NULL); cond [n][part_stride] (or NULL)
 * Partition edges e_l = f_lo + (f_hi - f_lo) l / Np; bin j is in partition l
 * when e_l <= f_j < e_{l+1} (last partition closed).  Empty partitions give
 * F_l = 0; an empty support gives F_hat = -inf.  Returns 0, or -1 on bad
 * arguments.                                                               */
int or_fstat(const double *data, const double *psd, int64_t nbins, int64_t k_lo, double df,
             double T_obs, const double *params, int64_t n, const int32_t *np, int32_t np_uniform,
             double *F_hat, double *F_part, int64_t part_stride, double *cond_out,
             double *amps_out, const int32_t *chans, int32_t nch) {
  if (nbins <= 0 || n < 0 || !(df > 0.0) || nch < 1) return -1;
  for (int c = 0; c < nch; ++c)
    if (!channel_ok(chans ? chans[c] : 0)) return -1;
  for (int64_t i = 0; i < n; ++i) {
    or_intr p = unpack(params + 6 * i);
    int npi = np ? np[i] : np_uniform;
    if (!params_ok(&p) || npi < 1) return -1;
    if (F_part && npi > part_stride) return -1;
  }
  for (int64_t j = 0; j < nbins * nch; ++j)
    if (!(psd[j] > 0.0)) return -1;
  const double f_first = (double)k_lo * df, f_last = (double)(k_lo + nbins - 1) * df;
  int err = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t i = 0; i < n; ++i) {
    or_intr p = unpack(params + 6 * i);
    int Np = np ? np[i] : np_uniform;
    double flo, fhi;
    double *fp = F_part ? F_part + i * part_stride : NULL;
    double *cp = cond_out ? cond_out + i * part_stride : NULL;
    double *ap = amps_out ? amps_out + 4 * i * part_stride : NULL;
    if (!support(&p, T_obs, f_first, f_last, &flo, &fhi)) {
      F_hat[i] = -INFINITY;
      for (int l = 0; l < Np; ++l) {
        if (fp) fp[l] = 0.0;
        if (cp) cp[l] = INFINITY;
        if (ap) for (int r = 0; r < 4; ++r) ap[4 * l + r] = 0.0;
      }
      continue;
    }
    or_acc *accN = calloc((size_t)Np * 4, sizeof(or_acc));
    or_acc *accM = calloc((size_t)Np * 16, sizeof(or_acc));
    double *edge = malloc(sizeof(double) * (size_t)(Np + 1));
    if (!accN || !accM || !edge) { err = 1; free(accN); free(accM); free(edge); continue; }
    double span = fhi - flo;
    for (int l = 0; l <= Np; ++l) edge[l] = flo + (span * (double)l) / (double)Np;
    or_pq pq = phase_consts(&p);
    int l = 0;
    for (int64_t j = 0; j < nbins; ++j) {
      double f = (double)(k_lo + j) * df;
      if (f < flo || f > fhi) continue;
      while (l < Np - 1 && f >= edge[l + 1]) ++l;
      for (int c = 0; c < nch; ++c) {   /* channels with independent noise: sums add */
        double complex A[4];
        basis_at(&p, &pq, f, chans ? chans[c] : 0, A);
        const int64_t jc = (int64_t)c * nbins + j;
        double complex s = data[2 * jc] + I * data[2 * jc + 1];
        for (int a = 0; a < 4; ++a) {
          acc_add(&accN[4 * l + a], creal(s * conj(A[a])) / psd[jc]);
          for (int b = 0; b < 4; ++b)
            acc_add(&accM[16 * l + 4 * a + b], creal(A[a] * conj(A[b])) / psd[jc]);
        }
      }
    }
    double sum = 0.0;
    for (int q = 0; q < Np; ++q) {
      double N[4], M[4][4], cnd;
      for (int a = 0; a < 4; ++a) {
        N[a] = 4.0 * df * acc_val(&accN[4 * q + a]);
        for (int b = 0; b < 4; ++b) M[a][b] = 4.0 * df * acc_val(&accM[16 * q + 4 * a + b]);
      }
      double a[4];
      double Fl = fstat_solve(M, N, &cnd, a);
      if (fp) fp[q] = Fl;
      if (cp) cp[q] = cnd;
      if (ap) for (int r = 0; r < 4; ++r) ap[4 * q + r] = a[r];
      sum += Fl;
    }
    F_hat[i] = sum / (double)Np;
    free(accN); free(accM); free(edge);
  }
  return err ? -2 : 0;
}
