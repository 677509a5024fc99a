"""High-precision (mpmath, 50 significant digits) end-to-end F-statistic for
tiny inputs: the arbiter of the FP64 parity bars.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``; the product library never
imports it.  It shares no code with ``fstat_oracle.c`` or with the HIP path;
every step is written again from the paper's definitions, at 50 digits,
taking the same readings of the points the paper leaves open:

* template phase Psi(f)/(2 pi) of App. A (restricted post-Newtonian phase with
  the non-spinning TaylorF2 coefficients through v^6 and the leading-order
  eccentric term), phi_c = 0;
* SPA time t_f = (1/2 pi) dPsi/df (Sec. IV) by numerical differentiation of
  the phase at working precision (not a hand-derived series);
* first-order analytic orbit with rigid arms of length L (Sec. IV allows any
  orbit model), the zeroth-order frequency-domain single-link response at t_f
  (Sec. IV, Eq. freDres with N = 0) and the first-generation TDI-X
  combination;
* basis templates A^1 = T+ g, A^2 = -Tx g, A^3 = -i T+ g, A^4 = i Tx g with
  g = f^{-7/6} exp(-i Psi) (Sec. II.A, Eq. response; App. B);
* <a, b> = 4 df Re sum a conj(b) / S (Sec. II.A), N^i = <s|A^i>,
  M^ij = <A^i|A^j>, F = 1/2 N^T M^{-1} N (Eq. coherent_F_stat), solved by LU
  at 50 digits, or by the pseudo-inverse with eigenvalues below 1e-12 of the
  largest dropped when M is singular;
* support [f_lo, f_hi] = the lowest and highest instantaneous frequency during
  [0, T_obs] (Sec. II.B) by root finding on t_f, clipped to the band; Np
  equal-width partitions, bin j in partition l iff e_l <= f_j < e_{l+1}, the
  last partition closed; F_hat = mean of the F_l (Eq. semi-cohF).

Inputs are the same doubles the other implementations take (data, PSD,
parameters); everything after them is evaluated at 50 digits, so the result
is the exact value of the definitions on those inputs to far below double
rounding.  Intended for <= 64 bins and a handful of parameter points.
"""
from __future__ import annotations

import mpmath as mp

# constants: the same double values the library and the C oracle take (the
# comparison is about arithmetic, not about the constants' last digits)
_MSUN_S = 4.925490947641267e-6      # G Msun / c^3 [s]
_YEAR_S = 31557600.0                # Julian year [s]
_C = 299792458.0
_AU_M = 1.495978707e11
_ARM_M = 2.5e9
_F0_ECC = 0.01                      # GW frequency at which e0 is defined [Hz]
RANK_CUT = mp.mpf("1e-12")
DPS = 50


class _Ctx:
    """Per-particle constants at working precision."""

    def __init__(self, theta6):
        tc, mc, dmu, th, ph, e0 = (mp.mpf(float(x)) for x in theta6)
        self.tc = tc
        self.mc = mc * mp.mpf(_MSUN_S)
        self.eta = (1 - dmu * dmu) / 4
        self.m = self.mc * self.eta ** mp.mpf(-0.6)
        eta = self.eta
        pi = mp.pi
        self.a2 = mp.mpf(3715) / 756 + 55 * eta / 9
        self.a3 = -16 * pi
        self.a4 = mp.mpf(15293365) / 508032 + 27145 * eta / 504 + 3085 * eta ** 2 / 72
        self.c5 = pi * (mp.mpf(38645) / 756 - 65 * eta / 9)
        self.a6c = (mp.mpf(11583231236531) / 4694215680 - 640 * pi ** 2 / 3
                    - 6848 * mp.euler / 21
                    + (mp.mpf(-15737765635) / 3048192 + 2255 * pi ** 2 / 12) * eta
                    + mp.mpf(76055) / 1728 * eta ** 2 - mp.mpf(127825) / 1296 * eta ** 3)
        self.e0sq = e0 * e0
        st, ct, sp, cp = mp.sin(th), mp.cos(th), mp.sin(ph), mp.cos(ph)
        self.k = (-st * cp, -st * sp, -ct)          # propagation direction -Omega
        self.u = (ct * cp, ct * sp, -st)             # polarisation basis
        self.v = (sp, -cp, mp.mpf(0))

    def cycles(self, f):
        """Psi(f) / (2 pi) in cycles (App. A), phi_c = 0."""
        pi = mp.pi
        v = mp.cbrt(pi * self.m * f)
        lv = mp.log(v)
        s = (1 + self.a2 * v ** 2 + self.a3 * v ** 3 + self.a4 * v ** 4
             + self.c5 * (1 + 3 * (lv + mp.log(mp.sqrt(6)))) * v ** 5
             + (self.a6c - mp.mpf(6848) / 21 * (lv + mp.log(4))) * v ** 6)
        ecc = -(mp.mpf(2355) / 1462) * self.e0sq * (mp.mpf(_F0_ECC) / f) ** (mp.mpf(19) / 9)
        newt = 3 / (128 * self.eta * v ** 5)
        return f * self.tc - mp.mpf(1) / 8 + newt * (s + ecc) / (2 * pi)

    def tf(self, f):
        """t_f = d(Psi / 2 pi)/df (Sec. IV)."""
        return mp.diff(self.cycles, f)


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def _positions(t):
    """Rigid constellation on the first-order analytic orbit [light-seconds]:
    spacecraft 1 on the orbit, 2 and 3 at p1 + L n with the orbit's arm
    directions n."""
    R = mp.mpf(_AU_M) / _C
    L = mp.mpf(_ARM_M) / _C
    e = L / (2 * mp.sqrt(3) * R)
    a = 2 * mp.pi * t / _YEAR_S
    orb = []
    for i in range(3):
        b = 2 * mp.pi * i / 3
        orb.append((R * mp.cos(a) + e * R / 2 * (mp.cos(2 * a - b) - 3 * mp.cos(b)),
                    R * mp.sin(a) + e * R / 2 * (mp.sin(2 * a - b) - 3 * mp.sin(b)),
                    -mp.sqrt(3) * e * R * mp.cos(a - b)))
    pos = [orb[0]]
    for i in (1, 2):
        d = [orb[i][c] - orb[0][c] for c in range(3)]
        nrm = mp.sqrt(_dot(d, d))
        pos.append(tuple(orb[0][c] + L * d[c] / nrm for c in range(3)))
    return pos


def _link(ctx, pos, r, s, f):
    """Zeroth-order FD single-link transfer y_{r<-s} for unit + and x."""
    L = mp.mpf(_ARM_M) / _C
    d = [pos[r][c] - pos[s][c] for c in range(3)]
    nrm = mp.sqrt(_dot(d, d))
    n = [x / nrm for x in d]
    kn = _dot(ctx.k, n)
    x = mp.pi * f * L * (1 - kn)
    sinc = mp.sin(x) / x if x != 0 else mp.mpf(1)
    ps = [pos[s][c] + pos[r][c] for c in range(3)]
    g = -1j * mp.pi * f * L * sinc * mp.expj(-mp.pi * f * (L + _dot(ctx.k, ps)))
    un, vn = _dot(ctx.u, n), _dot(ctx.v, n)
    return g * (un * un - vn * vn), g * (2 * un * vn)


def _tdi_x(ctx, f, t):
    L = mp.mpf(_ARM_M) / _C
    pos = _positions(t)
    z = mp.expj(-2 * mp.pi * f * L)
    y02, y20, y01, y10 = (_link(ctx, pos, 0, 2, f), _link(ctx, pos, 2, 0, f),
                          _link(ctx, pos, 0, 1, f), _link(ctx, pos, 1, 0, f))
    pre = 1 - z * z
    return tuple(pre * ((y02[q] + z * y20[q]) - (y01[q] + z * y10[q])) for q in range(2))


def basis(theta6, f):
    """The four basis templates at frequency f (a double): list of 4 mpc."""
    with mp.workdps(DPS):
        ctx = _Ctx(theta6)
        return _basis(ctx, mp.mpf(float(f)))


def _basis(ctx, f):
    cyc = ctx.cycles(f)
    g = f ** (mp.mpf(-7) / 6) * mp.expj(-2 * mp.pi * cyc)
    tp, tx = _tdi_x(ctx, f, ctx.tf(f))
    return [tp * g, -tx * g, -1j * tp * g, 1j * tx * g]


def support(theta6, T_obs, f_first, f_last):
    """(f_lo, f_hi) as mpf, or None when empty (Sec. II.B)."""
    with mp.workdps(DPS):
        ctx = _Ctx(theta6)
        return _support(ctx, mp.mpf(float(T_obs)), mp.mpf(float(f_first)), mp.mpf(float(f_last)))


def _support(ctx, T, fa, fb):
    ta, tb = ctx.tf(fa), ctx.tf(fb)
    if tb < 0 or ta > T:
        return None

    def root(t):
        return mp.findroot(lambda x: ctx.tf(x) - t, (fa, fb), solver="anderson")

    lo = fa if ta >= 0 else root(0)
    hi = fb if tb <= T else root(T)
    return (lo, hi) if lo <= hi else None


def _solve(N, M):
    """F = 1/2 N.a with M a = N (LU), or the pseudo-inverse when the smallest
    eigenvalue is below RANK_CUT of the largest.  Returns (F, cond)."""
    Mm = mp.matrix(M)
    lam, V = mp.eigsy(Mm)
    lam = [lam[i] for i in range(4)]
    lmax, lmin = max(lam), min(lam)
    if not lmax > 0:
        return mp.mpf(0), mp.inf
    cond = lmax / lmin if lmin > 0 else mp.inf
    if lmin > RANK_CUT * lmax:
        a = mp.lu_solve(Mm, mp.matrix(N))
        return sum(N[i] * a[i] for i in range(4)) / 2, cond
    F = mp.mpf(0)
    for i in range(4):
        if lam[i] <= RANK_CUT * lmax:
            continue
        proj = sum(V[r, i] * N[r] for r in range(4))
        F += proj * proj / lam[i] / 2
    return F, cond


def fstat(data, psd, k_lo, df, T_obs, theta6, npart):
    """Semi-coherent F of one parameter point on the grid f_j = (k_lo + j) df.

    data: complex [nbins] (doubles), psd: [nbins].  Returns
    (F_hat, [F_l], [cond(M_l)]) as Python floats (rounded from 50 digits);
    F_hat = -inf for an empty support."""
    nbins = len(data)
    with mp.workdps(DPS):
        ctx = _Ctx(theta6)
        dfm = mp.mpf(float(df))
        freqs = [mp.mpf(int(k_lo) + j) * dfm for j in range(nbins)]
        sup = _support(ctx, mp.mpf(float(T_obs)), freqs[0], freqs[-1])
        if sup is None:
            return float("-inf"), [0.0] * npart, [float("inf")] * npart
        lo, hi = sup
        edges = [lo + (hi - lo) * l / npart for l in range(npart + 1)]
        Ns = [[mp.mpf(0)] * 4 for _ in range(npart)]
        Ms = [[[mp.mpf(0)] * 4 for _ in range(4)] for _ in range(npart)]
        for j, f in enumerate(freqs):
            if f < lo or f > hi:
                continue
            l = 0
            while l < npart - 1 and f >= edges[l + 1]:
                l += 1
            A = _basis(ctx, f)
            s = mp.mpc(float(data[j].real), float(data[j].imag))
            S = mp.mpf(float(psd[j]))
            for a in range(4):
                Ns[l][a] += mp.re(s * mp.conj(A[a])) / S
                for b in range(4):
                    Ms[l][a][b] += mp.re(A[a] * mp.conj(A[b])) / S
        Fl, cl = [], []
        for l in range(npart):
            N = [4 * dfm * x for x in Ns[l]]
            M = [[4 * dfm * x for x in row] for row in Ms[l]]
            F, c = _solve(N, M)
            Fl.append(F)
            cl.append(c)
        Fhat = sum(Fl) / npart
        return float(Fhat), [float(x) for x in Fl], [float(c) for c in cl]
