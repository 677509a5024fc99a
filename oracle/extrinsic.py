"""Extrinsic parameters from the F-statistic amplitudes (App. B), plain numpy.

TEST INFRASTRUCTURE ONLY: the reference the library's extrinsic recovery is
checked against.  Forward map (D_L, iota, psi, phi_c) -> a_1..a_4 and its
inverse by Eq. extrinPara, with the arctangents read as two-argument ones:
psi = (1/2) atan2(A+ a4 - Ax a1, -(Ax a2 + A+ a3)) in (-pi/2, pi/2],
c = sgn(sin 2 psi) (+1 when sin 2 psi = 0), phi_c = atan2(c (A+ a4 - Ax a1),
-c (Ax a3 + A+ a2)), which lands in (0, pi]; (psi + pi/2, phi_c + pi) gives
the same a.

The three arctangent arguments are 2 r1 r2 sin 2psi sin phi_c, 2 r1 r2 cos 2psi
sin phi_c and 2 r1 r2 sin 2psi cos phi_c (r1, r2 the moduli of the circular
parts (a1 + a4) + i (a2 - a3) and (a1 - a4) - i (a2 + a3)), so the printed
ratios are 0/0 on sin 2psi sin phi_c = 0 and lose about eps A+^2 / |argument|
of accuracy near it (enough to flip c).  Where the arguments of either
arctangent are below 1e-6 A+^2 together, the phases of the circular parts,
phi_c - 2 psi and phi_c + 2 psi, give the same representative instead.  At iota = 0 or pi one
circular part vanishes (its modulus below 64 ulp of the other's) and only the
other's phase is defined: psi = 0 and phi_c is that phase.  All-zero a gives
(inf, nan, nan, nan).  D_L comes out in the units the a_i carry (1/D_L times
the template amplitude constant); physical() converts with the App. A
constant given the chirp mass.
"""
from __future__ import annotations

import numpy as np


def forward(D, iota, psi, phic):
    """a_1..a_4 of App. B; arrays broadcast, returns [..., 4]."""
    D, iota, psi, phic = np.broadcast_arrays(*(np.asarray(x, dtype=np.float64) for x in (D, iota, psi, phic)))
    c2, s2 = np.cos(2 * psi), np.sin(2 * psi)
    ci = np.cos(iota)
    p = 0.5 * (1.0 + ci * ci)
    cp, sp = np.cos(phic), np.sin(phic)
    a1 = (c2 * p * cp - s2 * ci * sp) / D
    a2 = -(s2 * p * cp + c2 * ci * sp) / D
    a3 = -(c2 * p * sp + s2 * ci * cp) / D
    a4 = (s2 * p * sp - c2 * ci * cp) / D
    return np.stack([a1, a2, a3, a4], axis=-1)


def inverse(a):
    """(D_L, iota, psi, phi_c) from a [..., 4] (App. B, Eq. extrinPara)."""
    a = np.asarray(a, dtype=np.float64)
    a1, a2, a3, a4 = a[..., 0], a[..., 1], a[..., 2], a[..., 3]
    r1 = np.sqrt((a1 + a4) ** 2 + (a2 - a3) ** 2)
    r2 = np.sqrt((a1 - a4) ** 2 + (a2 + a3) ** 2)
    Ap, Ax = r1 + r2, r1 - r2
    # A+^2 - Ax^2 factored: the plain difference cancels near iota = 0, pi
    A = Ap + np.sqrt(np.maximum((Ap - Ax) * (Ap + Ax), 0.0))
    with np.errstate(divide="ignore", invalid="ignore"):
        D = 2.0 / A
        iota = np.arccos(np.clip(-Ax / A, -1.0, 1.0))
    num = Ap * a4 - Ax * a1
    den = -(Ax * a2 + Ap * a3)
    psi = 0.5 * np.arctan2(num, den)
    c = np.where(np.sin(2.0 * psi) < 0.0, -1.0, 1.0)
    den2 = -(Ax * a3 + Ap * a2)
    phic = np.arctan2(c * num, c * den2)
    # (near-)0/0 ratios: phases of the circular parts
    eps64 = 64.0 * np.finfo(np.float64).eps
    th1 = np.arctan2(a2 - a3, a1 + a4)          # phi_c - 2 psi
    th2 = np.arctan2(-(a2 + a3), a1 - a4)       # phi_c + 2 psi
    sing = np.minimum(np.hypot(num, den), np.hypot(num, den2)) <= 1e-6 * Ap * Ap
    ph_s = np.mod(0.5 * (th1 + th2), np.pi)
    ph_s = np.where(ph_s == 0.0, np.pi, ph_s)
    d = np.mod(th2 - ph_s + np.pi, 2.0 * np.pi) - np.pi
    d = np.where(d == -np.pi, np.pi, d)
    psi = np.where(sing, 0.5 * d, psi)
    phic = np.where(sing, ph_s, phic)
    flat = np.minimum(r1, r2) <= eps64 * np.maximum(r1, r2)
    psi = np.where(flat, 0.0, psi)
    phic = np.where(flat, np.where(r1 < r2, th2, th1), phic)
    zero = A == 0.0
    iota = np.where(zero, np.nan, iota)
    psi = np.where(zero, np.nan, psi)
    phic = np.where(zero, np.nan, phic)
    return np.stack([D, iota, psi, phic], axis=-1)


G_MSUN_OVER_C3 = 4.925490947641267e-6    # [s]
C_LIGHT = 299792458.0                     # [m/s]


def amplitude_constant(mc_msun):
    """App. A: A D_L = -sqrt(5/24) Mc^{5/6} / pi^{2/3} (G = c = 1, seconds)."""
    return -np.sqrt(5.0 / 24.0) * (np.asarray(mc_msun) * G_MSUN_OVER_C3) ** (5.0 / 6.0) / np.pi ** (2.0 / 3.0)


def physical(out, mc_msun):
    """The inverse's (D, iota, psi, phi_c) for amplitudes of the unit-amplitude
    basis turned into D_L [m] and the phase of the App. A waveform: the
    basis's a are A D_L times those of App. B, so D_L = |A D_L| D (seconds,
    times c) and the negative sign of A shifts phi_c by pi (kept in (-pi, pi])."""
    out = np.array(out, dtype=np.float64, copy=True)
    K = np.abs(amplitude_constant(mc_msun))
    out[..., 0] = out[..., 0] * K * C_LIGHT
    ph = out[..., 3]
    out[..., 3] = np.where(ph > 0.0, ph - np.pi, ph + np.pi)
    return out
