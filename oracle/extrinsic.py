"""Extrinsic parameters from the F-statistic amplitudes (App. B), plain numpy.

TEST INFRASTRUCTURE ONLY: the reference the library's extrinsic recovery is
checked against.  Forward map (D_L, iota, psi, phi_c) -> a_1..a_4 and its
inverse, App. B.  The inverse is read with two-argument arctangents: psi =
(1/2) atan2(A+ a4 - Ax a1, -(Ax a2 + A+ a3)) in (-pi/2, pi/2], c = sgn(sin 2 psi)
(+1 when sin 2 psi = 0), phi_c = atan2(c (A+ a4 - Ax a1), -c (Ax a3 + A+ a2));
(psi + pi/2, phi_c + pi) gives the same a, and the forward map of the
recovered values reproduces a.  At iota = 0 or pi (one of the two circular
parts of a vanishes) both arctangent arguments are 0/0 and only 2 psi +- phi_c
is defined; there psi = 0 is taken and phi_c = atan2(-a3, a1).  The case is
recognised when the smaller circular part is below 64 ulp of the larger.  D_L comes out in the units the a_i carry
(1/D_L times the template amplitude constant).
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
    A = Ap + np.sqrt(np.maximum(Ap * Ap - Ax * Ax, 0.0))
    D = 2.0 / A
    iota = np.arccos(np.clip(-Ax / A, -1.0, 1.0))
    num = Ap * a4 - Ax * a1
    psi = 0.5 * np.arctan2(num, -(Ax * a2 + Ap * a3))
    c = np.where(np.sin(2.0 * psi) < 0.0, -1.0, 1.0)
    phic = np.arctan2(c * num, -c * (Ax * a3 + Ap * a2))
    flat = np.minimum(r1, r2) <= 64.0 * np.finfo(np.float64).eps * np.maximum(r1, r2)
    psi = np.where(flat, 0.0, psi)
    phic = np.where(flat, np.arctan2(-a3, a1), phic)
    return np.stack([D, iota, psi, phic], axis=-1)
