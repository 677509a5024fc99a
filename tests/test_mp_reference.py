"""The oracle against a 50-digit evaluation of the paper's definitions
(``oracle/mp_reference.py``) on the tiny workload: 64 bins, partitions of 64,
8, 2 and 1 bins (well conditioned, cond(M) up to ~1e8, and the rank-2
one-bin case solved by the pseudo-inverse), and supports cut by the
observation window inside the band.

Measured: the oracle's per-partition error is at most 0.15 eps cond(M_l)
relative (eps = 2^-52), and 2e-14 relative on singular partitions; the
bound asserted is 1 eps cond(M_l) + 64 eps.
"""
import numpy as np
import pytest

from oracle import mp_reference as R
from oracle import oracle as O
from tests.tiny_workload import NPARTS, tiny

EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def tw():
    return tiny()


@pytest.fixture(scope="module")
def truth(tw):
    out = {}
    for npart in NPARTS:
        rows = [R.fstat(tw["data"], tw["psd"], tw["g"].k_lo, tw["g"].df, tw["g"].T_obs, p, npart)
                for p in tw["pts"]]
        out[npart] = (np.array([r[0] for r in rows]), np.array([r[1] for r in rows]),
                      np.array([r[2] for r in rows]))
    return out


def test_support_edges_by_root_finding(tw):
    """Sec. II.B: the support is the range of instantaneous frequencies during
    [0, T_obs]; the 50-digit root of t_f(f) = 0 (resp. T_obs), with t_f the
    numerical derivative of the 50-digit phase, equals the oracle's edge to
    double rounding, and the edges fall inside the band where placed."""
    g = tw["g"]
    f = g.freqs()
    for i, p in enumerate(tw["pts"]):
        so = O.support(p, g.T_obs, g.f_first, g.f_last)
        sm = R.support(p, g.T_obs, g.f_first, g.f_last)
        assert so is not None and sm is not None
        assert abs(so[0] - float(sm[0])) <= 4e-16 * so[0]
        assert abs(so[1] - float(sm[1])) <= 4e-16 * so[1]
    lo = R.support(tw["pts"][3], g.T_obs, g.f_first, g.f_last)[0]
    hi = R.support(tw["pts"][4], g.T_obs, g.f_first, g.f_last)[1]
    assert f[20] < lo < f[21]
    assert f[40] < hi < f[41]


@pytest.mark.parametrize("npart", NPARTS)
def test_oracle_against_50_digits(tw, truth, npart):
    g = tw["g"]
    Fh, Fp, cond = O.fstat(tw["data"], tw["psd"], g.k_lo, g.df, g.T_obs, tw["pts"], [npart],
                           want_cond=True)
    Th, Tp, Tc = truth[npart]
    scale = np.maximum(np.abs(Tp), 1.0)
    err = np.abs(Fp[:, :npart] - Tp) / scale
    fin = Tc <= 1e12            # beyond: singular (empty or one-bin) partitions
    assert np.all(err[fin] <= EPS * Tc[fin] + 64 * EPS), np.max(err[fin] / (EPS * Tc[fin]))
    assert np.all(err[~fin] <= 1e-12)
    # the two supports cut inside the band leave bins out of every partition
    np.testing.assert_allclose(Fh, Th, rtol=1e-9, atol=0)
    if npart == 64:
        assert np.all(~fin)        # one bin: M has rank 2, the pseudo-inverse applies
    if npart == 32:
        assert Tc[fin].max() > 1e7     # near-singular two-bin partitions
