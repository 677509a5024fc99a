"""The tiny workload of the high-precision checks: 64 bins of the small
workload's grid around 30 mHz, noise plus the small workload's injection at
SNR 12 (over these bins), and five parameter points: the injection, a point
100 s away, a random point of the small workload's box, and two points whose
supports are cut by the observation window inside the band (the template's
instantaneous frequency enters the band after t = 0, resp. leaves it before
T_obs), so that the support edges fall between bins.  Inputs only: the
points are placed with the oracle's t_f, nothing here evaluates the statistic.
"""
import numpy as np

from oracle import oracle as O
from paper_2407_10797_amd import synth as S

NBINS = 64
NPARTS = (1, 8, 32, 64)   # 64, 8, 2 and 1 bins per partition


def tiny():
    g0 = S.grid_small()
    k_lo = int(round(0.03 / g0.df)) - NBINS // 2
    g = S.Grid(T_obs=g0.T_obs, df=g0.df, k_lo=k_lo, nbins=NBINS)
    inj = S.small_injection_params()
    sig = O.signal(inj, S.random_amplitudes(S.SMALL_SEEDS["inj"]), g.df, g.k_lo, g.nbins, g.T_obs)
    data, psd = S.make_data(g, 7007, sig, S.SMALL_SNR)
    f = g.freqs()
    # t_c shifts that put t_f = 0 midway between bins 20 and 21 (support
    # starts inside the band) and t_f = T_obs midway between bins 40 and 41
    p_lo = inj.copy()
    p_lo[0] -= O.tf(inj, f[20] + 0.5 * g.df)[0]
    p_hi = inj.copy()
    p_hi[0] += g.T_obs - O.tf(inj, f[40] + 0.5 * g.df)[0]
    pts = np.vstack([inj, inj + np.array([100.0, 0, 0, 0, 0, 0]),
                     S.uniform_box(S.small_box(inj), 1, 7008), p_lo, p_hi])
    pts[2, 0] = inj[0] + 300.0     # keep the random point's support on the band
    return dict(g=g, data=data, psd=psd, pts=pts)
