"""Seeded synthetic inputs shared by the tests and the benchmark.

This module holds the input recipe only: the frequency grids, the TDI-X noise
model the data are drawn from, Gaussian noise, random parameter draws, and
the scaling of an injected signal to a target SNR.  It contains none of the
F-statistic arithmetic: the injected waveform itself is produced by whatever
callable the caller passes in.

Workloads (2.5 yr of one TDI-X channel, LISA-like noise, Sec. II.A and
Sec. V of Fu, Wang & Mohanty 2024) are stand-ins for the paper's data
realisations, which are not public.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

YEAR_S = 31557600.0          # Julian year [s]
C_SI = 299792458.0
AU_M = 1.495978707e11        # astronomical unit [m]
ARM_M = 2.5e9                # nominal arm length [m]
S_ACC_ASD = 3e-15            # acceleration noise [m s^-2 Hz^-1/2]
S_OMS_ASD = 15e-12           # optical metrology noise [m Hz^-1/2]
F_KNEE_ACC = 0.4e-3          # acceleration-noise reddening knee [Hz]


@dataclasses.dataclass(frozen=True)
class Grid:
    """rFFT grid f_j = (k_lo + j) df, j < nbins, of an observation T_obs."""
    T_obs: float
    df: float
    k_lo: int
    nbins: int

    def freqs(self) -> np.ndarray:
        return (self.k_lo + np.arange(self.nbins, dtype=np.int64)).astype(np.float64) * self.df

    @property
    def f_first(self) -> float:
        return float(self.k_lo) * self.df

    @property
    def f_last(self) -> float:
        return float(self.k_lo + self.nbins - 1) * self.df


def grid_small() -> Grid:
    """T = 2^20 s, df = 2^-20 Hz, bins 20972..41943 (20-40 mHz): 20,972 bins."""
    return Grid(T_obs=2.0 ** 20, df=2.0 ** -20, k_lo=20972, nbins=41943 - 20972 + 1)


def grid_paper() -> Grid:
    """T = 7.89e7 s (2.5 yr), df = 1/T, bins 789,000..7,890,000 (10-100 mHz)."""
    T = 7.89e7
    return Grid(T_obs=T, df=1.0 / T, k_lo=789000, nbins=7890000 - 789000 + 1)


def grid_custom(T_obs: float, f_lo: float, f_hi: float) -> Grid:
    df = 1.0 / T_obs
    k_lo = int(math.ceil(f_lo * T_obs))
    k_hi = int(math.floor(f_hi * T_obs))
    return Grid(T_obs=T_obs, df=df, k_lo=k_lo, nbins=k_hi - k_lo + 1)


def psd_tdix(f: np.ndarray) -> np.ndarray:
    """One-sided PSD of first-generation TDI-X (fractional frequency units)
    for equal arms: 16 sin^2(x) [S_oms + (3 + cos 2x) S_acc], x = 2 pi f L/c,
    with the acceleration and optical-metrology noise levels above."""
    f = np.asarray(f, dtype=np.float64)
    x = 2.0 * np.pi * f * ARM_M / C_SI
    s_acc = S_ACC_ASD ** 2 * (1.0 + (F_KNEE_ACC / f) ** 2) / (2.0 * np.pi * f * C_SI) ** 2
    s_oms = S_OMS_ASD ** 2 * (2.0 * np.pi * f / C_SI) ** 2
    return 16.0 * np.sin(x) ** 2 * (s_oms + (3.0 + np.cos(2.0 * x)) * s_acc)


def psd_channel(f: np.ndarray, channel: str) -> np.ndarray:
    """One-sided PSD of a first-generation equal-arm TDI channel with the noise
    levels above: X, Y, Z as psd_tdix; A = E = S_X - S_XY and T = S_X + 2 S_XY
    with the Michelson cross spectrum S_XY = -8 sin^2(x) cos(x) (S_oms + 4 S_acc)
    (the channels A, E, T have independent noise)."""
    f = np.asarray(f, dtype=np.float64)
    if channel in ("X", "Y", "Z"):
        return psd_tdix(f)
    x = 2.0 * np.pi * f * ARM_M / C_SI
    s_acc = S_ACC_ASD ** 2 * (1.0 + (F_KNEE_ACC / f) ** 2) / (2.0 * np.pi * f * C_SI) ** 2
    s_oms = S_OMS_ASD ** 2 * (2.0 * np.pi * f / C_SI) ** 2
    s2, c1 = np.sin(x) ** 2, np.cos(x)
    if channel in ("A", "E"):
        return 8.0 * s2 * ((2.0 + c1) * s_oms + 2.0 * (3.0 + 2.0 * c1 + np.cos(2.0 * x)) * s_acc)
    if channel == "T":
        return 16.0 * s2 * ((1.0 - c1) * s_oms + 2.0 * (1.0 - c1) ** 2 * s_acc)
    raise ValueError(f"unknown channel {channel!r}")


def noise(psd: np.ndarray, df: float, seed: int) -> np.ndarray:
    """Stationary Gaussian noise on the grid: n_j = sqrt(S_j / (4 df)) (x + i y),
    x, y ~ N(0, 1), so that Var <n, h> = <h, h>."""
    rng = np.random.default_rng(seed)
    sig = np.sqrt(psd / (4.0 * df))
    out = np.empty(psd.shape, dtype=np.complex128)
    out.real = rng.standard_normal(psd.shape) * sig
    out.imag = rng.standard_normal(psd.shape) * sig
    return out


def snr_scale(signal: np.ndarray, psd: np.ndarray, df: float, snr: float) -> float:
    """Factor that brings a signal to optimal SNR `snr` (rho^2 = 4 df sum |h|^2/S)."""
    rho2 = 4.0 * df * float(np.sum(np.abs(signal) ** 2 / psd))
    return snr / math.sqrt(rho2)


# ---- parameter boxes -------------------------------------------------------
# theta6 = (t_c [s], Mc [Msun], delta_mu, theta [rad], phi [rad], e0)

def uniform_box(box: np.ndarray, n: int, seed: int) -> np.ndarray:
    """n points uniform in the hypercube box[6][2] (PSO search space, Sec. III.A)."""
    box = np.asarray(box, dtype=np.float64)
    rng = np.random.default_rng(seed)
    u = rng.random((n, 6))
    return box[:, 0] + u * (box[:, 1] - box[:, 0])


def random_amplitudes(seed: int) -> np.ndarray:
    """Four extrinsic amplitudes a_i drawn isotropically (N(0,1) each)."""
    return np.random.default_rng(seed).standard_normal(4)


def random_sky(seed: int):
    rng = np.random.default_rng(seed)
    return math.acos(rng.uniform(-1.0, 1.0)), rng.uniform(0.0, 2.0 * math.pi)


# Small workload: injection Mc = 30 Msun, e0 = 0.01, delta_mu = 0.1585 (Table I),
# t_c chosen so that the template's instantaneous GW frequency at T/2 is 30 mHz.
SMALL_TC = 26314556.013170715  # [s]
SMALL_MC = 30.0
SMALL_E0 = 0.01
SMALL_DMU = 0.1585
SMALL_SNR = 12.0
SMALL_SEEDS = dict(noise=1001, inj=1002, pts=1003)


def small_injection_params(seed: int = SMALL_SEEDS["inj"]) -> np.ndarray:
    th, ph = random_sky(seed)
    return np.array([SMALL_TC, SMALL_MC, SMALL_DMU, th, ph, SMALL_E0])


def small_eval_points(inj: np.ndarray, n: int = 256, seed: int = SMALL_SEEDS["pts"]) -> np.ndarray:
    """Injection plus n uniform points: Mc +-0.1 %, t_c +-1 day, full sky,
    e0 in [0, 0.1], delta_mu fixed."""
    rng = np.random.default_rng(seed)
    pts = np.empty((n, 6))
    pts[:, 0] = inj[0] + rng.uniform(-86400.0, 86400.0, n)
    pts[:, 1] = inj[1] * (1.0 + rng.uniform(-1e-3, 1e-3, n))
    pts[:, 2] = inj[2]
    pts[:, 3] = np.arccos(rng.uniform(-1.0, 1.0, n))
    pts[:, 4] = rng.uniform(0.0, 2.0 * math.pi, n)
    pts[:, 5] = rng.uniform(0.0, 0.1, n)
    return np.vstack([inj[None, :], pts])


def small_box(inj: np.ndarray) -> np.ndarray:
    return np.array([[inj[0] - 86400.0, inj[0] + 86400.0],
                     [inj[1] * (1 - 1e-3), inj[1] * (1 + 1e-3)],
                     [inj[2], inj[2]],
                     [0.0, math.pi], [0.0, 2.0 * math.pi], [0.0, 0.1]])


# Paper-scale workload: t_c range and sky from Table I, Mc in [10, 50] Msun,
# e0 in [0, 0.1], 2.5 yr of data at 1/T resolution over 10-100 mHz.
PAPER_BOX = np.array([[3.3 * YEAR_S, 3.8 * YEAR_S], [10.0, 50.0], [0.0, 0.9],
                      [0.0, math.pi], [0.0, 2.0 * math.pi], [0.0, 0.1]])
PAPER_SEEDS = dict(noise=2001, inj=2002, pts=2003)


def paper_injection_params(seed: int = PAPER_SEEDS["inj"]):
    rng = np.random.default_rng(seed)
    th = math.acos(rng.uniform(-1.0, 1.0))
    ph = rng.uniform(0.0, 2.0 * math.pi)
    p = np.array([3.5 * YEAR_S, rng.uniform(10.0, 50.0), rng.uniform(0.0, 0.9), th, ph,
                  rng.uniform(0.0, 0.1)])
    snr = rng.uniform(11.0, 14.0)
    return p, snr


def make_data(grid: Grid, seed_noise: int, signal: np.ndarray | None = None,
              snr: float | None = None, dtype=np.complex128):
    """Noise (+ optional signal scaled to `snr`) and the PSD on `grid`."""
    psd = psd_tdix(grid.freqs())
    d = noise(psd, grid.df, seed_noise)
    if signal is not None:
        d = d + snr_scale(signal, psd, grid.df, snr) * signal
    return d.astype(dtype), psd


def chebyshev_node_times(t0: float, dt: float, nseg: int) -> np.ndarray:
    """Times [nseg, 10] of an orbit table's nodes: t0 + dt (seg + (1 + s_k)/2),
    s_k = cos(pi (k + 1/2) / 10)."""
    s = np.cos(np.pi * (np.arange(10) + 0.5) / 10)
    return t0 + dt * (np.arange(nseg)[:, None] + 0.5 * (1.0 + s[None, :]))


def kepler_positions(t: np.ndarray) -> np.ndarray:
    """Positions [n, 3, 3] (spacecraft, xyz; seconds of light travel) of three
    spacecraft on exact heliocentric Kepler orbits that keep a triangle of
    side ~ARM_M tilted by ~60 degrees to the ecliptic (semi-major axis 1 AU,
    eccentricity ~ L / (2 sqrt 3 AU), orbital planes inclined by ~L / (2 AU)).
    Unlike a first-order analytic orbit the arms flex by about one per cent
    over a year: a stand-in for a numerically integrated orbit."""
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    R, alpha = AU_M / C_SI, ARM_M / (2.0 * AU_M)
    incl = math.atan(alpha / (1.0 + alpha / math.sqrt(3.0)))
    ecc = math.sqrt(1.0 + 2.0 * alpha / math.sqrt(3.0) + 4.0 * alpha * alpha / 3.0) - 1.0
    out = np.empty((t.size, 3, 3))
    for k in range(3):
        sig = 2.0 * np.pi * k / 3.0
        M = 2.0 * np.pi * t / YEAR_S - sig
        E = M.copy()
        for _ in range(8):                       # Kepler's equation, Newton
            E -= (E - ecc * np.sin(E) - M) / (1.0 - ecc * np.cos(E))
        xp = R * (np.cos(E) - ecc)               # in the orbital plane, perihelion on +x
        yp = R * math.sqrt(1.0 - ecc * ecc) * np.sin(E)
        x, z = xp * math.cos(incl), xp * math.sin(incl)
        out[:, k, 0] = x * math.cos(sig) - yp * math.sin(sig)
        out[:, k, 1] = x * math.sin(sig) + yp * math.cos(sig)
        out[:, k, 2] = z
    return out


def kepler_orbit_nodes(t0: float, dt: float, nseg: int) -> np.ndarray:
    """Orbit table [nseg, 3, 3, 10] (segment, spacecraft, xyz, node) of
    kepler_positions at the Chebyshev node times."""
    ts = chebyshev_node_times(t0, dt, nseg)
    pos = kepler_positions(ts.ravel()).reshape(nseg, 10, 3, 3)
    return np.ascontiguousarray(pos.transpose(0, 2, 3, 1))
