"""Python access to the plain FP64 CPU oracle (``fstat_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of the benchmark.  The product library never imports it.

Every function here is a thin ctypes wrapper around the C file, except
``inner``/``fstat_from_templates``, which restate the paper's definitions in
numpy for the pins (Sec. II.A, Eqs. "inner_product" and "coherent_F_stat").
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fstat_oracle.c")
_LIB = os.path.join(_HERE, "libfstat_oracle.so")

_dp = ctypes.POINTER(ctypes.c_double)
_i32p = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain IEEE double, no contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
               "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB + ".tmp", "-lquadmath", "-lm"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_LIB_NATIVE = os.path.join(_HERE, "libfstat_oracle_native.so")


def build_native() -> str:
    """The same oracle tuned for the host it runs on (-O3 -march=native; still
    plain IEEE double, no contraction, no fast math), for timing the CPU
    baseline only: built where it runs, since the host may differ from the one
    that built the default copy."""
    cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared", "-std=gnu11",
           "-ffp-contract=off", "-fno-fast-math", _SRC, "-o", _LIB_NATIVE + ".tmp", "-lquadmath",
           "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB_NATIVE + ".tmp", _LIB_NATIVE)
    return _LIB_NATIVE


_lib = None


def use_native() -> None:
    """Route the wrappers below through the host-tuned copy (build_native)."""
    global _lib
    _lib = _load(build_native())


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _load(_LIB)
    return _lib


def _load(path):
    if True:
        L = ctypes.CDLL(path)
        L.or_set_pn_order.argtypes = [ctypes.c_int]
        L.or_phase.argtypes = [_dp, ctypes.c_double, _dp, ctypes.c_int64, _dp, _dp]
        L.or_tf.argtypes = [_dp, _dp, ctypes.c_int64, _dp]
        L.or_orbit.argtypes = [_dp, ctypes.c_int64, ctypes.c_int, _dp]
        L.or_response.argtypes = [_dp, _dp, _dp, ctypes.c_int64, _dp]
        L.or_link.argtypes = [_dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, _dp]
        L.or_response_ch.argtypes = [_dp, _dp, _dp, ctypes.c_int64, ctypes.c_int, _dp]
        L.or_set_orbit.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int, _dp]
        L.or_positions.argtypes = [_dp, ctypes.c_int64, _dp]
        L.or_basis.argtypes = [_dp, _dp, ctypes.c_int64, ctypes.c_int, _dp]
        L.or_support.argtypes = [_dp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _dp]
        L.or_signal.argtypes = [_dp, _dp, ctypes.c_double, ctypes.c_int64, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_int, _dp]
        L.or_fstat.argtypes = [_dp, _dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double,
                               ctypes.c_double, _dp, ctypes.c_int64, _i32p, ctypes.c_int32,
                               _dp, _dp, ctypes.c_int64, _dp, _dp, _i32p, ctypes.c_int32]
    return L


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's particle loop (libgomp, process-wide)."""
    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def set_pn_order(order: int) -> None:
    lib().or_set_pn_order(int(order))


def phase_cycles(theta6, f, phic=0.0):
    """Psi(f)/(2 pi) as (hi, lo) doubles (App. A)."""
    t, tp = _d(theta6)
    f, fp = _d(np.atleast_1d(f))
    hi = np.empty_like(f); lo = np.empty_like(f)
    if lib().or_phase(tp, float(phic), fp, f.size, hi.ctypes.data_as(_dp), lo.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return hi, lo


def tf(theta6, f):
    """SPA time t_f = (1/2pi) dPsi/df (Sec. IV)."""
    t, tp = _d(theta6)
    f, fp = _d(np.atleast_1d(f))
    out = np.empty_like(f)
    if lib().or_tf(tp, fp, f.size, out.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return out


def orbit(t, rigid=False):
    """Spacecraft positions [n, 3, 3]: analytic orbit, or the rigid
    constellation (arms of length L along the orbit's arm directions)."""
    t, tp = _d(np.atleast_1d(t))
    out = np.empty((t.size, 3, 3))
    lib().or_orbit(tp, t.size, int(bool(rigid)), out.ctypes.data_as(_dp))
    return out


def set_orbit(t0=0.0, dt=1.0, nodes=None):
    """Use a numerical orbit: nodes [n_seg, 3, 3, 10] positions [s] at the
    Chebyshev points of each segment of length dt from t0 (see the C
    source); nodes=None goes back to the analytic constellation."""
    if nodes is None:
        lib().or_set_orbit(0.0, 1.0, 0, None)
        return
    nd, npp = _d(nodes)
    if lib().or_set_orbit(float(t0), float(dt), nd.shape[0], npp):
        raise ValueError("bad orbit table")


def chebyshev_times(t0, dt, n_seg):
    """Times [n_seg, 10] of an orbit table's nodes."""
    s = np.cos(np.pi * (np.arange(10) + 0.5) / 10)
    return t0 + dt * (np.arange(n_seg)[:, None] + 0.5 * (1.0 + s[None, :]))


def positions(t):
    """Spacecraft positions [n, 3, 3] the response uses (the table if set)."""
    t, tp = _d(np.atleast_1d(t))
    out = np.empty((t.size, 3, 3))
    lib().or_positions(tp, t.size, out.ctypes.data_as(_dp))
    return out


def response(theta6, f, t):
    """TDI-X transfer (T+, Tx) at frequency f with the orbit frozen at time t."""
    th, tp = _d(theta6)
    f, fp = _d(np.atleast_1d(f))
    t, tt = _d(np.broadcast_to(np.atleast_1d(t), f.shape))
    out = np.empty((f.size, 4))
    if lib().or_response(tp, fp, tt, f.size, out.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return out[:, 0] + 1j * out[:, 1], out[:, 2] + 1j * out[:, 3]


CHANNELS = {"X": 0, "Y": 1, "Z": 2, "A": 3, "E": 4, "T": 5}


def _ch(channel) -> int:
    return CHANNELS[channel] if isinstance(channel, str) else int(channel)


def response_ch(theta6, f, t, channel):
    """Transfer (T+, Tx) of a TDI channel ('X', 'Y', 'Z', 'A', 'E', 'T')."""
    th, tp = _d(theta6)
    f, fp = _d(np.atleast_1d(f))
    t, tt = _d(np.broadcast_to(np.atleast_1d(t), f.shape))
    out = np.empty((f.size, 4))
    if lib().or_response_ch(tp, fp, tt, f.size, _ch(channel), out.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return out[:, 0] + 1j * out[:, 1], out[:, 2] + 1j * out[:, 3]


def link(pos, r, s, theta, phi, f):
    p, pp = _d(pos)
    out = np.empty(4)
    lib().or_link(pp, int(r), int(s), float(theta), float(phi), float(f), out.ctypes.data_as(_dp))
    return out[0] + 1j * out[1], out[2] + 1j * out[3]


def basis(theta6, f, channel="X"):
    """The four basis templates A^i(f) of a channel: complex array [n, 4]."""
    th, tp = _d(theta6)
    f, fp = _d(np.atleast_1d(f))
    out = np.empty((f.size, 4, 2))
    if lib().or_basis(tp, fp, f.size, _ch(channel), out.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return out[..., 0] + 1j * out[..., 1]


def support(theta6, T_obs, f_first, f_last):
    th, tp = _d(theta6)
    out = np.empty(2)
    ok = lib().or_support(tp, float(T_obs), float(f_first), float(f_last), out.ctypes.data_as(_dp))
    if ok < 0:
        raise ValueError("bad parameters")
    return (float(out[0]), float(out[1])) if ok else None


def signal(theta6, amp4, df, k_lo, nbins, T_obs, channel="X"):
    """sum_i a_i A^i of a channel on the grid, zero outside the support:
    complex [nbins]."""
    th, tp = _d(theta6)
    a, ap = _d(amp4)
    out = np.empty((int(nbins), 2))
    if lib().or_signal(tp, ap, float(df), int(k_lo), int(nbins), float(T_obs), _ch(channel),
                       out.ctypes.data_as(_dp)):
        raise ValueError("bad parameters")
    return out[:, 0] + 1j * out[:, 1]


def fstat(data, psd, k_lo, df, T_obs, params, np_parts, part_stride=None, want_cond=False,
          want_amps=False, channels=None):
    """Semi-coherent F (Eq. "semi-cohF").  Returns (F_hat, F_part[, cond][, amps]):
    amps [n, stride, 4] are the maximising amplitudes a = M^{-1} N of each
    partition (Eq. "aandMN3"), minimum-norm when M is singular.  With
    `channels` (e.g. "AET"), data and psd are [channels, nbins] and N, M are
    summed over the channels (independent noise); without, one TDI-X channel."""
    chans = None
    if channels is not None:
        chans = np.ascontiguousarray([_ch(c) for c in channels], dtype=np.int32)
    nch = 1 if chans is None else len(chans)
    data = np.ascontiguousarray(data, dtype=np.complex128).reshape(nch, -1)
    dv = data.view(np.float64)
    psd, pp = _d(np.asarray(psd, dtype=np.float64).reshape(nch, -1))
    params = np.ascontiguousarray(np.atleast_2d(params), dtype=np.float64)
    n = params.shape[0]
    npa = np.ascontiguousarray(np.broadcast_to(np.asarray(np_parts, dtype=np.int32), (n,)))
    stride = int(part_stride or (npa.max() if n else 1))
    Fh = np.empty(n)
    Fp = np.zeros((n, stride))
    cond = np.zeros((n, stride)) if want_cond else None
    amps = np.zeros((n, stride, 4)) if want_amps else None
    rc = lib().or_fstat(dv.ctypes.data_as(_dp), pp, data.shape[1], int(k_lo), float(df),
                        float(T_obs), params.ctypes.data_as(_dp), n, npa.ctypes.data_as(_i32p), 0,
                        Fh.ctypes.data_as(_dp), Fp.ctypes.data_as(_dp), stride,
                        cond.ctypes.data_as(_dp) if want_cond else None,
                        amps.ctypes.data_as(_dp) if want_amps else None,
                        chans.ctypes.data_as(_i32p) if chans is not None else None, nch)
    if rc:
        raise ValueError(f"oracle fstat failed ({rc})")
    out = (Fh, Fp)
    if want_cond:
        out += (cond,)
    if want_amps:
        out += (amps,)
    return out


# ---- numpy restatements used by the pins ---------------------------------

def inner(a, b, psd, df):
    """<a,b> = 4 df Re sum a conj(b) / S (Sec. II.A, Eq. "inner_product")."""
    return 4.0 * df * np.real(np.sum(a * np.conj(b) / psd))


def fstat_from_templates(s, A, psd, df):
    """F = 1/2 N^T M^{-1} N from explicit templates A[n, 4] (least squares, so
    a singular M is handled by the minimum-norm solution)."""
    N = np.array([inner(s, A[:, i], psd, df) for i in range(4)])
    M = np.array([[inner(A[:, i], A[:, j], psd, df) for j in range(4)] for i in range(4)])
    a = np.linalg.lstsq(M, N, rcond=1e-12)[0]
    return 0.5 * N @ a, N, M
