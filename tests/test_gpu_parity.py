"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Tolerance (FP64 path): the statistic is required to agree with the oracle to
1e-9 relative.  Where a partition's 4x4 matrix M is ill-conditioned, any two
correct FP64 evaluations of 1/2 N^T M^{-1} N differ by about eps * cond(M)
relative (backward-stable solve; the noise component along the weak
eigen-direction is amplified by cond), so each per-partition value is
checked against  1e-9 + 4 eps cond(M_l)  relative (with |F| floored at 1,
the scale of the noise-only statistic, E[F_l] = 2); the constant and its
measurement against the 50-digit reference are in tests/bars.py.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_10797_amd import synth as S
from tests.bars import FP64_KCOND, FP64_REL

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def small(torch_cuda):
    from paper_2407_10797_amd import fstat
    g = S.grid_small()
    inj = S.small_injection_params()
    sig = O.signal(inj, S.random_amplitudes(S.SMALL_SEEDS["inj"]), g.df, g.k_lo, g.nbins, g.T_obs)
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    pts = S.small_eval_points(inj, n=256)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    yield dict(g=g, inj=inj, data=data, psd=psd, pts=pts, plan=plan)
    plan.close()


def _rel(a, b, floor=1.0):
    return np.abs(a - b) / np.maximum(np.abs(b), floor)


def _check_parts(Fg, Fo, cond, np_parts):
    bad = []
    worst = 0.0
    for i in range(Fo.shape[0]):
        npi = int(np_parts[i]) if np.ndim(np_parts) else int(np_parts)
        c = cond[i, :npi]
        fin = np.isfinite(c) & (c > 0)
        if fin.any():
            excess = np.maximum(_rel(Fg[i, :npi], Fo[i, :npi])[fin] - REL, 0.0)
            worst = max(worst, float(np.max(excess / (2.0 ** -52 * c[fin]))))
    print(f"  max (|GPU - oracle| - 1e-9) / (eps cond) {worst:.3f}", flush=True)
    for i in range(Fo.shape[0]):
        npi = int(np_parts[i]) if np.ndim(np_parts) else int(np_parts)
        tol = REL + FP64_KCOND * np.where(np.isfinite(cond[i, :npi]), cond[i, :npi], 0.0)
        r = _rel(Fg[i, :npi], Fo[i, :npi])
        if np.any(r > tol):
            bad.append((i, float(r.max()), float(tol[np.argmax(r - tol)])))
    assert not bad, bad[:5]


@pytest.mark.parametrize("npart", [1, 4, 16, 64, 256])
def test_small_workload_matches_oracle(small, torch_cuda, npart):
    """Injection + 256 box points of the 20,972-bin workload, FP64, every
    partition value and the mean compared element by element."""
    s = small
    print(f"[small] Np={npart} n={len(s['pts'])}", flush=True)
    Fo, Po, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, s["pts"],
                           [npart], want_cond=True)
    F, P = s["plan"].eval(torch_cuda.from_numpy(s["pts"]), npart, want_parts=True)
    F, P = F.cpu().numpy(), P.cpu().numpy()
    _check_parts(P, Po, cond, npart)
    # F_hat: mean of the parts; relative error bounded by the worst part
    tolF = REL + FP64_KCOND * np.nanmax(np.where(np.isfinite(cond), cond, 0.0), axis=1)
    assert np.all(_rel(F, Fo) <= tolF), np.max(_rel(F, Fo))
    if npart == 1:
        assert np.max(_rel(F, Fo)) < REL


@pytest.mark.parametrize("npart", [1, 16, 256])
def test_interpolating_and_exact_bin_loops_agree(small, torch_cuda, npart):
    """Default (per-item interpolation of the smooth factors, with exact
    fallback) vs FSTAT_EVAL_EXACT (exact template at every bin): within the
    plan's refinement budget (5e-10 relative) per partition, plus 4 eps
    cond(M_l); both against the oracle elsewhere."""
    s = small
    _, _, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, s["pts"],
                         [npart], want_cond=True)
    F, P = s["plan"].eval(torch_cuda.from_numpy(s["pts"]), npart, want_parts=True)
    items, rej, ref, mix = s["plan"].interp_stats(bin_mix=True)
    Fe, Pe = s["plan"].eval(torch_cuda.from_numpy(s["pts"]), npart, want_parts=True, exact=True)
    items_e, rej_e, ref_e = s["plan"].interp_stats()
    print(f"[interp] Np={npart}: {items} items, {rej} handed to the exact loop, {ref} refined; "
          f"bins direct {sum(mix[:3])}, recurrence {sum(mix[3:6])}, exact {mix[6]}", flush=True)
    assert items == items_e and rej_e == items_e and ref_e == 0
    # runs: at most one per lane of each interpolated item; [13] the exact items
    assert mix[13] == rej and sum(mix[7:13]) <= 64 * (items - rej)
    if npart == 1:
        # items of >= 32 bins exist only at Np = 1 here: most go through the
        # interpolating loop, so this compares the two loops, not one with itself
        assert rej < items // 2, (rej, items)
        # the short, fast-chirping items of this workload take the direct form
        # of the bin loop (the paper-scale tests cover the difference recurrence)
        assert sum(mix[:3]) > 0
    P, Pe = P.cpu().numpy(), Pe.cpu().numpy()
    c = np.where(np.isfinite(cond[:, :npart]), cond[:, :npart], 0.0)
    r = _rel(P[:, :npart], Pe[:, :npart])
    assert np.all(r <= 5e-10 + FP64_KCOND * c), float(r.max())


def test_uneven_np_in_one_launch(small, torch_cuda):
    """Mixed partition counts in one batch equal separate uniform launches."""
    s = small
    pts = s["pts"][:64]
    nps = np.array([1, 4, 16, 64, 256, 3, 7, 200] * 8, dtype=np.int32)
    F, P = s["plan"].eval(torch_cuda.from_numpy(pts), torch_cuda.from_numpy(nps), want_parts=True)
    F, P = F.cpu().numpy(), P.cpu().numpy()
    for k in np.unique(nps):
        idx = np.where(nps == k)[0]
        Fu, Pu = s["plan"].eval(torch_cuda.from_numpy(pts[idx]), int(k), want_parts=True)
        np.testing.assert_array_equal(F[idx], Fu.cpu().numpy())
        np.testing.assert_array_equal(P[idx, :k], Pu.cpu().numpy()[:, :k])


def test_many_partitions_ragged_mix(small, torch_cuda):
    """Np up to 1000 (more partitions than support bins, so many are empty)
    mixed with odd counts in one launch, element by element against the
    oracle."""
    s = small
    pts = s["pts"][:32]
    nps = np.array([1000, 3, 777, 1] * 8, dtype=np.int32)
    F, P = s["plan"].eval(torch_cuda.from_numpy(pts), torch_cuda.from_numpy(nps), 1000,
                          want_parts=True)
    Fo, Po, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, pts, nps,
                           part_stride=1000, want_cond=True)
    F, P = F.cpu().numpy(), P.cpu().numpy()
    _check_parts(P, Po, cond, nps)
    tolF = REL + FP64_KCOND * np.nanmax(np.where(np.isfinite(cond), cond, 0.0), axis=1)
    assert np.all(_rel(F, Fo) <= tolF), np.max(_rel(F, Fo))


def test_batch_composition_does_not_change_results(small, torch_cuda):
    """Results for a particle do not depend on which other particles share the launch."""
    s = small
    pts = s["pts"]
    full = s["plan"].eval(torch_cuda.from_numpy(pts), 16).cpu().numpy()
    part = s["plan"].eval(torch_cuda.from_numpy(pts[10:20]), 16).cpu().numpy()
    np.testing.assert_array_equal(full[10:20], part)


def test_waveform_matches_oracle(torch_cuda):
    from paper_2407_10797_amd import fstat
    g = S.grid_small()
    inj = S.small_injection_params()
    a = np.array([0.3, -1.2, 0.7, 0.05])
    ho = O.signal(inj, a, g.df, g.k_lo, g.nbins, g.T_obs)
    hg = fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, inj, a).cpu().numpy()
    nz = np.abs(ho) > 0
    assert np.array_equal(nz, np.abs(hg) > 0)
    assert np.max(np.abs(hg - ho)) <= 1e-9 * np.max(np.abs(ho))


def test_edge_cases(small, torch_cuda):
    """Empty support -> -inf; invalid parameters -> NaN (device pointers);
    more partitions than support bins -> empty partitions count as 0."""
    s = small
    p = s["inj"].copy()
    far = p.copy(); far[0] += 3e8
    bad = p.copy(); bad[1] = -1.0
    nan = p.copy(); nan[3] = np.nan
    F, P = s["plan"].eval(torch_cuda.from_numpy(np.vstack([p, far, bad, nan])), 1024,
                          want_parts=True)
    F, P = F.cpu().numpy(), P.cpu().numpy()
    assert np.isfinite(F[0]) and F[1] == -np.inf and np.isnan(F[2]) and np.isnan(F[3])
    assert np.all(P[1] == 0)
    Fo, Po, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, p, [1024],
                           want_cond=True)
    assert (Po[0] == 0).sum() > 500          # most of the 1024 partitions are empty
    np.testing.assert_array_equal(P[0] == 0, Po[0] == 0)
    _check_parts(P[:1], Po, cond, 1024)
    tolF = REL + FP64_KCOND * np.nanmax(np.where(np.isfinite(cond), cond, 0.0))
    assert abs(F[0] - Fo[0]) <= tolF * max(abs(Fo[0]), 1.0)


def test_host_pointer_errors(small, torch_cuda):
    """Host-pointer calls validate and fail with EINVAL and a message."""
    from paper_2407_10797_amd import fstat
    import ctypes
    s = small
    bad = s["inj"].copy(); bad[2] = 1.5
    prm = np.ascontiguousarray(bad[None, :])
    out = np.zeros(1)
    with pytest.raises(fstat.FstatError) as e:
        fstat.fstat_eval(s["plan"].handle, prm.ctypes.data, 1, None, 4, out.ctypes.data, None, None, 0, 0)
    assert e.value.code == fstat.FSTAT_EINVAL and "invalid" in str(e.value)
    with pytest.raises(fstat.FstatError):
        fstat.fstat_eval(s["plan"].handle, prm.ctypes.data, -1, None, 4, out.ctypes.data, None, None, 0, 0)
    # n = 0 is a no-op
    fstat.fstat_eval(s["plan"].handle, prm.ctypes.data, 0, None, 4, out.ctypes.data, None, None, 0, 0)
    # host pointer path gives the same values as the device path
    good = np.ascontiguousarray(s["pts"][:8])
    outh = np.zeros(8)
    fstat.fstat_eval(s["plan"].handle, good.ctypes.data, 8, None, 16, outh.ctypes.data, None, None, 0, 0)
    outd = s["plan"].eval(torch_cuda.from_numpy(good), 16).cpu().numpy()
    np.testing.assert_array_equal(outh, outd)


def test_plan_create_rejects_bad_psd(torch_cuda):
    from paper_2407_10797_amd import fstat
    g = S.grid_small()
    psd = S.psd_tdix(g.freqs()); psd[5] = 0.0
    data = np.zeros(g.nbins, dtype=np.complex128)
    desc = fstat.fstat_data_desc(g.T_obs, g.df, g.k_lo, g.nbins, data.ctypes.data, psd.ctypes.data)
    with pytest.raises(fstat.FstatError) as e:
        fstat.fstat_plan_create(desc)
    assert e.value.code == fstat.FSTAT_EINVAL
