"""Autotuner of the bin loop: the choice it makes is one of the candidates, it
is remembered (in the process and in $FSTAT_TUNE_CACHE), and the statistic
evaluated with the tuned shape still matches the oracle to the FP64 bar."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2407_10797_amd import synth as S
from tests.bars import FP64_KCOND, FP64_REL

pytestmark = pytest.mark.gpu

CHUNKS = {256, 512, 1024, 2048, 2560, 4096, 4608, 8192}
MULTS = {1, 2, 4}


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def small(torch_cuda, tmp_path_factory):
    import os
    from paper_2407_10797_amd import fstat
    cache = tmp_path_factory.mktemp("tune") / "tune.txt"
    os.environ["FSTAT_TUNE_CACHE"] = str(cache)
    g = S.grid_small()
    inj = S.small_injection_params()
    sig = O.signal(inj, S.random_amplitudes(S.SMALL_SEEDS["inj"]), g.df, g.k_lo, g.nbins, g.T_obs)
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    pts = np.vstack([inj[None, :], S.small_eval_points(inj, 63)])
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    yield dict(g=g, data=data, psd=psd, pts=pts, plan=plan, cache=cache)
    plan.close()
    del os.environ["FSTAT_TUNE_CACHE"]


@pytest.mark.parametrize("mixed", [False, True])
def test_autotune_choice_is_cached_and_correct(small, torch_cuda, mixed):
    s = small
    prm = torch_cuda.from_numpy(s["pts"]).cuda()
    c, m, ms = s["plan"].autotune(prm, 16, mixed=mixed, force=True)
    print(f"[autotune] mixed={mixed} Np=16: chunk {c} x{m} grid, {ms:.3f} ms", flush=True)
    assert c in CHUNKS and m in MULTS and ms > 0
    c2, m2, ms2 = s["plan"].autotune(prm, 16, mixed=mixed)
    assert (c2, m2, ms2) == (c, m, -1.0)
    key = "mixed" if mixed else "fp64"
    lines = [ln for ln in s["cache"].read_text().splitlines() if ln.split("|")[0].endswith(key)]
    assert lines and lines[-1].split("|")[1].split() == [str(c), str(m), "0"]
    Fo, Po, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, s["pts"],
                           [16], want_cond=True)
    F, Fp = s["plan"].eval(prm, 16, mixed=mixed, want_parts=True)
    Fp = Fp.cpu().numpy()[:, :16]
    c16 = np.where(np.isfinite(cond[:, :16]), cond[:, :16], 1e30)
    rel = np.abs(Fp - Po[:, :16]) / np.maximum(np.abs(Po[:, :16]), 1.0)
    tol = (1e-4 + 1e-6 * c16) if mixed else (FP64_REL + FP64_KCOND * c16)
    ok = np.isfinite(Po[:, :16])
    assert np.all(rel[ok] <= tol[ok]), float((rel[ok] / tol[ok]).max())


def test_autotuned_mode_on_a_pso_batch(small, torch_cuda):
    """FSTAT_AUTOTUNE_MODE on a batched-PSO-like batch (per-particle Np 256,
    64, 16, 1): the exact and interpolating loops are both timed, the choice is
    cached with its mode, and the plan's later evaluations (whichever loop they
    take) match the oracle to the FP64 bar, partition by partition."""
    from paper_2407_10797_amd import fstat
    s = small
    nps = np.array([256, 64, 16, 1] * (len(s["pts"]) // 4), dtype=np.int32)
    pts = s["pts"][:len(nps)]
    prm = torch_cuda.from_numpy(pts).cuda()
    c, m, ms = s["plan"].autotune(prm, nps, force=True, mode=True)
    lines = [ln for ln in s["cache"].read_text().splitlines() if " npmix " in ln and "mode" in ln]
    ex = int(lines[-1].split("|")[1].split()[2])
    print(f"[autotune] PSO-like batch: chunk {c} x{m}, {'exact' if ex else 'interpolating'} loop, "
          f"{ms:.3f} ms", flush=True)
    assert c in CHUNKS and m in MULTS and ms > 0 and ex in (0, 1)
    F, P = s["plan"].eval(prm, nps, 256, want_parts=True)
    items, rej, _ = s["plan"].interp_stats()
    assert (rej == items) == bool(ex)
    Fo, Po, cond = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, pts, nps,
                           part_stride=256, want_cond=True)
    P = P.cpu().numpy()
    for i, k in enumerate(nps):
        c_ = np.where(np.isfinite(cond[i, :k]), cond[i, :k], 0.0)
        rel = np.abs(P[i, :k] - Po[i, :k]) / np.maximum(np.abs(Po[i, :k]), 1.0)
        assert np.all(rel <= FP64_REL + FP64_KCOND * c_), (i, float(rel.max()))
    # back to the interpolating loop for the other tests on this plan
    s["plan"].autotune(prm, 16, force=True)


def test_autotune_rejects_host_pointers(small):
    from paper_2407_10797_amd import fstat
    import ctypes
    pts = np.ascontiguousarray(small["pts"])
    with pytest.raises(fstat.FstatError):
        fstat.fstat_autotune(small["plan"].handle, pts.ctypes.data_as(ctypes.c_void_p).value,
                             len(pts), 16, 0)
