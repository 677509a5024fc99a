"""fstat_eval_noalloc, the allocation-free variant of fstat_eval, against
fstat_eval through the C ABI: same kernels on a fixed scratch array instead
of the plan's workspace, so the results must be identical bit for bit.  Two
calls in a row, the second smaller (the scratch keeps the first call's
contents), on the FP64 interpolating, mixed and exact paths, plus the
host-side rejections (a call beyond the scratch, the surrogate)."""
import numpy as np
import pytest

from paper_2407_10797_amd import synth as S

pytestmark = pytest.mark.gpu


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
    sig = fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, inj,
                         S.random_amplitudes(S.SMALL_SEEDS["inj"])).cpu().numpy()
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    pts = S.small_eval_points(inj, n=320)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    yield dict(g=g, pts=pts, plan=plan)
    plan.close()


def _both(plan, torch, pts, np_parts, **kw):
    ref = plan.eval(torch.from_numpy(pts), np_parts, want_parts=True, want_amps=True, **kw)
    got = plan.eval(torch.from_numpy(pts), np_parts, want_parts=True, want_amps=True,
                    noalloc=True, **kw)
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ref], [t.cpu().numpy() for t in got]


@pytest.mark.parametrize("path", ["fp64", "mixed", "exact"])
def test_noalloc_equals_fstat_eval_on_two_calls(small, torch_cuda, path):
    kw = dict(mixed=path == "mixed", exact=path == "exact")
    pts = small["pts"]
    # first call: 320 particles at Np = 256 (about 85k work items)
    print(f"[noalloc] {path}: 320 particles, Np=256", flush=True)
    ref, got = _both(small["plan"], torch_cuda, pts, 256, **kw)
    for r, x in zip(ref, got):
        np.testing.assert_array_equal(x, r)
    assert np.isfinite(got[0]).all()
    # second call, smaller and ragged: 40 particles with Np 1..64 in one launch
    nps = np.array([1, 3, 16, 64, 7] * 8, dtype=np.int32)
    print(f"[noalloc] {path}: 40 particles, ragged Np up to 64", flush=True)
    ref, got = _both(small["plan"], torch_cuda, pts[:40], nps, **kw)
    for r, x in zip(ref, got):
        np.testing.assert_array_equal(x, r)
    assert np.isfinite(got[0]).all()


def test_noalloc_rejects_calls_beyond_its_scratch(small, torch_cuda):
    from paper_2407_10797_amd import fstat
    torch = torch_cuda
    n = 20000                     # 20,000 x (11 tiles + 256) items: ~2.8 GB > 128 MiB
    prm = torch.from_numpy(np.repeat(small["pts"][:1], n, axis=0)).cuda()
    F = torch.empty(n, device="cuda", dtype=torch.float64)
    with pytest.raises(fstat.FstatError) as e:
        fstat.fstat_eval_noalloc(small["plan"].handle, prm.data_ptr(), n, None, 256, F.data_ptr(),
                                 None, None, 256, fstat.FSTAT_DEVICE_PTRS)
    assert e.value.code == fstat.FSTAT_EINVAL and "scratch" in str(e.value)
    with pytest.raises(fstat.FstatError) as e:
        fstat.fstat_eval_noalloc(small["plan"].handle, prm.data_ptr(), 1, None, 4, F.data_ptr(),
                                 None, None, 4, fstat.FSTAT_DEVICE_PTRS | fstat.FSTAT_EVAL_SURROGATE)
    assert e.value.code == fstat.FSTAT_EUNSUPPORTED
    # a rejected call leaves the entry point usable
    ref, got = _both(small["plan"], torch, small["pts"][:8], 4)
    for r, x in zip(ref, got):
        np.testing.assert_array_equal(x, r)
