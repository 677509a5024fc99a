"""The HIP path against the 50-digit evaluation of the paper's definitions
(``oracle/mp_reference.py``) on the tiny workload (64 bins; partitions of 64,
8, 2 and 1 bins; supports cut by the observation window inside the band).
This measures which side errs where the FP64 bar allows eps * cond(M):
the errors of the GPU's FP64 and mixed paths against the exact values, as
multiples of eps * cond(M_l), are printed and bounded here.
"""
import numpy as np
import pytest

from oracle import mp_reference as R
from tests.bars import FP64_KCOND, FP64_REL
from tests.tiny_workload import NPARTS, tiny

pytestmark = pytest.mark.gpu
EPS = 2.0 ** -52


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


@pytest.fixture(scope="module")
def setup(torch_cuda):
    from paper_2407_10797_amd import fstat
    tw = tiny()
    g = tw["g"]
    truth = {}
    for npart in NPARTS:
        rows = [R.fstat(tw["data"], tw["psd"], g.k_lo, g.df, g.T_obs, p, npart) for p in tw["pts"]]
        truth[npart] = (np.array([r[0] for r in rows]), np.array([r[1] for r in rows]),
                        np.array([r[2] for r in rows]))
    plan = fstat.Plan(tw["data"], tw["psd"], g.T_obs, g.df, g.k_lo)
    yield tw, truth, plan
    plan.close()


@pytest.mark.parametrize("npart", NPARTS)
@pytest.mark.parametrize("path", ["fp64", "fp64-exact", "mixed"])
def test_gpu_against_50_digits(setup, torch_cuda, npart, path):
    tw, truth, plan = setup
    print(f"[mp] path={path} Np={npart} n={len(tw['pts'])}", flush=True)
    F, P = plan.eval(torch_cuda.from_numpy(tw["pts"]), npart, want_parts=True,
                     mixed=(path == "mixed"), exact=(path == "fp64-exact"))
    F, P = F.cpu().numpy(), P.cpu().numpy()[:, :npart]
    Th, Tp, Tc = truth[npart]
    err = np.abs(P - Tp) / np.maximum(np.abs(Tp), 1.0)
    fin = Tc <= 1e12
    ratio = err[fin] / (EPS * Tc[fin])
    print(f"  max rel err {err.max():.2e}; finite cond: "
          f"max cond {(Tc[fin].max() if fin.any() else 0.0):.2e}, "
          f"max err/(eps cond) {(ratio.max() if fin.any() else 0.0):.3f}; singular parts max err "
          f"{(err[~fin].max() if (~fin).any() else 0.0):.2e}", flush=True)
    if path == "mixed":
        well = fin & (Tc <= 1e4)
        assert np.all(err[well] <= 1e-4)
        return
    assert np.all(err[fin] <= FP64_REL + FP64_KCOND * Tc[fin])
    assert np.all(err[~fin] <= 1e-9)
    np.testing.assert_allclose(F, Th, rtol=1e-9)
