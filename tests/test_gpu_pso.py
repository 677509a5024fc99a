"""GPU PSO stage (Sec. III.A) against the step-by-step CPU reference."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import pso_oracle as PO
from paper_2407_10797_amd import synth as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2407_10797_amd import fstat
    g = S.grid_small()
    inj = S.small_injection_params()
    sig = O.signal(inj, S.random_amplitudes(S.SMALL_SEEDS["inj"]), g.df, g.k_lo, g.nbins, g.T_obs)
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    yield dict(g=g, inj=inj, data=data, psd=psd, plan=plan)
    plan.close()


def _boxes(inj, R, seed=4001):
    """Uneven per-run boxes around the injection: Mc widths log-spaced from
    1 % to 0.01 %, t_c windows of 1..30 days, full sky, e0 in [0, 0.1]."""
    rng = np.random.default_rng(seed)
    widths = np.logspace(-2, -4, R)
    boxes = np.zeros((R, 6, 2))
    for r in range(R):
        wt = rng.uniform(1, 30) * 86400.0
        ct = inj[0] + rng.uniform(-0.3, 0.3) * wt
        cm = inj[1] * (1 + rng.uniform(-0.3, 0.3) * widths[r])
        boxes[r, 0] = [ct - wt / 2, ct + wt / 2]
        boxes[r, 1] = [cm * (1 - widths[r] / 2), cm * (1 + widths[r] / 2)]
        boxes[r, 2] = [inj[2], inj[2]]
        boxes[r, 3] = [0.0, np.pi]
        boxes[r, 4] = [0.0, 2 * np.pi]
        boxes[r, 5] = [0.0, 0.1]
    return boxes


def _oracle_fit(s):
    def fit(params, nps):
        F, _ = O.fstat(s["data"], s["psd"], s["g"].k_lo, s["g"].df, s["g"].T_obs, params, nps)
        return F
    return fit


KW = dict(n_part=12, iters=8, ring_k=1, c1=1.5, c2=1.5, vmax=0.5, seed=4001)


def test_pso_trajectory_matches_reference(setup):
    s = setup
    boxes = _boxes(s["inj"], 3)
    nps = np.array([16, 4, 1], dtype=np.int32)
    print("[pso] 3 runs x 12 particles, 8 iterations", flush=True)
    got = s["plan"].pso(boxes, nps, w=(0.7, 0.7), want_final=True, use_graph=True, **KW)
    ref = PO.run(_oracle_fit(s), boxes, nps, w_start=0.7, w_end=0.7, **KW)
    np.testing.assert_allclose(got["trace"], ref["trace"], rtol=1e-8)
    np.testing.assert_allclose(got["final_x"], ref["final_x"], rtol=0, atol=1e-9)
    np.testing.assert_allclose(got["best_x"], ref["best_x"], rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(got["best_F"], ref["best_F"], rtol=1e-8)


def test_pso_graph_replay_equals_eager_and_linear_inertia(setup):
    s = setup
    boxes = _boxes(s["inj"], 2)
    nps = np.array([8, 2], dtype=np.int32)
    a = s["plan"].pso(boxes, nps, w=(0.9, 0.4), want_final=True, use_graph=True, **KW)
    b = s["plan"].pso(boxes, nps, w=(0.9, 0.4), want_final=True, use_graph=False, **KW)
    for k in ("trace", "final_x", "best_x", "best_F"):
        np.testing.assert_array_equal(a[k], b[k])
    ref = PO.run(_oracle_fit(s), boxes, nps, w_start=0.9, w_end=0.4, **KW)
    np.testing.assert_allclose(a["final_x"], ref["final_x"], rtol=0, atol=1e-9)


def test_graph_of_several_iterations_with_remainder(setup):
    """37 iterations: two replays of a 16-iteration graph and one 5-iteration
    graph, bit for bit the eager trajectory and the step-by-step reference."""
    s = setup
    boxes = _boxes(s["inj"], 2)
    nps = np.array([4, 1], dtype=np.int32)
    kw = dict(KW, iters=37)
    a = s["plan"].pso(boxes, nps, w=(0.9, 0.4), want_final=True, use_graph=True, **kw)
    b = s["plan"].pso(boxes, nps, w=(0.9, 0.4), want_final=True, use_graph=False, **kw)
    for k in ("trace", "final_x", "best_x", "best_F"):
        np.testing.assert_array_equal(a[k], b[k])
    ref = PO.run(_oracle_fit(s), boxes, nps, w_start=0.9, w_end=0.4, **kw)
    np.testing.assert_allclose(a["trace"], ref["trace"], rtol=1e-8)
    np.testing.assert_allclose(a["final_x"], ref["final_x"], rtol=0, atol=1e-9)


def test_runs_are_independent(setup):
    """A run's trajectory does not depend on the other runs in the launch."""
    s = setup
    boxes = _boxes(s["inj"], 4)
    nps = np.array([64, 16, 4, 1], dtype=np.int32)
    full = s["plan"].pso(boxes, nps, w=(0.7, 0.7), want_final=True, **KW)
    part = s["plan"].pso(boxes[:2], nps[:2], w=(0.7, 0.7), want_final=True, **KW)
    np.testing.assert_array_equal(full["trace"][:, :2], part["trace"])
    np.testing.assert_array_equal(full["final_x"][:2], part["final_x"])


def test_staggered_stages_in_one_launch(setup):
    """8 runs x 40 particles with per-run Np 256/64/16/1 in one launch: the run
    best never decreases, stays inside its box, and is a real evaluation."""
    s = setup
    boxes = _boxes(s["inj"], 8)
    nps = np.array([256, 64, 16, 1] * 2, dtype=np.int32)
    out = s["plan"].pso(boxes, nps, n_part=40, iters=30, ring_k=1, w=(0.7, 0.7), c1=1.5, c2=1.5,
                        vmax=0.5, seed=4001)
    assert np.all(np.diff(out["trace"], axis=0) >= 0)
    assert np.all(np.isfinite(out["best_F"]))
    assert np.all(out["best_x"] >= boxes[:, :, 0] - 1e-9) and np.all(out["best_x"] <= boxes[:, :, 1] + 1e-9)
    F = s["plan"].eval(out["best_x"], nps.astype(np.int32)).cpu().numpy()
    np.testing.assert_allclose(F, out["best_F"], rtol=1e-7)


def test_pso_rejects_bad_arguments(setup):
    from paper_2407_10797_amd import fstat
    s = setup
    boxes = _boxes(s["inj"], 1)
    with pytest.raises(fstat.FstatError):
        s["plan"].pso(boxes, [0], n_part=4, iters=1)
    bad = boxes.copy(); bad[0, 1] = [31.0, 29.0]
    with pytest.raises(fstat.FstatError):
        s["plan"].pso(bad, [1], n_part=4, iters=1)
    with pytest.raises(fstat.FstatError):
        s["plan"].pso(boxes, [1], n_part=2048, iters=1)
