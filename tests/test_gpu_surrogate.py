"""Surrogate network: GPU training kernels against the FP64 reference, and the
surrogate branch of the statistic."""
import numpy as np
import pytest

from oracle import mlp_oracle as MO

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@pytest.mark.parametrize("B", [64, 256])
def test_mlp_forward_backward_match_fp64_reference(torch_cuda, B):
    """BF16 MFMA operands with FP32 accumulation vs FP64: outputs within 1e-2,
    gradients of every parameter group within 3e-2 (norm-wise)."""
    from paper_2407_10797_amd import fstat
    rng = np.random.default_rng(B)
    p = MO.init(7).astype(np.float32)
    x = rng.uniform(-1, 1, (B, 3)).astype(np.float32)
    t = (-(1.0 / (1.0 + 0.45 * (x[:, 0] + 1.0))) ** (19.0 / 9.0)).astype(np.float32)
    loss, g, y = fstat.fstat_mlp_grad(p, x, t)
    y_ref, _, _ = MO.forward(p.astype(np.float64), x.astype(np.float64))
    loss_ref, g_ref = MO.loss_and_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64))
    print(f"[mlp] B={B} y rel {_rel(y, y_ref):.2e} loss {loss:.4e} vs {loss_ref:.4e}", flush=True)
    assert _rel(y, y_ref) < 1e-2
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref
    o = 0
    for name, shape in MO.SIZES:
        n = int(np.prod(shape))
        r = _rel(g[o:o + n], g_ref[o:o + n])
        print(f"   grad {name:3s} rel {r:.2e}", flush=True)
        assert r < 3e-2, name
        o += n


@pytest.mark.parametrize("R", [1, 100, 4096 + 17])
def test_fused_inference_matches_training_forward_and_fp64(torch_cuda, R):
    """The knot-evaluation kernel (whole network in one launch, ragged row
    count) against the training forward (same operand rounding: 1e-5) and the
    FP64 reference: BF16 operands (unit roundoff 2^-9) through three 256-term
    layers of an untrained network leave ~1 % (3e-2, the gradient bar)."""
    from paper_2407_10797_amd import fstat
    rng = np.random.default_rng(R)
    p = MO.init(11).astype(np.float32)
    x = rng.uniform(-1, 1, (R, 3)).astype(np.float32)
    y = fstat.fstat_mlp_forward(p, x)
    y_ref, _, _ = MO.forward(p.astype(np.float64), x.astype(np.float64))
    Bp = ((R + 63) // 64) * 64
    xp = np.zeros((Bp, 3), np.float32)
    xp[:R] = x
    _, _, y_tr = fstat.fstat_mlp_grad(p, xp, np.zeros(Bp, np.float32))
    print(f"[mlp-infer] R={R} vs training forward {_rel(y, y_tr[:R]):.2e}, vs FP64 {_rel(y, y_ref):.2e}",
          flush=True)
    assert np.all(np.isfinite(y))
    assert _rel(y, y_tr[:R]) < 1e-5
    assert _rel(y, y_ref) < 3e-2


def test_mlp_rejects_bad_batch(torch_cuda):
    from paper_2407_10797_amd import fstat
    p = MO.init(1).astype(np.float32)
    x = np.zeros((63, 3), np.float32)
    with pytest.raises(fstat.FstatError):
        fstat.fstat_mlp_grad(p, x, np.zeros(63, np.float32))


@pytest.fixture(scope="module")
def trained(torch_cuda):
    from oracle import oracle as O
    from paper_2407_10797_amd import fstat, synth as S
    g = S.grid_small()
    inj = S.small_injection_params()
    sig = O.signal(inj, S.random_amplitudes(S.SMALL_SEEDS["inj"]), g.df, g.k_lo, g.nbins, g.T_obs)
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    print("[surrogate] training 2e6 samples", flush=True)
    rep = plan.train_surrogate(n_samples=2_000_000, batch=4096, steps=3000, lr=2e-3, seed=5001,
                               want_trace=True)
    print(f"[surrogate] held-out rmse {rep['val_rmse']:.3e} max {rep['val_max']:.3e}; loss "
          f"{rep['loss_trace'][0]:.3e} -> {rep['loss_trace'][-100:].mean():.3e}", flush=True)
    yield dict(g=g, inj=inj, plan=plan, rep=rep, box=S.small_box(inj))
    plan.close()


def test_surrogate_training_converges(trained):
    rep = trained["rep"]
    tr = rep["loss_trace"]
    assert np.all(np.isfinite(tr))
    assert tr[-100:].mean() < 1e-2 * tr[:10].mean()
    assert rep["val_rmse"] < 1e-2


def test_surrogate_branch_against_plain(trained, torch_cuda):
    """Np >= 16 stages on the noisy data: every particle that falls back gives
    the plain statistic bit for bit; particles that keep the surrogate move by
    at most 2e-2 relative (on noise, a template change of mismatch m moves F
    by ~sqrt(m) sqrt(2 F) through the residual: the mismatch bound itself is
    checked on noise-free data below); Np = 1 never uses the surrogate."""
    from paper_2407_10797_amd import synth as S
    s = trained
    pts = S.uniform_box(s["box"], 320, 5002)
    for npart in (16, 64):
        F0 = s["plan"].eval(torch_cuda.from_numpy(pts), npart).cpu().numpy()
        F1 = s["plan"].eval(torch_cuda.from_numpy(pts), npart, surrogate=True).cpu().numpy()
        used, fb, flags = s["plan"].surrogate_stats(len(pts))
        print(f"[surrogate] Np={npart}: used {used}, fallback {fb}", flush=True)
        assert used + fb == len(pts) and int(flags.sum()) == used
        np.testing.assert_array_equal(F1[flags == 0], F0[flags == 0])
        rel = np.abs(F1 - F0) / np.maximum(np.abs(F0), 1.0)
        assert np.all(rel < 2e-2), float(rel.max())
    F0 = s["plan"].eval(torch_cuda.from_numpy(pts), 1).cpu().numpy()
    F1 = s["plan"].eval(torch_cuda.from_numpy(pts), 1, surrogate=True).cpu().numpy()
    np.testing.assert_array_equal(F0, F1)
    assert s["plan"].surrogate_stats() == (0, 0)


def test_surrogate_mismatch_on_noise_free_templates(trained, torch_cuda):
    """The surrogate's mismatch bound (1e-3; reading: 1 - F(data = analytic
    template; template = surrogate) / F(analytic; analytic) at the stage's Np,
    which absorbs a constant phase per partition): for particles that keep
    the surrogate, a plan whose data is the particle's own noise-free analytic
    template, with the same trained weights, gives F_sur >= (1 - 1e-3) F_plain
    (and F_sur <= F_plain: the analytic template is the best fit)."""
    from paper_2407_10797_amd import fstat, synth as S
    s = trained
    g = s["g"]
    w = s["plan"].surrogate_params()
    pts = S.uniform_box(s["box"], 320, 5002)
    psd = S.psd_tdix(g.freqs())
    checked = 0
    for npart in (16, 64):
        s["plan"].eval(torch_cuda.from_numpy(pts), npart, surrogate=True)
        _, _, flags = s["plan"].surrogate_stats(len(pts))
        kept = np.nonzero(flags)[0][:4]
        for i in kept:
            amps = S.random_amplitudes(5100 + int(i))
            h = fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, pts[i], amps).cpu().numpy()
            plan = fstat.Plan(h, psd, g.T_obs, g.df, g.k_lo)
            try:
                plan.surrogate_params(w)
                Fp = plan.eval(torch_cuda.from_numpy(pts[i:i + 1]), npart).cpu().numpy()[0]
                Fs = plan.eval(torch_cuda.from_numpy(pts[i:i + 1]), npart,
                               surrogate=True).cpu().numpy()[0]
                used, _ = plan.surrogate_stats()
            finally:
                plan.close()
            mm = 1.0 - Fs / Fp
            print(f"[surrogate] Np={npart} particle {i}: mismatch {mm:.2e}", flush=True)
            assert used == 1                       # same parameters, same decision
            assert -1e-9 <= mm <= 1e-3
            checked += 1
    assert checked > 0


def test_forced_fallback_gives_the_plain_statistic(trained, torch_cuda):
    """Corrupted weights: every particle falls back, and the statistic is the
    plain one bit for bit."""
    from paper_2407_10797_amd import fstat, synth as S
    s = trained
    g = s["g"]
    w = s["plan"].surrogate_params()
    bad = w + np.random.default_rng(5004).normal(0.0, 5.0, w.size).astype(np.float32)
    pts = S.uniform_box(s["box"], 320, 5002)
    psd = S.psd_tdix(g.freqs())
    data = S.noise(psd, g.df, 5005)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    try:
        plan.surrogate_params(bad)
        for npart in (16, 64):
            F0 = plan.eval(torch_cuda.from_numpy(pts), npart).cpu().numpy()
            F1 = plan.eval(torch_cuda.from_numpy(pts), npart, surrogate=True).cpu().numpy()
            used, fb, flags = plan.surrogate_stats(len(pts))
            print(f"[surrogate] corrupted weights, Np={npart}: used {used}, fallback {fb}",
                  flush=True)
            assert used == 0 and fb == len(pts) and not flags.any()
            np.testing.assert_array_equal(F1, F0)
    finally:
        plan.close()


def test_surrogate_gain_report(trained, torch_cuda):
    """What the trained network buys: time of the surrogate-assisted
    evaluation vs the plain one on the PSO workload's batch (320 particles,
    Np = 16) -- reported, whatever its sign."""
    import time
    import torch
    from paper_2407_10797_amd import synth as S
    s = trained
    prm = torch.from_numpy(S.uniform_box(s["box"], 320, 5003)).cuda()
    res = {}
    for name, sur in (("plain", False), ("surrogate", True)):
        for _ in range(3):
            s["plan"].eval(prm, 16, surrogate=sur)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(50):
            s["plan"].eval(prm, 16, surrogate=sur)
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / 50
    used, fb = s["plan"].surrogate_stats()
    print(f"[surrogate] 320 particles, Np=16: plain {1e3 * res['plain']:.3f} ms, surrogate "
          f"{1e3 * res['surrogate']:.3f} ms (gain x{res['plain'] / res['surrogate']:.3f}); "
          f"used {used}, fallback {fb}", flush=True)
    assert np.isfinite(res["plain"]) and np.isfinite(res["surrogate"])
