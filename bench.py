"""Benchmark: batched semi-coherent F-statistic on the paper-scale workload.

Workload (one step = one batched evaluation, all of the hot path):
  2.5 yr (T = 7.89e7 s) of one TDI-X channel, df = 1/T, 10-100 mHz ->
  7,101,001 bins; Gaussian noise from the TDI-X PSD plus one eccentric
  inspiral (Mc ~ U(10, 50), e0 ~ U(0, 0.1), SNR ~ U(11, 14)); 4096 particles
  uniform in t_c in [3.3, 3.8] yr, Mc in [10, 50] Msun, delta_mu in [0, 0.9],
  full sky, e0 in [0, 0.1]; Np = 64 equal-width frequency partitions.
Inputs are resident in device memory before the timed region starts.

Prints one JSON line (see the repository documentation for every field).
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks: vector ALU 256 CUs x 64 lanes x 2.4 GHz = 3.93e13
# lane-instructions/s, i.e. 78.6 TFLOP/s FP64 with FMA = 2; FP32 157.3 TFLOP/s
# (twice the FP64 rate: reached with packed FP32 instructions, which this
# build does not emit); HBM 8 TB/s.  A kernel that mixes FP64 and FP32 is held
# to the time floor f64 / peak64 + f32 / peak32.  The calibration leg measures
# the FP64 and unpacked FP32 FMA rates and the copy bandwidth on the box.
PEAK_VALU_TFLOPS = 78.6
PEAK_F32_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0
PEAK_LANE_INSTR = 256 * 64 * 2.4e9

# Algorithmic FLOPs of the interpolating loop (FMA = 2), derived from its
# arithmetic (see the repository documentation), per bin-template and per lane
# run (the lanes of an item that hold bins, each of which does its per-lane
# work once).  Direct loop, per bin: the item coordinate s and s^2, s^4, s^8
# (5), the phase polynomial in Estrin form (18) plus the linear and grid terms
# (5), sin/cos by table and Taylor series (22), w e^{i Phi} (6), and the
# moments sum W s^k: W s (2), s^6 (1), k = 0, 1 by additions (4) and 4 per
# further degree, 4 (D - 1), D the item's transfer degree: 63 + 4 (D - 1).
# FP64 difference recurrence, per bin: the grid term eps and the factor
# 1 + i eps (5), w e^{i Phi} x into the zeroth binomial moment (8), the series
# of e^{i phi} (10), E1 = E1(0) e^{i phi} (6), E0 <- E0 E1 (6), the difference
# updates (3) and the binomial moments' running sums (2 D): 38 + 2 D.  Per
# run, every loop applies the transfer coefficients to the moments, 4 sums of
# D + 1 terms (12 + 16 D); the recurrence also has its set-up (the start s,
# the Taylor shift of the phase polynomial (90), powers of the step (9), the
# forward differences (71), the two start factors (48: phase, two table
# sin/cos), the scaled differences (3): 223) and the moments' change from
# binomial to power form (Stirling numbers 2 D (D - 1), scaling 3 D, shift to
# the origin 2 D (D + 1), the run's end 2: 4 D^2 + 3 D + 2).  Every
# interpolated item takes its M-terms by quadrature (the few whose u the
# plan's model does not fit go to the exact loop).
ALG_FP64 = {"deg5": 79.0, "deg7": 87.0, "deg9": 95.0, "rec5": 48.0, "rec7": 52.0, "rec9": 56.0}
RUN_FP64 = {"deg5": 92.0, "deg7": 124.0, "deg9": 156.0, "rec5": 432.0, "rec7": 566.0, "rec9": 732.0}
# Mixed loop, per bin: the phase's forward differences in FP64 (9 additions,
# or 4 where the wave holds the fourth difference) and its reduction to one
# turn (1), FP32 sin/cos (2 instructions, not counted), w e^{i Phi} into the
# zeroth binomial moment (8 FP32) and the running sums (2 D FP32).  Per run:
# the start s (2), the Taylor shift of the phase polynomial (90), powers of
# the step (8), the bound on the fifth to ninth differences (18), the forward
# differences (D_1..D_4: 69; all nine: 99), the linear term (1), the start
# phase (4) and the run's end (2): 194 or 224 FP64; the moments' change to
# power form (4 D^2 + 3 D FP32); the coefficients (12 + 16 D FP64).
ALG_MIXED = {"deg4": (10.0, 16.0), "deg6": (10.0, 20.0),           # (FP64, FP32)
             "deg4_d4": (5.0, 16.0), "deg6_d4": (5.0, 20.0)}
RUN_MIXED = {"deg4": (300.0, 76.0), "deg6": (332.0, 162.0),
             "deg4_d4": (270.0, 76.0), "deg6_d4": (302.0, 162.0)}
BIN_MIX_KEYS = ("deg5", "deg7", "deg9", "rec5", "rec7", "rec9", "exact")
# The mixed path fills [0], [2] (transfer degree 4, 6; nine phase differences),
# [3], [5] (the same with four) and [6] (exact).
BIN_MIX_KEYS_MIXED = ("deg4", None, "deg6", "deg4_d4", None, "deg6_d4", "exact")


def bin_mix_dict(mixed, mix):
    """fstat_interp_stats bin_mix as two dicts keyed by the kind of work: the
    bins ([0..6]) and the lane runs ([7..12]; "exact": the items, [13])."""
    keys = BIN_MIX_KEYS_MIXED if mixed else BIN_MIX_KEYS
    return ({k: v for k, v in zip(keys, mix[:7]) if k is not None},
            {k: v for k, v in zip(keys, mix[7:14]) if k is not None})


def alg_flops(kind, mix, runs=True):
    """Algorithmic FLOPs of the main kernel over one launch, from the launch's
    bins and lane runs by kind of work (fstat_interp_stats bin_mix), as (FP64,
    FP32); runs=False: the per-bin work alone."""
    r = 1.0 if runs else 0.0
    if kind == "fp64":
        k = BIN_MIX_KEYS
        return sum(mix[i] * ALG_FP64[k[i]] + r * mix[7 + i] * RUN_FP64[k[i]] for i in range(6)), 0.0
    f64 = f32 = 0.0
    for i, k in enumerate(BIN_MIX_KEYS_MIXED[:6]):
        if k is not None:
            f64 += mix[i] * ALG_MIXED[k][0] + r * mix[7 + i] * RUN_MIXED[k][0]
            f32 += mix[i] * ALG_MIXED[k][1] + r * mix[7 + i] * RUN_MIXED[k][1]
    return f64, f32


def floor_peak(f64, f32, p64, p32):
    """Effective peak [TFLOP/s] of an FP64/FP32 operation mix on units of those rates."""
    return (f64 + f32) / (f64 / p64 + f32 / p32)


def calibrate(reps=10):
    """Measured peaks on this GPU: FP64 and unpacked FP32 FMA chains, and a
    1 GiB device-to-device copy."""
    from paper_2407_10797_amd import fstat
    f64, ms64 = fstat.calibrate(fstat.FSTAT_CALIB_FMA64, 2000, reps)
    f32, ms32 = fstat.calibrate(fstat.FSTAT_CALIB_FMA32, 2000, reps)
    bw, msc = fstat.calibrate(fstat.FSTAT_CALIB_COPY, 1 << 30, reps)
    return {"fp64_fma_tflops": f64, "fp32_fma_unpacked_tflops": f32, "copy_GBps": bw,
            "ms": {"fp64": ms64, "fp32": ms32, "copy": msc},
            "config": "FMA chains: 8 independent chains x 128 FMAs x 2000 rounds per lane, "
                      "16 blocks of 256 per CU; copy: 1 GiB, 16 B per lane access, read + written",
            "published": {"fp64_tflops": PEAK_VALU_TFLOPS, "fp32_tflops": PEAK_F32_TFLOPS,
                          "hbm_GBps": PEAK_HBM_GBPS}}


# Per bin-template figures of the main bin-loop kernel of each path counted
# by rocprofv3 (the interpolating loop k_eval_interp;
# profiles/k_eval_interp_paper_4096x64_counters.md): floating-point operations
# executed (FP64 + FP32, FMA = 2, x64 lanes), VALU instructions, HBM bytes read
# per bin-template (FETCH_SIZE x 2, calibrated on a plain copy) and bytes
# written per launch (WRITE_SIZE).
MAIN_KERNEL = {"fp64": "k_eval_interp<false>", "mixed": "k_eval_interp<true>"}
FLOP_PER_BIN = {"fp64": 69.19, "mixed": 30.90}      # FP64 + FP32
FLOP32_PER_BIN = {"fp64": 0.00, "mixed": 20.69}      # of which FP32
VALU_PER_BIN = {"fp64": 56.42, "mixed": 30.55}
VALU32_PER_BIN = {"fp64": 0.00, "mixed": 16.01}      # of which FP32 arithmetic
TRAFFIC = {"fp64": (0.3551, 1.046e+08), "mixed": (0.2081, 6.732e+07)}
# sha256 of the bin-loop kernels' code (fstat_kernels.hip and the two headers
# it builds on, comments removed) when those counters were taken; the figures
# are reported as null once it differs.
COUNTERS_SRC_SHA = "e8889c6449f65bacb229c420ddea1065f83206feb718405fdafe89e2bf523b38"
KERNEL_HEADERS = ("fstat_internal.h", "fstat_kernels.h")


def _kernel_sha():
    """sha256 of the code of the bin-loop kernels (fstat_kernels.hip and the two
    headers it builds on) with comments and blank space removed, so that only a
    change of the code itself marks the counter figures as stale."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2407_10797_amd", "csrc")
    h = hashlib.sha256()
    for f in KERNEL_HEADERS + ("fstat_kernels.hip",):
        with open(os.path.join(csrc, f)) as fh:
            src = fh.read()
        src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
        src = re.sub(r"//[^\n]*", " ", src)
        h.update(" ".join(src.split()).encode())
    return h.hexdigest()


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_workload(n_particles: int, seed_pts: int = 2003):
    import torch
    from paper_2407_10797_amd import fstat, synth as S
    g = S.grid_paper()
    psd = S.psd_tdix(g.freqs())
    noise = S.noise(psd, g.df, S.PAPER_SEEDS["noise"])
    inj, snr = S.paper_injection_params()
    amps = S.random_amplitudes(S.PAPER_SEEDS["inj"])
    sig = fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, inj, amps).cpu().numpy()
    data = noise + S.snr_scale(sig, psd, g.df, snr) * sig
    pts = S.uniform_box(S.PAPER_BOX, n_particles, seed_pts)
    return g, data, psd, pts, inj


def time_path(plan, prm, npart, steps, warmup, mixed, surrogate=False, exact=False):
    import torch
    for _ in range(warmup):
        plan.eval(prm, npart, mixed=mixed, surrogate=surrogate, exact=exact)
    torch.cuda.synchronize()
    plan.profile_read(reset=True)
    t0 = time.perf_counter()
    for _ in range(steps):
        F = plan.eval(prm, npart, mixed=mixed, surrogate=surrogate, exact=exact)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kms, mms, launches, bins = plan.profile_read(reset=True)
    return dict(seconds=t1 - t0, kernel_ms=kms / max(launches, 1), main_ms=mms / max(launches, 1),
                bins_per_launch=bins / max(launches, 1), F=F)


def pso_boxes(inj, R, seed=4001):
    """Uneven per-run boxes around the injection: Mc widths log-spaced from 1 %
    to 0.01 %, t_c windows of 1..30 days, full sky, e0 in [0, 0.1]."""
    rng = np.random.default_rng(seed)
    widths = np.logspace(-2, -4, R)
    boxes = np.zeros((R, 6, 2))
    for r in range(R):
        wt = rng.uniform(1, 30) * 86400.0
        ct = inj[0] + rng.uniform(-0.3, 0.3) * wt
        cm = inj[1] * (1 + rng.uniform(-0.3, 0.3) * widths[r])
        boxes[r] = [[ct - wt / 2, ct + wt / 2], [cm * (1 - widths[r] / 2), cm * (1 + widths[r] / 2)],
                    [inj[2], inj[2]], [0.0, np.pi], [0.0, 2 * np.pi], [0.0, 0.1]]
    return boxes


def pso_bench(iters, surrogate=True):
    """Batched PSO stage on the 20,972-bin workload: 8 runs x 40 particles,
    per-run Np 256/64/16/1 in every launch, (w, c1, c2) = (0.7, 1.5, 1.5)."""
    import torch
    from paper_2407_10797_amd import fstat, synth as S
    g = S.grid_small()
    inj = S.small_injection_params()
    sig = fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, inj,
                         S.random_amplitudes(S.SMALL_SEEDS["inj"])).cpu().numpy()
    data, psd = S.make_data(g, S.SMALL_SEEDS["noise"], sig, S.SMALL_SNR)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    boxes = pso_boxes(inj, 8)
    nps = np.array([256, 64, 16, 1] * 2, dtype=np.int32)
    out = {}
    # work-item shape and bin loop (interpolating or exact) for this batch: 40
    # points from each run's box at the run's Np
    pts = np.vstack([S.uniform_box(boxes[r], 40, 4100 + r) for r in range(len(boxes))])
    prm = torch.from_numpy(pts).cuda()
    c, m, _ = plan.autotune(prm, np.repeat(nps, 40), mode=True)
    plan.eval(prm, np.repeat(nps, 40))
    items, rej, _ = plan.interp_stats()
    out["tuned_chunk"], out["tuned_grid_mult"] = int(c), int(m)
    out["tuned_loop"] = "exact" if rej == items else "interpolating"
    for mode, graph in (("graph", True), ("eager", False)):
        plan.pso(boxes, nps, n_part=40, iters=20, use_graph=graph, seed=4001)   # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = plan.pso(boxes, nps, n_part=40, iters=iters, use_graph=graph, seed=4001)
        dt = time.perf_counter() - t0
        out[mode] = dict(iterations_per_s=iters / dt, templates_per_s=320 * iters / dt,
                         us_per_iteration=1e6 * dt / iters)
    out["best_F"] = [float(x) for x in res["best_F"]]
    out["config"] = "8 runs x 40 particles, per-run Np 256/64/16/1, 20,972-bin data, " \
                    f"{iters} iterations, w=0.7 c1=c2=1.5 vmax=0.5 ring radius 1"
    if surrogate:
        out["surrogate"] = pso_surrogate_report(plan, boxes, nps, iters, res, inj)
    plan.close()
    return out


def _recovery(x, inj):
    """Errors of estimates x [R, 6] against the injection: relative Mc, t_c in
    seconds, sky angle in radians, absolute e0."""
    th, ph = x[:, 3], x[:, 4]
    cosd = (np.sin(th) * np.sin(inj[3]) * np.cos(ph - inj[4]) + np.cos(th) * np.cos(inj[3]))
    return dict(Mc_rel=np.abs(x[:, 1] / inj[1] - 1.0).tolist(),
                tc_s=np.abs(x[:, 0] - inj[0]).tolist(),
                sky_rad=np.arccos(np.clip(cosd, -1.0, 1.0)).tolist(),
                e0_abs=np.abs(x[:, 5] - inj[5]).tolist())


def pso_surrogate_report(plan, boxes, nps, iters, res_plain, inj):
    """The batched PSO stage with the learned eccentric-phase surrogate in its
    Np >= 16 runs (the Np = 1 runs keep the analytic template), same seed as
    the plain run: throughput, fallback counts and the recovered parameters of
    both, against the injection."""
    import torch
    t0 = time.perf_counter()
    rep = plan.train_surrogate(steps=3000)
    train_s = time.perf_counter() - t0
    plan.pso(boxes, nps, n_part=40, iters=20, use_graph=True, seed=4001, surrogate=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = plan.pso(boxes, nps, n_part=40, iters=iters, use_graph=True, seed=4001, surrogate=True)
    dt = time.perf_counter() - t0
    used, fb = plan.surrogate_stats()
    plain = _recovery(res_plain["best_x"], inj)
    sur = _recovery(res["best_x"], inj)
    return dict(iterations_per_s=iters / dt, train_s=train_s, val_rmse=rep["val_rmse"],
                last_iteration_used=used, last_iteration_fallback=fb,
                best_F=[float(x) for x in res["best_F"]], np_runs=[int(v) for v in nps],
                recovered_plain=plain, recovered_surrogate=sur,
                best_x_rel_diff=(np.abs(res["best_x"] - res_plain["best_x"])
                                 / np.maximum(np.abs(res_plain["best_x"]), 1e-300)).tolist())


def search_bench(iters, ckpt, last_stage=3, resume=False, seed=2004):
    """The three-stage search (Sec. III.B) on the paper-scale workload with the
    paper's run counts (24 t_c intervals x 24 runs, 24 x 8, 2 x 48; 128
    particles; N_seg 16, 16, 1) and `iters` iterations per stage; stages 1-2
    on the mixed path, stage 3 in FP64.  Runs stage by stage through the
    checkpoint file `ckpt` (kept with resume=True), so that a search longer
    than one process can be continued by the next, up to `last_stage`; `seed`
    seeds the PSO streams (the data stay the benchmark's)."""
    import torch
    from paper_2407_10797_amd import fstat, synth as S
    g, data, psd, pts, inj = make_workload(4096)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo)
    prm = torch.from_numpy(pts).cuda()
    plan.autotune(prm, 16, mixed=True)
    plan.autotune(prm, 1)
    if not resume and os.path.exists(ckpt):
        os.remove(ckpt)
    desc = dict(seed=seed, flags=(fstat.FSTAT_EVAL_MIXED, fstat.FSTAT_EVAL_MIXED, 0),
                checkpoint=ckpt, iters=tuple(iters))
    res, stage_s, evals = None, [None] * 3, [None] * 3
    for stage in range(1, last_stage + 1):
        res = plan.search(fstat.search_desc(S.PAPER_BOX, max_stage=stage, **desc))
        k = stage - 1
        if res["stages_resumed"] >= stage:
            _log(f"search stage {stage}: taken from {ckpt}")
            continue
        stage_s[k], evals[k] = res["stage_ms"][k] / 1e3, int(res["evals"][k])
        _log(f"search stage {stage}: {evals[k]:.3e} evaluations in {stage_s[k]:.1f} s "
             f"({evals[k] / stage_s[k]:.3e}/s); best F {res['best_F']:.2f}")
    F_true = plan.eval(torch.from_numpy(inj[None]).cuda(), 1).cpu().numpy()[0]
    plan.close()
    names = ["t_c", "Mc", "delta_mu", "theta", "phi", "e0"]
    out = dict(config=f"paper-scale workload, box {S.PAPER_BOX.tolist()}, runs (24x24, 24x8, 2x48) x 128 "
                      f"particles, iterations {tuple(iters)}, N_seg (16, 16, 1), stages 1-2 mixed, "
                      "stage 3 FP64",
               seed=seed, stages_done=int(res["stages_done"]), stage_s=stage_s, evals=evals,
               evals_per_s=[e / s if e and s else None for e, s in zip(evals, stage_s)],
               best_F=float(res["best_F"]), F_injection_coherent=float(F_true),
               stage1_F=[float(x) for x in res["stage1_F"]],
               stage2_F=[float(x) for x in res["stage2_F"]],
               estimate=dict(zip(names, map(float, res["best_x"]))),
               injection=dict(zip(names, map(float, inj))))
    if res["stages_done"] == 3:
        out["extrinsic"] = dict(zip(["D_L_m", "iota", "psi", "phi_c"], map(float, res["extrinsic"])))
    return out


def aet_bench(pts, npart, steps, warmup, autotune=True):
    """The same batch on three channels with independent noise (A, E, T),
    N and M summed over them: FP64 path."""
    import torch
    from paper_2407_10797_amd import fstat, synth as S
    g = S.grid_paper()
    inj, snr = S.paper_injection_params()
    amps = S.random_amplitudes(S.PAPER_SEEDS["inj"])
    f = g.freqs()
    psd = np.array([S.psd_channel(f, c) for c in "AET"])
    sig = np.array([fstat.waveform(g.T_obs, g.df, g.k_lo, g.nbins, inj, amps, channel=c).cpu().numpy()
                    for c in "AET"])
    rho2 = sum(4 * g.df * np.sum(np.abs(sig[i]) ** 2 / psd[i]) for i in range(3))
    data = np.array([S.noise(psd[i], g.df, S.PAPER_SEEDS["noise"] + 100 * (i + 1)) for i in range(3)])
    data += sig * (snr / np.sqrt(rho2))
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo, profile=True, channels="AET")
    del data, sig
    prm = torch.from_numpy(pts).cuda()
    extra = {}
    if autotune:
        c, m, _ = plan.autotune(prm, npart)
        extra.update(tuned_chunk=c, tuned_grid_mult=m)
    r = time_path(plan, prm, npart, steps, warmup, False)
    items, rejected, refined = plan.interp_stats()
    plan.close()
    tps = len(pts) * steps / r["seconds"]
    return dict(templates_per_s=tps, ms_per_step=1e3 * r["seconds"] / steps,
                stage_ms=r["kernel_ms"], main_kernel_ms=r["main_ms"],
                channel_bin_templates_per_s=3 * r["bins_per_launch"] / (r["kernel_ms"] * 1e-3),
                work_items=items, exact_items=rejected, refined_items=refined,
                config="A, E, T with independent noise, same particles, Np and bins as fp64", **extra)


def orbit_bench(plan, g, pts, npart, steps, warmup, mixed):
    """The main batch with a numerical orbit: exact Kepler orbits tabulated at
    Chebyshev points over 2^20-s segments covering the observation."""
    import torch
    from paper_2407_10797_amd import synth as S
    dt = 2.0 ** 20
    nseg = int(np.ceil((g.T_obs + 0.5 * dt) / dt))
    plan.set_orbit(-0.5 * dt, dt, S.kepler_orbit_nodes(-0.5 * dt, dt, nseg))
    try:
        prm = torch.from_numpy(pts).cuda()
        r = time_path(plan, prm, npart, steps, warmup, mixed)
        items, rejected, refined = plan.interp_stats()
    finally:
        plan.set_orbit()
    tps = len(pts) * steps / r["seconds"]
    return dict(templates_per_s=tps, ms_per_step=1e3 * r["seconds"] / steps,
                stage_ms=r["kernel_ms"], main_kernel_ms=r["main_ms"],
                bin_templates_per_s=r["bins_per_launch"] / (r["kernel_ms"] * 1e-3),
                work_items=items, exact_items=rejected, refined_items=refined,
                config=f"Kepler-orbit table, {nseg} segments of 2^20 s, same particles, Np and "
                       "bins as the analytic-orbit line")


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, data, psd, pts, npart, sample, sample_1core):
    """The oracle (built here with -O3 -march=native, plain IEEE double) on a
    sample of the batch: all the threads OpenMP is given, then one thread."""
    from oracle import oracle as O
    O.use_native()
    threads = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))
    O.set_threads(threads)
    t0 = time.perf_counter()
    O.fstat(data, psd, g.k_lo, g.df, g.T_obs, pts[:sample], [npart])
    dt = time.perf_counter() - t0
    O.set_threads(1)
    t0 = time.perf_counter()
    O.fstat(data, psd, g.k_lo, g.df, g.T_obs, pts[sample:sample + sample_1core], [npart])
    dt1 = time.perf_counter() - t0
    O.set_threads(threads)
    return {"value": sample / dt, "unit": "templates/s", "cores": threads, "kind": "oracle",
            "sample": f"{sample} of the {len(pts)} particles, Np={npart}, full 7,101,001-bin data, "
                      f"{dt:.1f} s on {threads} threads; one thread: {sample_1core} further "
                      f"particles in {dt1:.1f} s",
            "value_1core": sample_1core / dt1, "cpu_model": _cpu_model(),
            "build": "gcc -O3 -march=native -fopenmp -ffp-contract=off -fno-fast-math"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--np", type=int, default=64)
    ap.add_argument("--particles", type=int, default=4096)
    ap.add_argument("--cpu-sample", type=int, default=32)
    ap.add_argument("--cpu-sample-1core", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-aet", action="store_true", help="skip the three-channel measurement")
    ap.add_argument("--no-orbit", action="store_true", help="skip the numerical-orbit measurement")
    ap.add_argument("--only", choices=["fp64", "mixed", "mixed+surrogate", "pso", "search", "aet",
                                       "orbit", "exact"],
                    default=None,
                    help="one paper-scale variant, or only the batched PSO measurement, or only "
                         "the three-stage search")
    ap.add_argument("--search-iters", default="400,400,800",
                    help="PSO iterations of the three search stages (--only search)")
    ap.add_argument("--search-checkpoint", default="fstat_search.ckpt")
    ap.add_argument("--search-last-stage", type=int, default=3)
    ap.add_argument("--search-seed", type=int, default=2004, help="seed of the search's PSO streams")
    ap.add_argument("--search-resume", action="store_true",
                    help="continue from --search-checkpoint instead of starting afresh")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-steps", type=int, default=3000)
    ap.add_argument("--no-autotune", action="store_true", help="keep the default work-item shape")
    ap.add_argument("--no-calibrate", action="store_true",
                    help="skip measuring the FMA and copy peaks")
    ap.add_argument("--pso-iters", type=int, default=2000, help="0 skips the PSO measurement")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run one plain device-to-device copy of BYTES (for scaling "
                         "FETCH_SIZE/WRITE_SIZE counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: measures exactly one GPU (got --gpus {args.gpus}); "
              "sharding across GPUs is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2407_10797_amd import fstat
    assert torch.cuda.is_available(), "bench.py needs a HIP device"
    if args.copy_calibration:
        n = args.copy_calibration // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 8 * n}))
        return
    if args.only == "search":
        out = {"search": search_bench([int(x) for x in args.search_iters.split(",")],
                                      args.search_checkpoint, args.search_last_stage,
                                      args.search_resume, args.search_seed)}
        print(json.dumps(out), flush=True)
        return
    if args.only == "pso":
        out = {"pso": pso_bench(args.pso_iters, surrogate=not args.no_surrogate)}
        _log(f"pso: {out['pso']['graph']['iterations_per_s']:.1f} iterations/s with hipGraph, "
             f"{out['pso']['eager']['iterations_per_s']:.1f} eager")
        print(json.dumps(out), flush=True)
        return
    calib = None
    if not args.no_calibrate:
        calib = calibrate()
        _log(f"calibration: FP64 FMA {calib['fp64_fma_tflops']:.1f} TFLOP/s, unpacked FP32 FMA "
             f"{calib['fp32_fma_unpacked_tflops']:.1f} TFLOP/s, copy {calib['copy_GBps']:.0f} GB/s")
    _log("building workload")
    g, data, psd, pts, inj = make_workload(args.particles)
    plan = fstat.Plan(data, psd, g.T_obs, g.df, g.k_lo, profile=True)
    prm = torch.from_numpy(pts).cuda()
    torch.cuda.synchronize()
    variants = {}
    same_src = _kernel_sha() == COUNTERS_SRC_SHA
    for name, mixed, sur in (("fp64", False, False), ("mixed", True, False),
                             ("mixed+surrogate", True, True)):
        if (mixed and args.no_mixed) or (args.only and args.only != name) or (sur and args.no_surrogate):
            continue
        extra = {}
        try:
            if sur:
                t0 = time.perf_counter()
                rep = plan.train_surrogate(steps=args.surrogate_steps)
                extra = dict(train_s=time.perf_counter() - t0, val_rmse=rep["val_rmse"])
            if not args.no_autotune and not sur:
                c, m, ms = plan.autotune(prm, args.np, mixed=mixed)
                extra.update(tuned_chunk=c, tuned_grid_mult=m)
                _log(f"{name}: autotuned work item {c} bins, grid x{m}")
            r = time_path(plan, prm, args.np, args.steps, args.warmup, mixed, sur)
            items, rejected, refined, mix = plan.interp_stats(bin_mix=True)
            bmix, rmix = bin_mix_dict(mixed, mix)
            extra.update(work_items=items, exact_items=rejected, refined_items=refined,
                         bin_mix=bmix, run_mix=rmix)
            if sur:
                extra["used"], extra["fallback"] = plan.surrogate_stats()
        except fstat.FstatError as e:
            _log(f"{name}: {e}")
            continue
        tps = args.particles * args.steps / r["seconds"]
        kind = "mixed" if mixed else "fp64"
        secs = r["main_ms"] * 1e-3          # the main kernel alone (HIP events)
        bins = r["bins_per_launch"]
        # algorithmic FLOPs of the main kernel per launch, from its bin and run mix
        a64, a32 = alg_flops(kind, mix)
        alg = a64 + a32
        peak = floor_peak(a64, a32, PEAK_VALU_TFLOPS, PEAK_F32_TFLOPS)
        achieved = alg / secs / 1e12
        step_secs = r["seconds"] / args.steps
        b64, b32 = alg_flops(kind, mix, runs=False)
        roof = dict(bound="alu", achieved=achieved, peak=round(peak, 1), unit="TFLOP/s",
                    frac=achieved / peak, flop_per_launch=alg, flop_fp32_per_launch=a32,
                    frac_step=alg / step_secs / 1e12 / peak,
                    flop_bins_per_launch=b64 + b32,
                    frac_bins=(b64 + b32) / secs / 1e12 / floor_peak(b64, b32, PEAK_VALU_TFLOPS,
                                                                     PEAK_F32_TFLOPS))
        if calib:
            pm = floor_peak(a64, a32, calib["fp64_fma_tflops"], calib["fp32_fma_unpacked_tflops"])
            roof.update(peak_measured=round(pm, 1), frac_measured=achieved / pm)
        # the counted figures belong to the kernel sources they were counted on
        rd, wr = TRAFFIC[kind]
        traffic = rd * bins + wr if same_src else None
        roof["traffic"] = traffic
        variants[name] = dict(templates_per_s=tps, ms_per_step=1e3 * r["seconds"] / args.steps,
                              stage_ms=r["kernel_ms"], main_kernel=MAIN_KERNEL[kind],
                              main_kernel_ms=r["main_ms"], bins_per_launch=bins,
                              bin_templates_per_s=bins / (r["kernel_ms"] * 1e-3),
                              executed_flop_per_bin=FLOP_PER_BIN[kind] if same_src else None,
                              # issue slots: unpacked FP32 issues at the FP64 rate (measured
                              # by the calibration leg), so every VALU instruction counts once
                              valu_issue_frac=VALU_PER_BIN[kind] * bins / secs / PEAK_LANE_INSTR
                              if same_src else None,
                              hbm_GBps=traffic / secs / 1e9 if traffic else None,
                              roofline=roof, **extra)
        _log(f"{name}: {tps:.1f} templates/s, bin-loop stage {r['kernel_ms']:.2f} ms, main kernel "
             f"{r['main_ms']:.2f} ms, {r['bins_per_launch']:.3e} bin-templates/launch")
    if args.only == "exact":
        # the exact template at every bin (FSTAT_EVAL_EXACT): the reference the
        # interpolating loop is measured against; not part of the default run
        for name, mixed in (("exact-fp64", False), ("exact-mixed", True)):
            r = time_path(plan, prm, args.np, args.steps, args.warmup, mixed, exact=True)
            variants[name] = dict(templates_per_s=args.particles * args.steps / r["seconds"],
                                  ms_per_step=1e3 * r["seconds"] / args.steps,
                                  stage_ms=r["kernel_ms"], main_kernel_ms=r["main_ms"],
                                  main_kernel="k_eval_exact<true>" if mixed else "k_eval_exact<false>",
                                  bins_per_launch=r["bins_per_launch"])
            _log(f"{name}: {variants[name]['templates_per_s']:.1f} templates/s, bin-loop stage "
                 f"{r['kernel_ms']:.2f} ms")
    if not args.no_orbit and args.only in (None, "orbit"):
        for name, mixed in (("orbit-fp64", False), ("orbit-mixed", True)):
            if mixed and args.no_mixed:
                continue
            try:
                variants[name] = v = orbit_bench(plan, g, pts, args.np, args.steps, args.warmup,
                                                 mixed)
                _log(f"{name}: {v['templates_per_s']:.1f} templates/s, bin-loop stage "
                     f"{v['stage_ms']:.2f} ms, main kernel {v['main_kernel_ms']:.2f} ms")
            except fstat.FstatError as e:
                _log(f"{name}: {e}")
    plan.close()
    if not args.no_aet and args.only in (None, "aet"):
        try:
            variants["aet-fp64"] = aet_bench(pts, args.np, args.steps, args.warmup,
                                             not args.no_autotune)
            v = variants["aet-fp64"]
            _log(f"aet-fp64: {v['templates_per_s']:.1f} templates/s (3 channels), bin-loop stage "
                 f"{v['stage_ms']:.2f} ms, main kernel {v['main_kernel_ms']:.2f} ms")
        except fstat.FstatError as e:
            _log(f"aet-fp64: {e}")
    head = variants.get("fp64") or next(iter(variants.values()))
    if "roofline" not in head:
        head = dict(head, roofline=None)
    out = {
        "metric": "F-stat templates/s at 7.1M bins, Np=64; %roofline; plain vs mixed+surrogate",
        "value": head["templates_per_s"],
        "unit": "templates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "paper-scale: 2.5 yr TDI-X, 7,101,001 bins (10-100 mHz), "
                               f"{args.particles} particles per batch, Np={args.np}, FP64 path",
                   "global_batch": args.particles, "np": args.np, "nbins": int(g.nbins)},
        "roofline": head.get("roofline"),
        "variants": variants,
    }
    if calib:
        out["calibration"] = calib
    if args.pso_iters > 0:
        _log("batched PSO stage")
        out["pso"] = pso_bench(args.pso_iters, surrogate=not args.no_surrogate)
        _log(f"pso: {out['pso']['graph']['iterations_per_s']:.1f} iterations/s with hipGraph, "
             f"{out['pso']['eager']['iterations_per_s']:.1f} eager")
    if not args.no_cpu:
        _log("timing the CPU oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(g, data, psd, pts, args.np, args.cpu_sample,
                                           args.cpu_sample_1core)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
