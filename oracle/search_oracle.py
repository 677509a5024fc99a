"""Plain three-stage hierarchical search (Sec. III.B, Fig. 2 of arXiv:2407.10797).

TEST INFRASTRUCTURE ONLY: the reference the library's search driver is
checked against, written from the paper's description of the stages:

  * stage 1: the t_c range of the full box is cut into n_slices equal,
    contiguous intervals; runs[0] PSO runs in each (N_seg = np[0]); the best of
    each interval is kept (MAX);
  * stage 2: around each of those, a box of widths width2 in (t_c, Mc), the
    other parameters over their full ranges; runs[1] runs in each; the single
    best over all of them is kept;
  * stage 3: around that point, a box of widths width3 in (t_c, Mc, theta,
    phi, e0) with delta_mu over its full range, and the same box around
    theta -> pi - theta (the statistic's theta degeneracy); runs[2] runs in
    each (N_seg = np[2], the fully coherent statistic); the best of the two is
    the estimate.

Box edges are clipped to the full box, except phi when the full box spans the
whole circle (the statistic is periodic in phi).  Every MAX takes the first of
equal values.  Runs of a stage form one batch (run index = space x runs + k)
seeded with seed + stage x 0x9E3779B97F4A7C15 (mod 2^64).
"""
from __future__ import annotations

import numpy as np

from oracle import pso_oracle

SEED_STEP = 0x9E3779B97F4A7C15


def _centred(full, j, c, w):
    lo, hi = c - 0.5 * w, c + 0.5 * w
    if j == 4 and full[4, 1] - full[4, 0] >= 2.0 * np.pi:
        return lo, hi
    lo, hi = max(lo, full[j, 0]), min(hi, full[j, 1])
    if hi < lo:
        lo = hi = min(max(c, full[j, 0]), full[j, 1])
    return lo, hi


def boxes(cfg, stage, centres=None):
    """Search boxes [n, 6, 2] of one stage."""
    full = np.asarray(cfg["box"], dtype=np.float64).reshape(6, 2)
    if stage == 1:
        n = int(cfg["n_slices"])
        out = np.repeat(full[None], n, axis=0)
        lo, hi = full[0]
        for k in range(n):
            out[k, 0, 0] = lo + (hi - lo) * k / n
            out[k, 0, 1] = hi if k + 1 == n else lo + (hi - lo) * (k + 1) / n
        return out
    centres = np.atleast_2d(np.asarray(centres, dtype=np.float64))
    if stage == 2:
        out = np.repeat(full[None], len(centres), axis=0)
        for k, c in enumerate(centres):
            out[k, 0] = _centred(full, 0, c[0], cfg["width2"][0])
            out[k, 1] = _centred(full, 1, c[1], cfg["width2"][1])
        return out
    c = centres[0]
    w = cfg["width3"]
    out = np.repeat(full[None], 2, axis=0)
    for m, th in enumerate((c[3], np.pi - c[3])):
        out[m, 0] = _centred(full, 0, c[0], w[0])
        out[m, 1] = _centred(full, 1, c[1], w[1])
        out[m, 3] = _centred(full, 3, th, w[2])
        out[m, 4] = _centred(full, 4, c[4], w[3])
        out[m, 5] = _centred(full, 5, c[5], w[4])
    return out


def _stage(fitness, cfg, stage, bx):
    runs = int(cfg["runs"][stage - 1])
    box = np.repeat(bx, runs, axis=0)
    res = pso_oracle.run(fitness, box, [cfg["np"][stage - 1]] * len(box), cfg["n_part"],
                         cfg["iters"][stage - 1], cfg["ring_k"], cfg["w"][0], cfg["w"][1],
                         cfg["c1"], cfg["c2"], cfg["vmax"],
                         (int(cfg["seed"]) + stage * SEED_STEP) % (1 << 64))
    best = []
    for sp in range(len(bx)):
        F = res["best_F"][sp * runs:(sp + 1) * runs]
        k = int(np.argmax(F)) if np.any(F > -np.inf) else -1
        x = res["best_x"][sp * runs + k] if k >= 0 else bx[sp].mean(axis=1)
        best.append((np.array(x, dtype=np.float64), float(F[k]) if k >= 0 else -np.inf))
    return best


def search(fitness, cfg):
    """fitness(params[m, 6], np[m]) -> F_hat[m].  Returns the per-stage bests
    and the estimate."""
    s1 = _stage(fitness, cfg, 1, boxes(cfg, 1))
    s2 = _stage(fitness, cfg, 2, boxes(cfg, 2, [x for x, _ in s1]))
    k = int(np.argmax([F for _, F in s2]))
    s3 = _stage(fitness, cfg, 3, boxes(cfg, 3, [s2[k][0]]))
    m = int(np.argmax([F for _, F in s3]))
    return dict(stage1=s1, stage2=s2, stage3=s3, best_x=s3[m][0], best_F=s3[m][1])
