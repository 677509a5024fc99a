"""Plain particle swarm reference (Sec. III.A of arXiv:2407.10797).

TEST INFRASTRUCTURE ONLY: used by the tests to check the device PSO stage
step by step.  Written from the paper's description of the dynamics:

  * search space: a hypercube, normalised to [0, 1]^6 per run;
  * initialisation x ~ U[a, b], v ~ U[a - x, b - x];
  * each iteration: fitness of every particle (let-them-fly: particles
    outside the box get -inf and are not evaluated), personal best p_i
    (strict improvement), local best l_i over the ring neighbourhood
    {i-K, ..., i+K} (global best when it covers the swarm), then
    v <- w v + c1 r1 (p - x) + c2 r2 (l - x) with r1, r2 ~ U[0, 1] drawn per
    particle, dimension and iteration; |v_j| <= vmax; x <- x + v;
  * inertia weight linear in the iteration index; fixed iteration count.
Ties in the best searches go to the lowest particle index.

Random numbers are numpy's Philox4x64-10 bit generator (the counter-based
generator of Salmon et al., SC'11): key (seed, run), counter
(t, particle, block, 0), t = 0 at initialisation and k + 1 at iteration k,
uniform = (bits >> 11) * 2^-53.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1


def philox_block(seed: int, run: int, ctr) -> np.ndarray:
    """Philox4x64-10 output block for counter `ctr` (numpy generates counter+1 first)."""
    c = (sum(int(w) << (64 * i) for i, w in enumerate(ctr)) - 1) % (1 << 256)
    words = [(c >> (64 * i)) & _MASK for i in range(4)]
    bg = np.random.Philox(counter=np.array(words, dtype=np.uint64),
                          key=np.array([int(seed) & _MASK, int(run) & _MASK], dtype=np.uint64))
    return bg.random_raw(4).astype(np.uint64)


def uniforms12(seed: int, run: int, t: int, i: int) -> np.ndarray:
    raw = np.concatenate([philox_block(seed, run, [t, i, b, 0]) for b in range(3)])
    return (raw >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def run(fitness, box, np_runs, n_part, iters, ring_k, w_start, w_end, c1, c2, vmax, seed):
    """fitness(params[m, 6], np[m]) -> F_hat[m].  Returns a dict with best_x
    (physical), best_F, trace [iters, R] and final_x (normalised)."""
    box = np.asarray(box, dtype=np.float64).reshape(-1, 6, 2)
    R, Pn = box.shape[0], int(n_part)
    lo, hi = box[:, :, 0], box[:, :, 1]
    x = np.zeros((R, Pn, 6)); v = np.zeros((R, Pn, 6))
    for r in range(R):
        for i in range(Pn):
            u = uniforms12(seed, r, 0, i)
            x[r, i] = u[:6]
            v[r, i] = u[6:] - u[:6]
    pbx = x.copy()
    pbf = np.full((R, Pn), -np.inf)
    trace = np.zeros((iters, R))
    gb = np.zeros(R, dtype=int)
    for k in range(iters):
        params = lo[:, None, :] + x * (hi - lo)[:, None, :]
        outside = np.any((x < 0.0) | (x > 1.0), axis=2)
        F = np.full((R, Pn), -np.inf)
        inside = ~outside
        if inside.any():
            nps = np.broadcast_to(np.asarray(np_runs)[:, None], (R, Pn))
            F[inside] = fitness(params[inside], nps[inside])
        better = F > pbf
        pbf = np.where(better, F, pbf)
        pbx = np.where(better[:, :, None], x, pbx)
        for r in range(R):
            gb[r] = int(np.argmax(pbf[r]))       # first maximum = lowest index
            trace[k, r] = pbf[r, gb[r]]
        w = w_start + (w_end - w_start) * k / (iters - 1) if iters > 1 else w_start
        for r in range(R):
            for i in range(Pn):
                if ring_k <= 0 or 2 * ring_k + 1 >= Pn:
                    lb = gb[r]
                else:
                    lb = -1
                    for d in range(-ring_k, ring_k + 1):
                        q = (i + d) % Pn
                        if lb < 0 or pbf[r, q] > pbf[r, lb] or (pbf[r, q] == pbf[r, lb] and q < lb):
                            lb = q
                u = uniforms12(seed, r, k + 1, i)
                vn = w * v[r, i] + c1 * u[:6] * (pbx[r, i] - x[r, i]) + c2 * u[6:] * (pbx[r, lb] - x[r, i])
                vn = np.clip(vn, -vmax, vmax)
                v[r, i] = vn
                x[r, i] = x[r, i] + vn
    best_x = np.array([lo[r] + pbx[r, gb[r]] * (hi[r] - lo[r]) for r in range(R)])
    best_F = np.array([pbf[r, gb[r]] for r in range(R)])
    return dict(best_x=best_x, best_F=best_F, trace=trace, final_x=x)
