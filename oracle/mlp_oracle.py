"""Plain FP64 reference of the surrogate network (forward and backward).

TEST INFRASTRUCTURE ONLY: the GPU training kernels' gradients are checked
against these.  Network: 3 -> 256 -> 256 -> 256 -> 256 -> 1, SiLU after each
hidden layer, squared-error loss averaged over the batch.  Parameter layout
(flat): W1[256][3] b1[256] | W2[256][256] b2 | W3 b3 | W4 b4 | w5[256] b5.
"""
from __future__ import annotations

import numpy as np

H = 256
SIZES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("W4", (H, H)), ("b4", (H,)), ("w5", (H,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SIZES])


def init(seed: int) -> np.ndarray:
    """He-style uniform initialisation (scale sqrt(3/fan_in)), zero biases."""
    rng = np.random.default_rng(seed)
    d = {}
    for name, shape in SIZES:
        if name.startswith("b"):
            d[name] = np.zeros(shape)
        else:
            fan_in = shape[1] if len(shape) == 2 else shape[0]
            lim = np.sqrt(3.0 / fan_in)
            d[name] = rng.uniform(-lim, lim, shape)
    return pack(d)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(flat, x):
    p = unpack(flat)
    zs, hs = [], [np.asarray(x, dtype=np.float64)]
    for l in (1, 2, 3, 4):
        z = hs[-1] @ p[f"W{l}"].T + p[f"b{l}"]
        zs.append(z)
        hs.append(z * _sig(z))
    y = hs[-1] @ p["w5"] + p["b5"][0]
    return y, zs, hs


def loss_and_grad(flat, x, t):
    """Mean squared error and its gradient with respect to the flat parameters."""
    p = unpack(flat)
    y, zs, hs = forward(flat, x)
    B = x.shape[0]
    e = y - t
    loss = float(np.mean(e * e))
    dy = 2.0 * e / B
    g = {"w5": hs[4].T @ dy, "b5": np.array([dy.sum()])}
    dh = np.outer(dy, p["w5"])
    for l in (4, 3, 2, 1):
        z = zs[l - 1]
        s = _sig(z)
        dz = dh * s * (1.0 + z * (1.0 - s))
        g[f"W{l}"] = dz.T @ hs[l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        dh = dz @ p[f"W{l}"]
    return loss, pack(g)
