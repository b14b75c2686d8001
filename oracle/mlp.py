"""CPU reference of the signed-distance network (TEST INFRASTRUCTURE ONLY).

Plain FP64 numpy. The network maps a point x of the domain box [lo, hi] to a
signed-distance estimate (negative inside the body):

    xh = 2 (x - lo) / (hi - lo) - 1                 (box -> [-1, 1]^3)
    z  = 2 pi B xh,  phi = [sin z; cos z]            (B: 32 x 3, fixed; 64 features)
    h1 = silu(W1 phi + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3)
    y  = w4 . h3 + b4                                (silu(v) = v / (1 + exp(-v)))

Loss over a batch: mean of (y - t)^2 / 2 with t the signed distance clamped
to [-T, T]. Gradients by hand-written reverse mode; Adam update.

Parameter vector layout (float, 12,545 entries): W1 (64x64, row-major,
out x in), b1 (64), W2, b2, W3, b3, w4 (64), b4 (1).
"""
from __future__ import annotations

import numpy as np

H = 64
NF = 32
SIZES = [("W1", (H, 2 * NF)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)),
         ("b3", (H,)), ("w4", (H,)), ("b4", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SIZES:
        n = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + n], np.float64).reshape(shp)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], np.float64).ravel() for name, _ in SIZES])


def init_params(seed):
    """Glorot-uniform weights, zero biases, from a seeded generator."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shp in SIZES:
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            p[name] = rng.uniform(-lim, lim, shp)
        elif name == "w4":
            lim = np.sqrt(6.0 / (H + 1))
            p[name] = rng.uniform(-lim, lim, shp)
        else:
            p[name] = np.zeros(shp)
    return pack(p)


def fourier_matrix(seed, sigma):
    return np.random.default_rng(seed + 1).normal(0.0, sigma, (NF, 3))


def features(x, lo, hi, B):
    xh = 2.0 * (np.asarray(x, np.float64) - lo) / (hi - lo) - 1.0
    z = 2.0 * np.pi * xh @ np.asarray(B, np.float64).T
    return np.concatenate([np.sin(z), np.cos(z)], axis=1)


def sig(v):
    return 1.0 / (1.0 + np.exp(-v))


def forward(theta, x, lo, hi, B, keep=False):
    p = unpack(theta)
    phi = features(x, lo, hi, B)
    a1 = phi @ p["W1"].T + p["b1"]; h1 = a1 * sig(a1)
    a2 = h1 @ p["W2"].T + p["b2"]; h2 = a2 * sig(a2)
    a3 = h2 @ p["W3"].T + p["b3"]; h3 = a3 * sig(a3)
    y = h3 @ p["w4"] + p["b4"][0]
    if keep:
        return y, (phi, a1, h1, a2, h2, a3, h3)
    return y


def dsilu(a):
    s = sig(a)
    return s * (1.0 + a * (1.0 - s))


def loss_and_grad(theta, x, sdf, lo, hi, B, T):
    """Loss and its gradient (reverse mode, by hand)."""
    p = unpack(theta)
    y, (phi, a1, h1, a2, h2, a3, h3) = forward(theta, x, lo, hi, B, keep=True)
    t = np.clip(sdf, -T, T)
    n = y.shape[0]
    r = y - t
    loss = 0.5 * np.mean(r * r)
    gy = r / n
    g = {"w4": h3.T @ gy, "b4": np.array([gy.sum()])}
    gh3 = np.outer(gy, p["w4"])
    ga3 = gh3 * dsilu(a3)
    g["W3"] = ga3.T @ h2
    g["b3"] = ga3.sum(0)
    gh2 = ga3 @ p["W3"]
    ga2 = gh2 * dsilu(a2)
    g["W2"] = ga2.T @ h1
    g["b2"] = ga2.sum(0)
    gh1 = ga2 @ p["W2"]
    ga1 = gh1 * dsilu(a1)
    g["W1"] = ga1.T @ phi
    g["b1"] = ga1.sum(0)
    return loss, pack(g)


def loss_only(theta, x, sdf, lo, hi, B, T):
    y = forward(theta, x, lo, hi, B)
    r = y - np.clip(sdf, -T, T)
    return 0.5 * np.mean(r * r)


def adam_step(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1); returns new theta, m, v."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
