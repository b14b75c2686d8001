"""Learned in-out filter workflow over the libvms C-ABI.

Exact signed distances come from the library's sampler (vms_sdf_sample); the
network is trained by the library's own forward/backward/Adam kernels; the
margin is calibrated on held-out points drawn like the queries:
m = safety x max |prediction - exact clamped distance|. Classification with the
filter keeps exact labels wherever the margin exceeds the network's error.
"""
from __future__ import annotations

import numpy as np

from . import inputs as I
from . import vms

FEATURES = 32


def fourier_matrix(seed: int, sigma: float) -> np.ndarray:
    return np.random.default_rng(seed + 1).normal(0.0, sigma, (FEATURES, 3))


def glorot_params(seed: int) -> np.ndarray:
    """Initial parameters: Glorot-uniform weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp in ((64, 64), (64,), (64, 64), (64,), (64, 64), (64,), (64,), (1,)):
        if len(shp) == 2:
            lim = np.sqrt(6.0 / (shp[0] + shp[1]))
            parts.append(rng.uniform(-lim, lim, shp).ravel())
        elif len(parts) == 6:
            lim = np.sqrt(6.0 / 65)
            parts.append(rng.uniform(-lim, lim, shp))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate(parts)


class LearnedFilter:
    def __init__(self, surf, trunc=0.05, seed=0, sigma=2.0, device="cuda:0", pad=2.0):
        """The network's box is the surface's bounding box grown by pad x trunc."""
        import torch
        self.torch = torch
        self.dev = torch.device(device)
        self.surf = surf
        self.lo = surf.verts.min(0) - pad * trunc
        self.hi = surf.verts.max(0) + pad * trunc
        self.trunc = trunc
        self.B = fourier_matrix(seed, sigma)
        self.theta0 = glorot_params(seed)
        self.h_inout = vms.inout_prepare(surf)
        self.net = vms.vms_mlp_create(self.lo, self.hi, self.theta0, self.B, trunc)
        self.margin = float("inf")

    def _dev(self, x):
        t = self.torch
        x = t.as_tensor(np.ascontiguousarray(x, np.float64), device=self.dev)
        return x[:, 0].contiguous(), x[:, 1].contiguous(), x[:, 2].contiguous()

    def exact_sdf(self, pts):
        px, py, pz = self._dev(pts)
        out = self.torch.empty(px.numel(), dtype=self.torch.float64, device=self.dev)
        vms.vms_sdf_sample(self.h_inout, px, py, pz, self.trunc, out)
        return out

    def train(self, n_samples, steps, batch, lr, seed=1, near_frac=0.7, decay=(0.3, 0.1)):
        """Adam on exact clamped distances; the learning rate drops by the factors in
        decay at 60% and 85% of the steps."""
        pts = I.sdf_sample_points(self.surf, self.lo, self.hi, n_samples, seed,
                                  near_frac=near_frac, near_dist=2 * self.trunc)
        px, py, pz = self._dev(pts)
        sdf = self.exact_sdf(pts)
        cuts = [int(0.6 * steps), int(0.85 * steps), steps]
        rates = [lr, lr * decay[0], lr * decay[1]]
        done, loss = 0, None
        for c, r in zip(cuts, rates):
            if c > done:
                loss = vms.vms_mlp_train(self.net, px, py, pz, sdf, c - done, batch, r)
                done = c
        return loss

    def predict(self, pts):
        px, py, pz = self._dev(pts)
        pred = self.torch.empty(px.numel(), dtype=self.torch.float32, device=self.dev)
        vms.vms_mlp_predict(self.net, px, py, pz, pred)
        return pred

    def calibrate(self, pts, safety=1.25, grid=None, min_samples=32):
        """Margin from held-out points: safety x the largest |prediction - exact
        clamped distance|. With grid = (nx, ny, nz) the margin is per cell of a
        uniform grid over the network box (cells with fewer than min_samples
        held-out points get +inf: the network never decides there). Returns the
        global margin and the errors."""
        pred = self.predict(pts).cpu().numpy().astype(np.float64)
        exact = self.exact_sdf(pts).cpu().numpy()
        inside = np.isfinite(pred)        # outside the box the answer is exact
        err = np.abs(pred[inside] - exact[inside])
        self.margin = float(safety * err.max()) if err.size else 0.0
        vms.vms_mlp_set_margin(self.net, self.margin)
        if grid is None:
            vms.vms_mlp_set_margin_grid(self.net, None)
            self.grid = None
            return self.margin, err
        n = np.asarray(grid, np.int64)
        x = np.asarray(pts, np.float64)[inside]
        c = np.floor((x - self.lo) / (self.hi - self.lo) * n).astype(np.int64)
        c = np.clip(c, 0, n - 1)
        cell = (c[:, 2] * n[1] + c[:, 1]) * n[0] + c[:, 0]
        nc = int(np.prod(n))
        emax = np.zeros(nc)
        np.maximum.at(emax, cell, err)
        cnt = np.bincount(cell, minlength=nc)
        m = np.where(cnt >= min_samples, safety * emax, np.inf).astype(np.float32)
        self.grid = m.reshape(n[2], n[1], n[0])
        vms.vms_mlp_set_margin_grid(self.net, self.grid)
        return self.margin, err

    def classify(self, pts, learned=True):
        t = self.torch
        px, py, pz = self._dev(pts)
        lab = t.zeros(px.numel(), dtype=t.uint8, device=self.dev)
        mode = vms.VMS_INOUT_LEARNED if learned else vms.VMS_INOUT_EXACT
        vms.inout_classify_prepared(self.h_inout, px, py, pz, lab, mode,
                                    self.net.value if learned else None)
        return lab

    def close(self):
        if self.net:
            vms.vms_mlp_destroy(self.net)
            self.net = None
        if self.h_inout:
            vms.inout_release(self.h_inout)
            self.h_inout = None
