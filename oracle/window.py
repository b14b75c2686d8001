"""Windows of a large octree for the CPU reference (TEST INFRASTRUCTURE ONLY).

At sizes where the reference cannot derive the whole mesh and CSR pattern in
reasonable time, it works on the leaves around the places of interest: a
window holds every leaf that can share a node with them and enough of those
leaves' neighbours for their hanging vertices (Alg. 3) to be found. Nothing
here computes the method; it only selects leaves.
"""
from __future__ import annotations

import numpy as np


class Leaves:
    """A set of leaves of a linear octree (the subset keeps the tree's order)."""

    def __init__(self, ax, ay, az, level, max_level, origin=(0.0, 0.0, 0.0), root_len=1.0):
        self.ax = np.ascontiguousarray(ax, np.int32)
        self.ay = np.ascontiguousarray(ay, np.int32)
        self.az = np.ascontiguousarray(az, np.int32)
        self.level = np.ascontiguousarray(level, np.uint8)
        self.max_level = int(max_level)
        self.origin = tuple(float(o) for o in origin)
        self.root_len = float(root_len)

    @property
    def n(self) -> int:
        return int(self.ax.shape[0])

    def side(self) -> np.ndarray:
        return np.int64(1) << (self.max_level - self.level.astype(np.int64))


def boxes(tree):
    lo = np.stack([tree.ax, tree.ay, tree.az], 1).astype(np.int64)
    return lo, tree.side().astype(np.int64)


def subset(tree, idx):
    idx = np.asarray(idx, np.int64)
    return Leaves(tree.ax[idx], tree.ay[idx], tree.az[idx], tree.level[idx], tree.max_level,
                  tree.origin, tree.root_len)


class LeafIndex:
    """Leaves bucketed by a uniform grid whose cell is the largest leaf side:
    leaves are aligned to their side, so each lies inside exactly one cell."""

    def __init__(self, tree):
        self.lo, self.side = boxes(tree)
        self.cell = int(self.side.max()) if self.side.size else 1
        c = self.lo // self.cell
        self.dims = c.max(0) + 1 if c.size else np.ones(3, np.int64)
        cid = (c[:, 2] * self.dims[1] + c[:, 1]) * self.dims[0] + c[:, 0]
        self.order = np.argsort(cid, kind="stable")
        self.cid = cid[self.order]

    def meeting(self, blo, bhi):
        """Indices (ascending) of the leaves whose closed box meets [blo, bhi]."""
        blo = np.asarray(blo, np.int64); bhi = np.asarray(bhi, np.int64)
        c0 = np.maximum((blo - 1) // self.cell, 0)
        c1 = np.minimum(bhi // self.cell, self.dims - 1)
        if np.any(c1 < c0):
            return np.zeros(0, np.int64)
        gx, gy, gz = np.meshgrid(*(np.arange(c0[k], c1[k] + 1) for k in range(3)), indexing="ij")
        ids = ((gz * self.dims[1] + gy) * self.dims[0] + gx).ravel()
        a = np.searchsorted(self.cid, ids, side="left")
        b = np.searchsorted(self.cid, ids, side="right")
        if (b - a).sum() == 0:
            return np.zeros(0, np.int64)
        cand = self.order[np.concatenate([np.arange(x, y) for x, y in zip(a, b) if y > x])]
        lo, side = self.lo[cand], self.side[cand]
        hit = np.all((lo <= bhi) & (lo + side[:, None] >= blo), axis=1)
        return np.sort(cand[hit])


def node_window(index, pos):
    """For a node at integer position pos: the leaves that can hold it as a
    master (a leaf's box grown by twice its side contains it: the node is one
    of its corners or a master of one of its hanging corners) and the leaves
    of the window around them (every neighbour of those leaves)."""
    near = index.meeting(pos - 2 * index.cell, pos + 2 * index.cell)
    lo, side = index.lo[near], index.side[near]
    cand = near[np.all((lo - 2 * side[:, None] <= pos) & (pos <= lo + 3 * side[:, None]), axis=1)]
    smax = int(index.side[cand].max())
    return cand, index.meeting(pos - 6 * smax, pos + 6 * smax)


def element_window(index, e):
    """The leaves around leaf e: every leaf meeting its box grown by twice its
    side (its neighbours, which decide which of its corners hang)."""
    s = int(index.side[e])
    return index.meeting(index.lo[e] - 2 * s, index.lo[e] + 3 * s)
