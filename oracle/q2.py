"""Triquadratic (Q2) elements of the CPU reference (TEST INFRASTRUCTURE ONLY).

The paper's matrix-assembly comparison (the table of assembly times for linear
and quadratic bases) runs on a uniform 16^3 mesh, and App. A tabulates the basis
values and gradients at the (bf+1)^d Gauss points: 27 nodes and 3 x 3 x 3
Gauss points per element for bf = 2. This module numbers the nodes of a
uniform octree (all leaves on one level, so no node hangs), builds the CSR
pattern of the node pairs that share an element, and drives the plain C
element routines in ``oracle.c`` (same VMS integrand as the trilinear case,
complex-step Jacobian with the stabilisation parameters frozen).

Node numbering: node positions are integers on the grid of half the finest
element side (2 x anchor + s x side, s in {0, 1, 2}); nodes are numbered by the
Morton key of those integers (x in the lowest bit); element node a is
(a % 3, a // 3 % 3, a // 9), x fastest; dof = 4 node + c.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import core as _core
from . import mesh as _mesh

# 3-point Gauss-Legendre rule on [-1, 1]
GAUSS3_X = (-math.sqrt(0.6), 0.0, math.sqrt(0.6))
GAUSS3_W = (5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0)


def points():
    """The 27 Gauss points (x fastest) and their reference weights."""
    xi = np.array([[GAUSS3_X[a % 3], GAUSS3_X[(a // 3) % 3], GAUSS3_X[a // 9]] for a in range(27)])
    w = np.array([GAUSS3_W[a % 3] * GAUSS3_W[(a // 3) % 3] * GAUSS3_W[a // 9] for a in range(27)])
    return xi, w


class Q2Mesh:
    pass


def derive_q2_mesh(tree):
    """Nodes, element node lists and the CSR pattern of a uniform octree."""
    lev = np.asarray(tree.level, np.int64)
    if lev.size == 0 or (lev != lev[0]).any():
        raise ValueError("Q2 elements need every leaf on one level (no hanging nodes)")
    M = int(tree.max_level)
    side = np.int64(1) << (M - int(lev[0]))
    anc = np.stack([tree.ax, tree.ay, tree.az], 1).astype(np.int64)
    off = np.array([[a % 3, (a // 3) % 3, a // 9] for a in range(27)], np.int64)
    pos = 2 * anc[:, None, :] + off[None, :, :] * side                 # (E, 27, 3), half units
    keys = _mesh.morton_key(pos[..., 0], pos[..., 1], pos[..., 2])
    node_keys, inv = np.unique(keys.ravel(), return_inverse=True)
    el_node = inv.reshape(-1, 27).astype(np.int64)
    n = node_keys.size
    # node pairs of every element, plus every diagonal (all nodes are in some element)
    pairs = (el_node[:, :, None] * n + el_node[:, None, :]).ravel()
    pairs = np.unique(np.concatenate([pairs, np.arange(n, dtype=np.int64) * (n + 1)]))
    prow, pcol = pairs // n, pairs % n
    deg = np.bincount(prow, minlength=n)
    nrow_ptr = np.zeros(n + 1, np.int64)
    nrow_ptr[1:] = np.cumsum(deg)
    row_ptr = np.zeros(4 * n + 1, np.int64)
    row_ptr[1:] = np.cumsum(np.repeat(4 * deg, 4))
    col_idx = np.empty(row_ptr[-1], np.int32)
    for node in range(n):
        cols = (4 * pcol[nrow_ptr[node]:nrow_ptr[node + 1], None] + np.arange(4)).ravel()
        for c in range(4):
            r = 4 * node + c
            col_idx[row_ptr[r]:row_ptr[r + 1]] = cols
    m = Q2Mesh()
    m.n_nodes = n
    m.node_keys = node_keys
    m.node_xyz_half = _mesh._decode(node_keys)   # integer positions, half-side units
    m.el_node = el_node
    m.h = tree.root_len * float(side) / float(1 << M)
    m.row_ptr = row_ptr
    m.col_idx = col_idx
    m.nnz = int(row_ptr[-1])
    return m


def node_xyz(tree, m):
    return np.asarray(tree.origin, np.float64) + \
        tree.root_len * (m.node_xyz_half.astype(np.float64) / float(1 << (tree.max_level + 1)))


def _lib():
    L = _core.lib()
    if not getattr(L, "_q2_ready", False):
        p = C.c_void_p
        L.or_q2_element.restype = None
        L.or_q2_element.argtypes = [p, C.c_double, C.c_int, p, p, p, p, p, p]
        L.or_q2_element_frozen.restype = None
        L.or_q2_element_frozen.argtypes = [p, C.c_double, C.c_int, p, p, p, p, p, p]
        L.or_q2_assemble.restype = C.c_int64
        L.or_q2_assemble.argtypes = [p, C.c_int64, p, p, C.c_int, p, p] + [p] * 7 + [p] * 4
        L._q2_ready = True
    return L


def element(prm, h, U, U0, xi=None, w=None):
    """One element: residual (108) and Jacobian (108 x 108, dof 4 a + c) at the
    Gauss points (weights scaled by (h/2)^3) unless xi, w are given."""
    if xi is None:
        xi, w = points()
        w = w * (h / 2.0) ** 3
    c = _core._c
    R = np.zeros(108)
    J = np.zeros((108, 108))
    _lib().or_q2_element(C.byref(prm), float(h), xi.shape[0], _core._p(c(xi, np.float64)),
                         _core._p(c(w, np.float64)), _core._p(c(U, np.float64)),
                         _core._p(c(U0, np.float64)), _core._p(R), _core._p(J))
    return R, J


def element_frozen(prm, h, Ub, U, U0):
    xi, w = points()
    w = w * (h / 2.0) ** 3
    c = _core._c
    R = np.zeros(108)
    _lib().or_q2_element_frozen(C.byref(prm), float(h), 27, _core._p(c(xi, np.float64)),
                                _core._p(c(w, np.float64)), _core._p(c(Ub, np.float64)),
                                _core._p(c(U, np.float64)), _core._p(c(U0, np.float64)), _core._p(R))
    return R


def assemble(tree, m, fields, prm=None, vals=True, resid=True):
    """Global Q2 Jacobian values (CSR of m) and residual, FP64."""
    prm = prm or _core.params()
    xi, w = points()
    c = _core._c
    E = m.el_node.shape[0]
    V = np.zeros(m.nnz) if vals else None
    R = np.zeros(4 * m.n_nodes) if resid else None
    f = {k: c(fields[k], np.float64) for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")}
    h = np.full(E, m.h)
    rc = _lib().or_q2_assemble(C.byref(prm), E, _core._p(c(m.el_node, np.int32)), _core._p(h), 27,
                               _core._p(c(xi, np.float64)), _core._p(c(w, np.float64)),
                               _core._p(f["ux"]), _core._p(f["uy"]), _core._p(f["uz"]), _core._p(f["p"]),
                               _core._p(f["ux0"]), _core._p(f["uy0"]), _core._p(f["uz0"]),
                               _core._p(m.row_ptr), _core._p(m.col_idx), _core._p(V), _core._p(R))
    if rc != 0:
        raise RuntimeError(f"pattern misses an entry of element {-rc - 1}")
    return V, R
