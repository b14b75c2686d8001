"""CPU reference of the VMS assembly / in-out path (TEST INFRASTRUCTURE ONLY).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module. It never touches the HIP library and the HIP library never
touches it.

It drives the plain C routines in ``oracle.c`` (physics with a complex-step
Jacobian, exact predicates, recursive adaptive quadrature) and the numpy mesh
derivation in ``mesh.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

from . import mesh as _mesh

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OUT, IN, INTERCEPTED = 0, 1, 2
ALL_TERMS = 0x3FF
# Gauss abscissae, correctly rounded: 1/sqrt3 on [-1, 1]; (1 -+ 1/sqrt3)/2 on [0, 1]
XI = float.fromhex("0x1.279a74590331cp-1")
G_MINUS = float.fromhex("0x1.b0cb174df99c7p-3")
G_PLUS = float.fromhex("0x1.93cd3a2c8198ep-1")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB,
               SRC, "-lm"]
        subprocess.check_call(cmd)
    return LIB


class Params(C.Structure):
    _fields_ = [("rho", C.c_double), ("mu", C.c_double), ("dt", C.c_double),
                ("theta", C.c_double), ("c_t", C.c_double), ("c_i", C.c_double),
                ("term_mask", C.c_int32), ("pad", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        p = C.c_void_p
        L.or_assemble.restype = C.c_int64
        L.or_assemble.argtypes = [p, C.c_int64] + [p] * 7 + [p] * 7 + [p] * 4 + [C.c_int64, C.c_int64]
        L.or_surface_assemble.restype = C.c_int64
        L.or_surface_assemble.argtypes = ([p, p, C.c_int64] + [p] * 10 + [p] * 7 + [p] * 4)
        L.or_apply_jacobian.restype = None
        L.or_apply_jacobian.argtypes = [p, C.c_int64] + [p] * 7 + [p] * 7 + [p] * 2
        L.or_element.restype = None
        L.or_element.argtypes = [p, C.c_double, C.c_int, p, p, C.c_int, p, p, p, p, p]
        L.or_element_frozen.restype = None
        L.or_element_frozen.argtypes = [p, C.c_double, C.c_int, p, p, C.c_int, p, p, p, p, p]
        L.or_taus.restype = None
        L.or_taus.argtypes = [p, C.c_double, C.c_int, p, p, p, p]
        L.or_orient3d.restype = C.c_int
        L.or_orient3d.argtypes = [p, p, p, p]
        L.or_orient2d.restype = C.c_int
        L.or_orient2d.argtypes = [p, p, p, C.c_int, C.c_int]
        L.or_seg_tri.restype = C.c_int
        L.or_seg_tri.argtypes = [p] * 5
        L.or_label_points.restype = C.c_int64
        L.or_label_points.argtypes = [C.c_int64, p, C.c_int64, p, C.c_int64, p, p]
        L.or_subquad.restype = C.c_int64
        L.or_subquad.argtypes = ([C.c_int64, p, C.c_int64, p, p, C.c_double, C.c_int, C.c_int,
                                  C.c_int64, p, p, p, p, p, C.c_int64, p, p, p, p, p])
        L.or_coords.restype = None
        L.or_coords.argtypes = [p, C.c_double, C.c_int, C.c_int64, p, p, p, p]
        L.or_unsigned_dist.restype = None
        L.or_unsigned_dist.argtypes = [C.c_int64, p, p, C.c_int64, p, p]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def params(rho=1.0, mu=0.01, dt=0.01, theta=0.5, c_t=4.0, c_i=36.0, term_mask=ALL_TERMS):
    return Params(rho, mu, dt, theta, c_t, c_i, term_mask, 0)


# ---------------------------------------------------------------------------
# Geometry: exact predicates, labels, markers, adaptive quadrature
# ---------------------------------------------------------------------------


def orient3d(a, b, c, d) -> int:
    a, b, c, d = (_c(x, np.float64) for x in (a, b, c, d))
    return lib().or_orient3d(_p(a), _p(b), _p(c), _p(d))


def orient2d(a, b, c, i=0, j=1) -> int:
    a, b, c = (_c(x, np.float64) for x in (a, b, c))
    return lib().or_orient2d(_p(a), _p(b), _p(c), i, j)


def seg_tri(P, Q, a, b, c) -> int:
    P, Q, a, b, c = (_c(x, np.float64) for x in (P, Q, a, b, c))
    return lib().or_seg_tri(_p(P), _p(Q), _p(a), _p(b), _p(c))


def label_points(surf, xyz):
    """Exact labels (1 IN / on surface, 0 OUT) of points (n, 3); returns (labels, n_degenerate)."""
    v = _c(surf.verts, np.float64)
    t = _c(surf.tris, np.int32)
    x = _c(xyz, np.float64).reshape(-1, 3)
    lab = np.zeros(x.shape[0], np.uint8)
    nd = lib().or_label_points(v.shape[0], _p(v), t.shape[0], _p(t), x.shape[0], _p(x), _p(lab))
    return lab, int(nd)


def coords(origin, root_len, F, A, B, gsel):
    """x = origin + root_len*((A + B*g) 2^-F) per axis; gsel in {0, -1 (g-), +1 (g+)}."""
    A = _c(A, np.int64).reshape(-1, 3)
    B = _c(B, np.int64).reshape(-1)
    g = _c(gsel, np.int8).reshape(-1, 3)
    o = _c(origin, np.float64)
    out = np.zeros((A.shape[0], 3))
    lib().or_coords(_p(o), float(root_len), int(F), A.shape[0], _p(A), _p(B), _p(g), _p(out))
    return out


def vertex_xyz(tree, ms):
    """Physical coordinates of every vertex position (hanging included)."""
    xi = _mesh._decode(ms.vertex_keys)
    n = xi.shape[0]
    return coords(tree.origin, tree.root_len, tree.max_level, xi, np.zeros(n, np.int64),
                  np.zeros((n, 3), np.int8))


def markers(tree, ms, surf):
    """Alg. 4: count IN labels of the eight vertex positions of each element."""
    vx = vertex_xyz(tree, ms)
    vlab, nd = label_points(surf, vx)
    cnt = vlab[ms.elem_vertex].astype(np.int64).sum(1)
    mk = np.full(tree.n, INTERCEPTED, np.uint8)
    mk[cnt == 8] = IN
    mk[cnt == 0] = OUT
    return mk, vlab, nd


def subquad(tree, surf, el_idx, depth, cap=None):
    """Kept (OUT) sub-cell Gauss points of the given elements, depth-first order.

    Returns dict: el, key, lvl, xyz, n_labelled, n_degenerate."""
    el_idx = _c(el_idx, np.int64)
    v = _c(surf.verts, np.float64)
    t = _c(surf.tris, np.int32)
    if cap is None:
        cap = max(1, int(el_idx.size) * 8 * 8 ** max(depth, 0))
    out_el = np.zeros(cap, np.int64)
    out_key = np.zeros(cap, np.int32)
    out_lvl = np.zeros(cap, np.uint8)
    out_xyz = np.zeros((cap, 3))
    st = np.zeros(2, np.int64)
    o = _c(tree.origin, np.float64)
    n = lib().or_subquad(v.shape[0], _p(v), t.shape[0], _p(t), _p(o), float(tree.root_len),
                         tree.max_level, depth, el_idx.size, _p(el_idx), _p(_c(tree.ax, np.int32)),
                         _p(_c(tree.ay, np.int32)), _p(_c(tree.az, np.int32)),
                         _p(_c(tree.level, np.uint8)), cap, _p(out_el), _p(out_key), _p(out_lvl),
                         _p(out_xyz), _p(st))
    if n > cap:
        return subquad(tree, surf, el_idx, depth, cap=int(n))
    return {"el": out_el[:n], "key": out_key[:n], "lvl": out_lvl[:n], "xyz": out_xyz[:n],
            "n_labelled": int(st[0]), "n_degenerate": int(st[1])}


def subgp_xi(tree, el, key, lvl, depth):
    """Reference coordinates (in the parent element) and weights of sub-cell points."""
    el = np.asarray(el, np.int64)
    key = np.asarray(key, np.int64)
    lvl = np.asarray(lvl, np.int64)
    n = el.size
    srel = np.zeros((n, 3), np.int64)   # sub-cell anchor relative to the element, fine units
    M = tree.max_level
    SE = (np.int64(1) << (M - tree.level[el].astype(np.int64) + depth))   # element side, fine units
    gp = (key >> (3 * (depth - lvl))) & 7
    for k in range(1, depth + 1):       # digit of level k, present if k <= lvl
        d = (key >> (3 * (depth - k + 1))) & 7
        on = k <= lvl
        for ax in range(3):
            srel[:, ax] += np.where(on & (((d >> ax) & 1) == 1), SE >> k, 0)
    S = SE >> lvl
    xi = np.zeros((n, 3))
    for ax in range(3):
        g = np.where((gp >> ax) & 1, G_PLUS, G_MINUS)
        xi[:, ax] = 2.0 * (srel[:, ax] + S * g) / SE - 1.0
    h = tree.root_len * (SE.astype(np.float64) / float(1 << (M + depth)))
    w = (h / (2.0 ** (lvl + 1))) ** 3
    return xi, w


# ---------------------------------------------------------------------------
# Assembly
# ---------------------------------------------------------------------------


def element_h(tree):
    return tree.root_len * (tree.side().astype(np.float64) / float(1 << tree.max_level))


def std_points(h):
    """The 2x2x2 Gauss points (x fastest) and weights (h/2)^3."""
    xi = np.array([[XI if (g >> k) & 1 else -XI for k in range(3)] for g in range(8)])
    return xi, np.full(8, (h / 2.0) ** 3)


def point_lists(tree, mk, sub, depth, subset=None):
    """Per element: 8 Gauss points for OUT, kept sub-cell points for INTERCEPTED, none for IN.

    subset: optional element indices; the other elements get no points."""
    E = tree.n
    h = element_h(tree)
    keep = np.ones(E, bool)
    if subset is not None:
        keep = np.zeros(E, bool)
        keep[np.asarray(subset, np.int64)] = True
        if sub is not None and sub["el"].size:
            sel = keep[sub["el"]]
            sub = {k: (v[sel] if isinstance(v, np.ndarray) else v) for k, v in sub.items()}
    counts = np.where((mk == OUT) & keep, 8, 0).astype(np.int64)
    if sub is not None and sub["el"].size:
        np.add.at(counts, sub["el"], 1)
    off = np.zeros(E + 1, np.int64)
    off[1:] = np.cumsum(counts)
    xi = np.zeros((off[-1], 3))
    w = np.zeros(off[-1])
    sxi = np.array([[XI if (g >> k) & 1 else -XI for k in range(3)] for g in range(8)])
    outs = np.nonzero((mk == OUT) & keep)[0]
    for g in range(8):
        xi[off[outs] + g] = sxi[g]
        w[off[outs] + g] = (h[outs] / 2.0) ** 3
    if sub is not None and sub["el"].size:
        sx, sw = subgp_xi(tree, sub["el"], sub["key"], sub["lvl"], depth)
        # sub points come grouped by element in ascending element order
        order = np.argsort(sub["el"], kind="stable")
        el_sorted = sub["el"][order]
        first = np.searchsorted(el_sorted, el_sorted, side="left")
        rank = np.arange(el_sorted.size) - first
        dst = off[el_sorted] + rank
        xi[dst] = sx[order]
        w[dst] = sw[order]
    return off, xi, w


def assemble(tree, ms, fields, prm=None, mk=None, sub=None, depth=3, vals=True, resid=True,
             el_range=None, subset=None):
    """Global Jacobian values (CSR of ``ms``) and residual, FP64.

    Inactive nodes (no contribution from any non-IN element) get an identity
    diagonal block and a zero residual."""
    prm = prm or params()
    E = tree.n
    mk = np.zeros(E, np.uint8) if mk is None else mk
    off, xi, w = point_lists(tree, mk, sub, depth, subset)
    h = element_h(tree)
    Cm = _c(ms.C, np.float64)
    V = np.zeros(ms.nnz) if vals else None
    R = np.zeros(4 * ms.n_nodes) if resid else None
    f = {k: _c(fields[k], np.float64) for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")}
    b, e = (0, E) if el_range is None else el_range
    rc = lib().or_assemble(C.byref(prm), E, _p(_c(ms.nm, np.int32)), _p(_c(ms.masters, np.int32)),
                           _p(Cm), _p(_c(h, np.float64)), _p(off), _p(_c(xi, np.float64)),
                           _p(_c(w, np.float64)), _p(f["ux"]), _p(f["uy"]), _p(f["uz"]),
                           _p(f["p"]), _p(f["ux0"]), _p(f["uy0"]), _p(f["uz0"]),
                           _p(ms.row_ptr), _p(ms.col_idx), _p(V), _p(R), b, e)
    if rc != 0:
        raise RuntimeError(f"pattern misses an entry of element {-rc - 1}")
    if el_range is None and subset is None and V is not None:
        inact = np.nonzero(~ms.node_active)[0]
        for n in inact:
            for c in range(4):
                r = 4 * n + c
                k = ms.row_ptr[r] + np.searchsorted(ms.col_idx[ms.row_ptr[r]:ms.row_ptr[r + 1]], r)
                V[k] = 1.0
    return V, R


# Surface quadrature of the weak boundary terms: three points per triangle at
# barycentric coordinates (2/3, 1/6, 1/6) and permutations, a third of the
# area each (exact for quadratics).
SURF_BARY = ((2.0 / 3.0, 1.0 / 6.0, 1.0 / 6.0), (1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0),
             (1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0))


def surface_points(tree, surf, mk):
    """Surface Gauss points of eq. (weakbc), each in the leaf octant that
    contains it (half-open boxes at the finest resolution); points in IN
    octants or outside the domain are dropped. The normal is that of the fluid
    domain: minus the body's outward normal. Returns el, xi, w, n, tri sorted
    by element (stable in triangle, then point order)."""
    v = _c(surf.verts, np.float64)
    t = _c(surf.tris, np.int64)
    a, b, c = v[t[:, 0]], v[t[:, 1]], v[t[:, 2]]
    e1, e2 = b - a, c - a
    cr = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                   e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                   e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], 1)
    ln = np.sqrt(cr[:, 0] * cr[:, 0] + cr[:, 1] * cr[:, 1] + cr[:, 2] * cr[:, 2])
    nf = -cr / ln[:, None]
    wt = 0.5 * ln / 3.0
    nt = t.shape[0]
    x = np.zeros((nt, 3, 3))
    for k, (l0, l1, l2) in enumerate(SURF_BARY):
        x[:, k] = (l0 * a + l1 * b) + l2 * c
    x = x.reshape(-1, 3)
    tri = np.repeat(np.arange(nt), 3)
    w = np.repeat(wt, 3)
    n = np.repeat(nf, 3, axis=0)
    M = tree.max_level
    o = np.asarray(tree.origin, np.float64)
    sc = float(1 << M) / tree.root_len
    q = np.floor((x - o) * sc).astype(np.int64)
    inside = np.all((q >= 0) & (q < (1 << M)), axis=1)
    el = np.full(x.shape[0], -1, np.int64)
    A = np.stack([tree.ax, tree.ay, tree.az], 1).astype(np.int64)
    lev = np.asarray(tree.level, np.int64)
    for L in np.unique(lev):
        sel = np.nonzero(lev == L)[0]
        keys = A[sel, 0] | (A[sel, 1] << 21) | (A[sel, 2] << 42)
        order = np.argsort(keys)
        ks = keys[order]
        m = (q >> (M - L)) << (M - L)
        pk = m[:, 0] | (m[:, 1] << 21) | (m[:, 2] << 42)
        pos = np.clip(np.searchsorted(ks, pk), 0, ks.size - 1)
        hit = inside & (ks[pos] == pk)
        el[hit] = sel[order[pos[hit]]]
    keep = el >= 0
    keep[keep] = mk[el[keep]] != IN
    el, x, w, n, tri = el[keep], x[keep], w[keep], n[keep], tri[keep]
    side = tree.side().astype(np.float64)
    h = tree.root_len * (side[el] / float(1 << M))
    lo = o + tree.root_len * (A[el].astype(np.float64) / float(1 << M))
    xi = 2.0 * (x - lo) / h[:, None] - 1.0
    order = np.argsort(el, kind="stable")
    return {"el": el[order], "xi": xi[order], "w": w[order], "n": n[order], "tri": tri[order],
            "xyz": x[order]}


def weak_bc_tau(tree, surf, sp, mu, c_b):
    """tau_B = c_b mu / h_b per element of the surface points, h_b the largest
    distance from the element's fluid (OUT) corners to the surface, at least
    0.01 h (the remark after eq. (weakbc))."""
    els = np.unique(sp["el"])
    h = element_h(tree)[els]
    A = np.stack([tree.ax, tree.ay, tree.az], 1)[els].astype(np.float64)
    o = np.asarray(tree.origin, np.float64)
    lo = o + tree.root_len * A / float(1 << tree.max_level)
    off = np.array([[(v >> k) & 1 for k in range(3)] for v in range(8)], np.float64)
    cx = (lo[:, None, :] + h[:, None, None] * off[None]).reshape(-1, 3)
    lab, _ = label_points(surf, cx)
    d = unsigned_distance(surf, cx)
    d = np.where(lab == 0, d, 0.0).reshape(-1, 8).max(1)
    hb = np.maximum(d, 0.01 * h)
    return els, c_b * mu / hb


def weak_bc(tree, ms, surf, mk, fields, c_b=4.0, g=(0.0, 0.0, 0.0), prm=None, vals=True,
            resid=True):
    """Weak boundary terms of eq. (weakbc) (surface terms only), FP64: CSR
    values of ``ms`` and residual, the Jacobian by complex step with tau_B and
    the inflow indicator frozen."""
    prm = prm or params()
    sp = surface_points(tree, surf, mk)
    els, tau = weak_bc_tau(tree, surf, sp, prm.mu, c_b)
    cnt = np.bincount(np.searchsorted(els, sp["el"]), minlength=els.size)
    off = np.zeros(els.size + 1, np.int64)
    off[1:] = np.cumsum(cnt)
    V = np.zeros(ms.nnz) if vals else None
    R = np.zeros(4 * ms.n_nodes) if resid else None
    f = {k: _c(fields[k], np.float64) for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")}
    gg = _c(np.asarray(g, np.float64), np.float64)
    rc = lib().or_surface_assemble(C.byref(prm), _p(gg), els.size, _p(_c(els, np.int32)),
                                   _p(_c(ms.nm, np.int32)), _p(_c(ms.masters, np.int32)),
                                   _p(_c(ms.C, np.float64)), _p(_c(element_h(tree), np.float64)),
                                   _p(off), _p(_c(sp["xi"], np.float64)), _p(_c(sp["w"], np.float64)),
                                   _p(_c(sp["n"], np.float64)), _p(_c(tau, np.float64)),
                                   _p(f["ux"]), _p(f["uy"]), _p(f["uz"]), _p(f["p"]), _p(f["ux0"]),
                                   _p(f["uy0"]), _p(f["uz0"]), _p(ms.row_ptr), _p(ms.col_idx),
                                   _p(V), _p(R))
    if rc != 0:
        raise RuntimeError(f"pattern misses an entry of surface item {-rc - 1}")
    return V, R, sp


def element_weights(tree, mk, sub, sp, ts_over_tv):
    """eq. (Wpart): W(e) = n_Vgp(e)/n_Tgp + (T_s/T_v) n_Sgp(e)/n_Tgp with
    n_Tgp = 8 for trilinear elements; n_Vgp = 8 for OUT, the kept sub-cell
    points for INTERCEPTED, 0 for IN; n_Sgp the element's surface points
    (``sp`` from ``surface_points``, or None)."""
    nv = np.where(mk == OUT, 8, 0).astype(np.int64)
    if sub is not None and sub["el"].size:
        np.add.at(nv, sub["el"], 1)
    ns = np.zeros(tree.n, np.int64)
    if sp is not None and sp["el"].size:
        np.add.at(ns, sp["el"], 1)
    return nv.astype(np.float64) / 8.0 + ts_over_tv * (ns.astype(np.float64) / 8.0)


def jacobian_apply(tree, ms, fields, x, prm=None, mk=None, sub=None, depth=3):
    """y = J x in FP64 without forming J: the derivative of the residual along
    x with the stabilisation parameters frozen at the state (the reading of the
    Jacobian), by one complex-step evaluation per element. Rows of inactive
    nodes get y = x (their identity blocks, as in ``assemble``)."""
    prm = prm or params()
    E = tree.n
    mk = np.zeros(E, np.uint8) if mk is None else mk
    off, xi, w = point_lists(tree, mk, sub, depth)
    h = element_h(tree)
    f = {k: _c(fields[k], np.float64) for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")}
    x = _c(x, np.float64)
    y = np.zeros(4 * ms.n_nodes)
    lib().or_apply_jacobian(C.byref(prm), E, _p(_c(ms.nm, np.int32)), _p(_c(ms.masters, np.int32)),
                            _p(_c(ms.C, np.float64)), _p(_c(h, np.float64)), _p(off),
                            _p(_c(xi, np.float64)), _p(_c(w, np.float64)), _p(f["ux"]), _p(f["uy"]),
                            _p(f["uz"]), _p(f["p"]), _p(f["ux0"]), _p(f["uy0"]), _p(f["uz0"]), _p(x),
                            _p(y))
    inact = np.nonzero(~ms.node_active)[0]
    for c in range(4):
        y[4 * inact + c] = x[4 * inact + c]
    return y


def dirichlet_nodes(ms, mk):
    """CG nodes of IN elements (their own corners that are independent
    vertices; hanging corners impose nothing on their masters): the nodes on
    which the solution procedure sets Dirichlet conditions (Section
    "Algorithms", the step that labels elements). Sorted node ids."""
    ev = ms.elem_vertex[np.asarray(mk) == IN].ravel()
    ev = ev[~ms.vertex_is_hanging[ev]]
    keys = np.unique(ms.vertex_keys[ev])
    pos = np.searchsorted(ms.node_keys, keys)
    assert np.array_equal(ms.node_keys[pos], keys)
    return pos.astype(np.int64)


def apply_dirichlet(ms, V, R, nodes):
    """Rows of the given nodes become identity rows (every other entry of the
    row zero) with zero residual (the iterate already holds the prescribed
    values, so Newton's update vanishes there). Returns new arrays."""
    V = np.array(V, np.float64)
    R = None if R is None else np.array(R, np.float64)
    for nd in np.asarray(nodes, np.int64):
        for c in range(4):
            r = 4 * nd + c
            lo, hi = ms.row_ptr[r], ms.row_ptr[r + 1]
            V[lo:hi] = 0.0
            V[lo + np.nonzero(ms.col_idx[lo:hi] == r)[0]] = 1.0
            if R is not None:
                R[r] = 0.0
    return V, R


def csr_matvec(ms, V, x):
    """y = A x for the assembled CSR (ms.row_ptr, ms.col_idx, values V), written
    out entry by entry."""
    V = np.asarray(V, np.float64)
    rid = np.repeat(np.arange(ms.row_ptr.size - 1), np.diff(ms.row_ptr))
    y = np.zeros(ms.row_ptr.size - 1)
    np.add.at(y, rid, V * np.asarray(x, np.float64)[ms.col_idx])
    return y


def linear_solve(ms, V, b):
    """Newton's linear step A x = b solved exactly (sparse LU): the definition
    that the Krylov methods of the solution procedure approximate (the paper
    uses BiCGStab, appendix on solver selection)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    n = ms.row_ptr.size - 1
    A = sp.csr_matrix((np.asarray(V, np.float64), ms.col_idx, ms.row_ptr), shape=(n, n))
    return sla.spsolve(A.tocsc(), np.asarray(b, np.float64))


def element(prm, h, xi, w, Cmat, Um, U0m):
    """Residual (nm*4) and Jacobian ((nm*4)^2) of one element in master space."""
    xi = _c(xi, np.float64).reshape(-1, 3)
    w = _c(w, np.float64)
    nm = Cmat.shape[1]
    Cm = _c(Cmat, np.float64)
    Um = _c(Um, np.float64).reshape(nm, 4)
    U0m = _c(U0m, np.float64).reshape(nm, 3)
    R = np.zeros(nm * 4)
    J = np.zeros((nm * 4) ** 2)
    lib().or_element(C.byref(prm), float(h), xi.shape[0], _p(xi), _p(w), nm, _p(Cm), _p(Um),
                     _p(U0m), _p(R), _p(J))
    return R, J.reshape(nm * 4, nm * 4)


def element_frozen(prm, h, xi, w, Cmat, Ub, Ue, U0m):
    """Residual at Ue with stabilisation parameters frozen at Ub (master space)."""
    xi = _c(xi, np.float64).reshape(-1, 3)
    nm = Cmat.shape[1]
    R = np.zeros(nm * 4)
    lib().or_element_frozen(C.byref(prm), float(h), xi.shape[0], _p(xi), _p(_c(w, np.float64)), nm,
                            _p(_c(Cmat, np.float64)), _p(_c(Ub, np.float64)), _p(_c(Ue, np.float64)),
                            _p(_c(U0m, np.float64)), _p(R))
    return R


def taus(prm, h, xi, Uv, U0v):
    xi = _c(xi, np.float64).reshape(-1, 3)
    out = np.zeros((xi.shape[0], 3))
    lib().or_taus(C.byref(prm), float(h), xi.shape[0], _p(xi), _p(_c(Uv, np.float64)),
                  _p(_c(U0v, np.float64)), _p(out))
    return out


def unsigned_distance(surf, xyz):
    v = _c(surf.verts, np.float64)
    t = _c(surf.tris, np.int32)
    x = _c(xyz, np.float64).reshape(-1, 3)
    out = np.zeros(x.shape[0])
    lib().or_unsigned_dist(t.shape[0], _p(v), _p(t), x.shape[0], _p(x), _p(out))
    return out


def signed_distance(surf, xyz):
    """Exact-sign distance: negative inside (labels from the exact test)."""
    d = unsigned_distance(surf, xyz)
    lab, _ = label_points(surf, xyz)
    return np.where(lab == 1, -d, d)


derive_mesh = _mesh.derive_mesh
