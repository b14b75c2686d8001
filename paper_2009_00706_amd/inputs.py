"""Seeded synthetic inputs: linear octrees, watertight triangle surfaces, nodal fields.

This module only *generates* inputs. It holds none of the method's arithmetic:
no node numbering, no hanging-node derivation, no quadrature, no in-out test,
no physics. Both the CPU reference and the HIP library consume what it writes.

Octree leaves are stored as a linear octree (Section "Octree based Mesh
Generation" of the paper): integer anchors (ax, ay, az) in units of
2**-max_level of the root side, plus a level. A leaf at level L has side
2**(max_level - L) units. Leaves are returned sorted by the Morton key of their
anchor (x in the lowest bit) and are 2:1 balanced across faces, edges and
vertices.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import os

import numpy as np

# ---------------------------------------------------------------------------
# Morton keys (x lowest bit), 21 bits per axis
# ---------------------------------------------------------------------------


def _spread3(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x1FFFFF)
    v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
    return v


def morton_key(x, y, z) -> np.ndarray:
    """Interleave the bits of non-negative integer coordinates, x lowest."""
    return _spread3(np.asarray(x)) | (_spread3(np.asarray(y)) << np.uint64(1)) | (
        _spread3(np.asarray(z)) << np.uint64(2))


# ---------------------------------------------------------------------------
# Octrees
# ---------------------------------------------------------------------------


@dataclass
class Octree:
    ax: np.ndarray          # int32 anchors, units of 2**-max_level of the root side
    ay: np.ndarray
    az: np.ndarray
    level: np.ndarray       # uint8
    max_level: int
    origin: tuple = (0.0, 0.0, 0.0)
    root_len: float = 1.0
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.ax.shape[0])

    def side(self) -> np.ndarray:
        return (np.int64(1) << (self.max_level - self.level.astype(np.int64)))


def _sort_leaves(ax, ay, az, lev):
    key = morton_key(ax, ay, az)
    o = np.argsort(key, kind="stable")
    return ax[o], ay[o], az[o], lev[o], key[o]


def _children(ax, ay, az, lev, M):
    half = (np.int64(1) << (M - lev.astype(np.int64) - 1))
    cx, cy, cz, cl = [], [], [], []
    for c in range(8):  # Morton order of children, x fastest
        dx, dy, dz = c & 1, (c >> 1) & 1, (c >> 2) & 1
        cx.append(ax + dx * half)
        cy.append(ay + dy * half)
        cz.append(az + dz * half)
        cl.append(lev + 1)
    return (np.concatenate(cx), np.concatenate(cy), np.concatenate(cz),
            np.concatenate(cl).astype(np.int64))


def uniform_octree(level: int, max_level: int | None = None, origin=(0.0, 0.0, 0.0),
                   root_len: float = 1.0) -> Octree:
    M = level if max_level is None else max_level
    n = 1 << level
    s = 1 << (M - level)
    g = np.arange(n, dtype=np.int64) * s
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    ax, ay, az = X.ravel(), Y.ravel(), Z.ravel()
    lev = np.full(ax.shape, level, dtype=np.int64)
    ax, ay, az, lev, _ = _sort_leaves(ax, ay, az, lev)
    return Octree(ax.astype(np.int32), ay.astype(np.int32), az.astype(np.int32),
                  lev.astype(np.uint8), M, tuple(origin), float(root_len),
                  {"kind": "uniform", "level": level})


def _locate(keys_sorted, px, py, pz):
    """Index of the leaf containing each integer point (leaves cover the point)."""
    k = morton_key(px, py, pz)
    return np.searchsorted(keys_sorted, k, side="right") - 1


def balance_21(ax, ay, az, lev, M, ext):
    """Split leaves until face-, edge- and vertex-neighbours differ by <= 1 level.

    ext = (ex, ey, ez): the domain extent in max-level units (leaves tile
    [0,ex) x [0,ey) x [0,ez)).

    A leaf at level L needs every leaf touching it at level >= L - 1. Such a
    neighbour point either lies in a sibling or in a same-size neighbour of
    the leaf's parent P (level L - 1), and a leaf coarser than P that covers a
    point of that neighbour covers the whole neighbour, anchor included. So it
    suffices to test, once per distinct parent, the leaves at the anchors of
    its 26 neighbours (an eighth of the queries of a per-leaf test).
    """
    ax = ax.astype(np.int64); ay = ay.astype(np.int64); az = az.astype(np.int64)
    lev = lev.astype(np.int64)
    ex, ey, ez = ext
    dirs = [(i, j, k) for i in (-1, 0, 1) for j in (-1, 0, 1) for k in (-1, 0, 1)
            if (i, j, k) != (0, 0, 0)]
    while True:
        ax, ay, az, lev, keys = _sort_leaves(ax, ay, az, lev)
        split = np.zeros(ax.shape[0], dtype=bool)
        has_parent = lev > 0
        plev = lev[has_parent] - 1
        pside = np.int64(1) << (M - plev)
        pm = pside - 1
        px, py, pz = ax[has_parent] & ~pm, ay[has_parent] & ~pm, az[has_parent] & ~pm
        # distinct parents (sorted by level, then Morton key of the anchor)
        pk = morton_key(px, py, pz)
        o = np.lexsort((pk, plev))
        first = np.ones(o.size, dtype=bool)
        first[1:] = (pk[o][1:] != pk[o][:-1]) | (plev[o][1:] != plev[o][:-1])
        u = o[first]
        px, py, pz, plev, pside = px[u], py[u], pz[u], plev[u], pside[u]
        for (i, j, k) in dirs:
            nx = px + i * pside
            ny = py + j * pside
            nz = pz + k * pside
            ok = (nx >= 0) & (ny >= 0) & (nz >= 0) & (nx < ex) & (ny < ey) & (nz < ez)
            idx = _locate(keys, nx[ok], ny[ok], nz[ok])
            bad = lev[idx] < plev[ok]
            split[idx[bad]] = True
        if not split.any():
            return ax, ay, az, lev
        cx, cy, cz, cl = _children(ax[split], ay[split], az[split], lev[split], M)
        keep = ~split
        ax = np.concatenate([ax[keep], cx])
        ay = np.concatenate([ay[keep], cy])
        az = np.concatenate([az[keep], cz])
        lev = np.concatenate([lev[keep], cl])


def refined_octree(M: int, lmin: int, refine, ext=None, origin=(0.0, 0.0, 0.0),
                   root_len: float = 1.0, meta=None, balance: bool = True) -> Octree:
    """Top-down construction: start uniform at lmin, split while refine() says so.

    refine(cx, cy, cz, h, level) -> bool mask, with octant centres and side in
    physical units. Leaves are then 2:1 balanced (faces, edges, vertices).
    """
    if ext is None:
        ext = (1 << M, 1 << M, 1 << M)
    s0 = 1 << (M - lmin)
    gx = np.arange(0, ext[0], s0, dtype=np.int64)
    gy = np.arange(0, ext[1], s0, dtype=np.int64)
    gz = np.arange(0, ext[2], s0, dtype=np.int64)
    X, Y, Z = np.meshgrid(gx, gy, gz, indexing="ij")
    ax, ay, az = X.ravel(), Y.ravel(), Z.ravel()
    lev = np.full(ax.shape, lmin, dtype=np.int64)
    unit = root_len / float(1 << M)
    done = ([], [], [], [])
    while ax.size:
        side = (np.int64(1) << (M - lev)).astype(np.float64)
        h = side * unit
        cx = origin[0] + (ax + 0.5 * side) * unit
        cy = origin[1] + (ay + 0.5 * side) * unit
        cz = origin[2] + (az + 0.5 * side) * unit
        m = np.asarray(refine(cx, cy, cz, h, lev), dtype=bool) & (lev < M)
        for lst, arr in zip(done, (ax, ay, az, lev)):
            lst.append(arr[~m])
        ax, ay, az, lev = _children(ax[m], ay[m], az[m], lev[m], M)
    ax, ay, az, lev = (np.concatenate(l) for l in done)
    n_pre = int(ax.shape[0])
    if balance:
        ax, ay, az, lev = balance_21(ax, ay, az, lev, M, ext)
    ax, ay, az, lev, _ = _sort_leaves(ax, ay, az, lev)
    md = {"kind": "refined", "n_before_balance": n_pre}
    if meta:
        md.update(meta)
    return Octree(ax.astype(np.int32), ay.astype(np.int32), az.astype(np.int32),
                  lev.astype(np.uint8), M, tuple(origin), float(root_len), md)


def sphere_refined_octree(center, r, lmin, lmax, beta, M=None) -> Octree:
    """Refine octants whose centre lies within beta*h of the sphere |x-c| = r."""
    M = lmax if M is None else M
    c = np.asarray(center, dtype=np.float64)

    def refine(cx, cy, cz, h, lev):
        d = np.sqrt((cx - c[0]) ** 2 + (cy - c[1]) ** 2 + (cz - c[2]) ** 2)
        return (np.abs(d - r) < beta * h) & (lev < lmax)

    return refined_octree(M, lmin, refine, meta={"body": "sphere", "beta": beta,
                                                  "lmin": lmin, "lmax": lmax})


def check_balanced(t: Octree, ext=None) -> bool:
    """True iff all face/edge/vertex neighbours differ by at most one level."""
    M = t.max_level
    ext = ext or (1 << M, 1 << M, 1 << M)
    ax, ay, az, lev = (a.astype(np.int64) for a in (t.ax, t.ay, t.az, t.level))
    ax2, ay2, az2, lev2 = balance_21(ax, ay, az, lev, M, ext)
    return ax2.shape[0] == ax.shape[0]


# ---------------------------------------------------------------------------
# Watertight surfaces (outward-oriented, counter-clockwise seen from outside)
# ---------------------------------------------------------------------------


@dataclass
class Surface:
    verts: np.ndarray   # (nv, 3) float64
    tris: np.ndarray    # (nt, 3) int32
    meta: dict = field(default_factory=dict)

    @property
    def n_tri(self):
        return int(self.tris.shape[0])


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(subdiv: int, r: float, center) -> Surface:
    v, f = _icosahedron()
    for _ in range(subdiv):
        verts = [row for row in v]
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        v = np.array(verts)
        f = np.array(nf, dtype=np.int64)
    s = Surface(v * r + np.asarray(center, dtype=np.float64), f.astype(np.int32),
                {"kind": "icosphere", "subdiv": subdiv, "r": r, "center": list(center)})
    orient_outward(s)
    return s


def random_rotation(rng) -> np.ndarray:
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


def ellipsoid(semi, center, rot, n_lat: int, n_lon: int) -> Surface:
    """Latitude-longitude tessellation with pole fans: 2*n_lon*(n_lat-1) triangles."""
    th = np.pi * (np.arange(1, n_lat) / n_lat)          # interior latitudes
    ph = 2 * np.pi * (np.arange(n_lon) / n_lon)
    T, P = np.meshgrid(th, ph, indexing="ij")
    ring = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    v = np.concatenate([[[0, 0, 1.0]], ring, [[0, 0, -1.0]]])
    v = v * np.asarray(semi)
    v = v @ np.asarray(rot).T + np.asarray(center)
    tris = []
    idx = lambda i, j: 1 + i * n_lon + (j % n_lon)
    for j in range(n_lon):
        tris.append([0, idx(0, j), idx(0, j + 1)])
    for i in range(n_lat - 2):
        for j in range(n_lon):
            a, b, c, d = idx(i, j), idx(i, j + 1), idx(i + 1, j), idx(i + 1, j + 1)
            tris += [[a, c, b], [b, c, d]]
    s_ = len(v) - 1
    for j in range(n_lon):
        tris.append([s_, idx(n_lat - 2, j + 1), idx(n_lat - 2, j)])
    s = Surface(v, np.array(tris, dtype=np.int32),
                {"kind": "ellipsoid", "semi": list(map(float, semi)), "center": list(map(float, center))})
    orient_outward(s)
    return s


def _orient_sign(a, b, c, d):
    """Sign of det[a - d; b - d; c - d] for rows of points (negative: d on the
    side from which a, b, c turn counter-clockwise): float64 with a generous
    forward error bound, exact rational arithmetic where the bound cannot
    decide."""
    from fractions import Fraction
    ad, bd, cd = a - d, b - d, c - d
    m1 = bd[:, 0] * cd[:, 1] - cd[:, 0] * bd[:, 1]
    m2 = cd[:, 0] * ad[:, 1] - ad[:, 0] * cd[:, 1]
    m3 = ad[:, 0] * bd[:, 1] - bd[:, 0] * ad[:, 1]
    det = ad[:, 2] * m1 + bd[:, 2] * m2 + cd[:, 2] * m3
    perm = (np.abs(ad[:, 2]) * (np.abs(bd[:, 0] * cd[:, 1]) + np.abs(cd[:, 0] * bd[:, 1])) +
            np.abs(bd[:, 2]) * (np.abs(cd[:, 0] * ad[:, 1]) + np.abs(ad[:, 0] * cd[:, 1])) +
            np.abs(cd[:, 2]) * (np.abs(ad[:, 0] * bd[:, 1]) + np.abs(bd[:, 0] * ad[:, 1])))
    sign = np.sign(det).astype(np.int64)
    amb = np.abs(det) <= 1e-13 * perm
    # four points with one coordinate equal lie in an axis plane: exactly 0
    same = np.zeros(det.shape, bool)
    for k in range(3):
        same |= (a[:, k] == b[:, k]) & (a[:, k] == c[:, k]) & (a[:, k] == d[:, k])
    sign[amb & same] = 0
    for r in np.nonzero(amb & ~same)[0]:
        vals = [float(x) for p in (a, b, c, d) for x in p[r]]
        if all((x * 2.0 ** 60).is_integer() for x in vals):
            A, B, C, D = ([int(x * 2.0 ** 60) for x in p[r]] for p in (a, b, c, d))   # exact
        else:
            A, B, C, D = ([Fraction(float(x)) for x in p[r]] for p in (a, b, c, d))
        u = [A[k] - D[k] for k in range(3)]
        v = [B[k] - D[k] for k in range(3)]
        w = [C[k] - D[k] for k in range(3)]
        e = (u[2] * (v[0] * w[1] - w[0] * v[1]) + v[2] * (w[0] * u[1] - u[0] * w[1]) +
             w[2] * (u[0] * v[1] - v[0] * u[1]))
        sign[r] = (e > 0) - (e < 0)
    return sign


def _edges(tris):
    """Every undirected edge once: (t1, t2, k1, k2), the two triangles and the
    position k of the edge's first vertex in each (edge k runs k -> k + 1)."""
    nt = tris.shape[0]
    t = tris.astype(np.int64)
    a = np.concatenate([t[:, k] for k in range(3)])
    b = np.concatenate([t[:, (k + 1) % 3] for k in range(3)])
    tid = np.tile(np.arange(nt), 3)
    kk = np.repeat(np.arange(3), nt)
    key = np.minimum(a, b) * (t.max() + 1) + np.maximum(a, b)
    o = np.lexsort((tid, key))
    p, q = o[0::2], o[1::2]
    return tid[p], tid[q], kk[p], kk[q]


def _flip_to_convex(v, tris, max_rounds=100):
    """Flip every edge whose fold is concave (the far vertex of one triangle
    strictly outside the other's plane, exact sign) until none is left. The
    vertices lie on a convex surface, so the flips converge to a triangulation
    of their convex hull; orientation is kept."""
    tris = tris.astype(np.int64).copy()
    for _ in range(max_rounds):
        t1, t2, k1, k2 = _edges(tris)
        far = tris[t2, (k2 + 2) % 3]
        bad = np.nonzero(_orient_sign(v[tris[t1, 0]], v[tris[t1, 1]], v[tris[t1, 2]], v[far]) < 0)[0]
        if bad.size == 0:
            return tris.astype(np.int32)
        t = tris.astype(np.int64)
        nv = int(t.max()) + 1
        present = set((np.minimum(t[:, [0, 1, 2]], t[:, [1, 2, 0]]) * nv +
                       np.maximum(t[:, [0, 1, 2]], t[:, [1, 2, 0]])).ravel().tolist())
        used = set()
        for e in bad:
            a, b = int(t1[e]), int(t2[e])
            if a in used or b in used:
                continue
            u, w_ = tris[a, k1[e]], tris[a, (k1[e] + 2) % 3]
            vv = tris[a, (k1[e] + 1) % 3]
            x = tris[b, (k2[e] + 2) % 3]
            if min(x, w_) * nv + max(x, w_) in present:
                continue
            tris[a] = (u, x, w_)
            tris[b] = (x, vv, w_)
            present.add(min(x, w_) * nv + max(x, w_))
            used.update((a, b))
    raise RuntimeError("edge flips did not converge")


def rounded_box(half, fillet, center, n_face: int) -> Surface:
    """Box with rounded edges and corners (fillet radius), from a cube-surface grid.

    Each point p of a uniform n_face x n_face grid on every face of the cube
    surface [-1,1]^3, scaled to the outer box, maps to c + fillet (p - c)/|p - c|,
    with c the closest point of the inner box (half - fillet): 12 n_face^2
    triangles. Each grid quad is split along the diagonal that makes its fold
    convex (the quad's fourth vertex not strictly outside the first triangle's
    plane, decided exactly), then any remaining concave fold across a quad edge
    is flipped, so that the mesh bounds a convex body exactly.
    """
    half = np.asarray(half, dtype=np.float64)
    inner = half - fillet
    t = np.linspace(-1.0, 1.0, n_face + 1)
    verts = {}
    vl = []
    quads = []

    def vid(p):
        key = tuple(np.round(p, 12))
        if key not in verts:
            verts[key] = len(vl)
            vl.append(p)
        return verts[key]

    for axis in range(3):
        for sgn in (-1.0, 1.0):
            u_ax, v_ax = [a for a in range(3) if a != axis]
            ids = np.empty((n_face + 1, n_face + 1), dtype=np.int64)
            for i in range(n_face + 1):
                for j in range(n_face + 1):
                    p = np.zeros(3)
                    p[axis] = sgn
                    p[u_ax] = t[i]
                    p[v_ax] = t[j]
                    ids[i, j] = vid(p)
            # (e_u x e_v) . e_axis is +1 for axes 0 and 2, -1 for axis 1: wind the
            # quads so that every face's normal points out of the box
            out = (1.0 if axis != 1 else -1.0) * sgn > 0
            for i in range(n_face):
                for j in range(n_face):
                    a, b, c, d = ids[i, j], ids[i + 1, j], ids[i, j + 1], ids[i + 1, j + 1]
                    quads.append((a, b, d, c) if out else (a, c, d, b))
    cube = np.array(vl)
    pts = cube * half
    cl = np.clip(pts, -inner, inner)
    dv = pts - cl
    nrm = np.linalg.norm(dv, axis=1, keepdims=True)
    nrm[nrm == 0] = 1.0
    v = cl + fillet * dv / nrm + np.asarray(center)
    # quad (p0, p1, p2, p3) in outward order: diagonal p0-p2 unless p3 lies
    # strictly outside the plane of (p0, p1, p2), then diagonal p1-p3
    q = np.array(quads, dtype=np.int64)
    concave = _orient_sign(v[q[:, 0]], v[q[:, 1]], v[q[:, 2]], v[q[:, 3]]) < 0
    tris = np.where(concave[:, None, None],
                    np.stack([q[:, [0, 1, 3]], q[:, [1, 2, 3]]], 1),
                    np.stack([q[:, [0, 1, 2]], q[:, [0, 2, 3]]], 1)).reshape(-1, 3)
    # folds across the quads' edges (where the grid meets the fillets)
    tris = _flip_to_convex(v, tris)
    s = Surface(v, np.array(tris, dtype=np.int32),
                {"kind": "rounded_box", "half": half.tolist(), "fillet": fillet,
                 "center": list(map(float, center))})
    orient_outward(s)
    return s


def merge_surfaces(parts) -> Surface:
    vs, ts, off = [], [], 0
    for p in parts:
        vs.append(p.verts)
        ts.append(p.tris.astype(np.int64) + off)
        off += p.verts.shape[0]
    return Surface(np.concatenate(vs), np.concatenate(ts).astype(np.int32),
                   {"kind": "union", "parts": [p.meta for p in parts]})


def signed_volume(s: Surface) -> float:
    a, b, c = (s.verts[s.tris[:, k]] for k in range(3))
    return float(np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0)


def orient_outward(s: Surface) -> None:
    """Flip all triangles if the enclosed signed volume is negative (in place)."""
    if signed_volume(s) < 0:
        s.tris[:] = s.tris[:, [0, 2, 1]]


def is_watertight(s: Surface) -> bool:
    """Every directed edge appears once and its reverse appears once."""
    t = s.tris.astype(np.int64)
    e = np.concatenate([t[:, [0, 1]], t[:, [1, 2]], t[:, [2, 0]]])
    nv = int(t.max()) + 1
    fwd = e[:, 0] * nv + e[:, 1]
    rev = e[:, 1] * nv + e[:, 0]
    if np.unique(fwd).shape[0] != fwd.shape[0]:
        return False
    return bool(np.isin(rev, fwd).all())


# ---------------------------------------------------------------------------
# Nodal fields: sum of four random Fourier modes, pressure ~ U(-1, 1)
# ---------------------------------------------------------------------------


def _modes(rng):
    k = rng.integers(1, 4, size=(4, 3))
    a = rng.normal(size=(4, 3))
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    phi = rng.uniform(0.0, 2 * np.pi, size=4)
    return k, a, phi


def fourier_velocity(xyz_hat, k, a, phi):
    arg = 2 * np.pi * (xyz_hat @ k.T) + phi          # (n, 4)
    return np.sin(arg) @ a                             # (n, 3)


def make_fields(node_xyz: np.ndarray, seed: int, shortest_side: float = 1.0) -> dict:
    """Seeded nodal fields at the given node coordinates (n, 3), float64 SoA.

    Draw order per seed: mode wavenumbers k in {1,2,3}^3 (4x3), unit amplitudes,
    phases U[0, 2pi), nodal p ~ U(-1, 1). The previous-step velocity uses the same
    recipe with seed + 10000.
    """
    xh = np.asarray(node_xyz, dtype=np.float64) / shortest_side
    n = xh.shape[0]
    rng = np.random.default_rng(seed)
    k, a, phi = _modes(rng)
    p = rng.uniform(-1.0, 1.0, size=n)
    u = fourier_velocity(xh, k, a, phi)
    rng0 = np.random.default_rng(seed + 10000)
    k0, a0, phi0 = _modes(rng0)
    u0 = fourier_velocity(xh, k0, a0, phi0)
    c = np.ascontiguousarray
    return {"ux": c(u[:, 0]), "uy": c(u[:, 1]), "uz": c(u[:, 2]), "p": c(p),
            "ux0": c(u0[:, 0]), "uy0": c(u0[:, 1]), "uz0": c(u0[:, 2])}


FIELD_NAMES = ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")

# Physical parameters shared by every workload (rho, mu, dt, theta, C_t, C_I)
DEFAULT_PARAMS = dict(rho=1.0, mu=0.01, dt=0.01, theta=0.5, c_t=4.0, c_i=36.0)

# Non-dyadic offset of the immersed bodies, so that no grid line or sub-cell
# Gauss point coordinate coincides with a surface vertex plane.
BODY_OFFSET = (1e-6 * math.pi, 1e-6 * math.e, 1e-6 * math.sqrt(2.0))


def sphere_workload(lmin=5, lmax=8, beta=4.0, subdiv=4, r=0.1):
    """Immersed sphere at the cube centre (plus a non-dyadic offset)."""
    c = tuple(0.5 + o for o in BODY_OFFSET)
    tree = sphere_refined_octree(c, r, lmin, lmax, beta)
    surf = icosphere(subdiv, r, c)
    return tree, surf


def box_surface(lo, hi) -> Surface:
    """Axis-aligned box as 12 outward triangles."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    v = np.array([[hi[0] if c & 1 else lo[0], hi[1] if c & 2 else lo[1], hi[2] if c & 4 else lo[2]]
                  for c in range(8)])
    quads = [(0, 2, 6, 4), (1, 5, 7, 3), (0, 4, 5, 1), (2, 3, 7, 6), (0, 1, 3, 2), (4, 6, 7, 5)]
    t = []
    for a, b, c, d in quads:
        t += [[a, b, c], [a, c, d]]
    s = Surface(v, np.array(t, np.int32), {"kind": "box", "lo": lo.tolist(), "hi": hi.tolist()})
    orient_outward(s)
    return s


def sdf_sample_points(surf: Surface, lo, hi, n: int, seed: int, near_frac: float = 0.7,
                      near_dist: float = 0.1):
    """Training positions for the signed-distance network: a fraction near the
    surface (area-weighted random surface point, offset along the triangle
    normal by U(-near_dist, near_dist)), the rest uniform in the box."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    n_near = int(round(near_frac * n))
    a, b, c = (surf.verts[surf.tris[:, k]] for k in range(3))
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1)
    t = rng.choice(surf.n_tri, n_near, p=area / area.sum())
    r1, r2 = rng.uniform(size=(2, n_near))
    s = np.sqrt(r1)
    pts = (1 - s)[:, None] * a[t] + (s * (1 - r2))[:, None] * b[t] + (s * r2)[:, None] * c[t]
    nrm = cr[t] / np.linalg.norm(cr[t], axis=1, keepdims=True)
    pts = pts + nrm * rng.uniform(-near_dist, near_dist, n_near)[:, None]
    uni = rng.uniform(lo, hi, (n - n_near, 3))
    out = np.concatenate([pts, uni])
    out = np.clip(out, lo, hi)
    return out[rng.permutation(n)]


def ellipsoid_refined_octree(center, semi, rot, lmin, lmax, beta, balance=True) -> Octree:
    """Refine octants whose centre lies within about beta*h of the ellipsoid
    surface (distance estimated as |r - 1| * min(semi), r the normalised radius)."""
    c = np.asarray(center, np.float64)
    a = np.asarray(semi, np.float64)
    R = np.asarray(rot, np.float64)

    def refine(cx, cy, cz, h, lev):
        y = (np.stack([cx, cy, cz], 1) - c) @ R      # body frame
        r = np.sqrt(((y / a) ** 2).sum(1))
        return (np.abs(r - 1.0) * a.min() < beta * h) & (lev < lmax)

    return refined_octree(lmax, lmin, refine, balance=balance,
                          meta={"body": "ellipsoid", "beta": beta, "lmin": lmin, "lmax": lmax})


def _batch_tree(arg):
    target, semi, R, c, ntri, lmin = arg
    n_lat = max(3, int(round(np.sqrt(ntri / 4.0))))
    surf = ellipsoid(semi, c, R, n_lat, 2 * n_lat)
    # the band count at beta = 1 grows about 4x per level
    l_ref = lmin + 2
    n_ref = ellipsoid_refined_octree(c, semi, R, lmin, l_ref, 1.0).n
    lmax = int(np.clip(np.round(l_ref + np.log(target / n_ref) / np.log(4.0)), lmin + 1, 11))
    beta = float(np.clip(target / (n_ref * 4.0 ** (lmax - l_ref)), 0.25, 8.0))
    tree = None
    for _ in range(8):
        tree = ellipsoid_refined_octree(c, semi, R, lmin, lmax, beta)
        if abs(tree.n - target) <= 0.1 * target:
            break
        beta = float(np.clip(beta * (target / tree.n), 0.05, 32.0))
    tree.meta["target"] = target
    return tree, surf


def batch_workload(n_trees: int, seed: int, size_lo=1e4, size_hi=5e5, lmin=4, tri_lo=2000,
                   tri_hi=20000, workers=None):
    """Independent octrees of log-uniform target sizes, each refined around its own
    ellipsoid (semi-axes U(0.05, 0.2), random rotation, centre U(0.25, 0.75)^3,
    lat-long tessellation with U(tri_lo, tri_hi) triangles).

    Each tree gets the finest level whose refinement band of about one cell
    (beta = 1) holds the target leaf count most closely, then beta is adjusted
    (the count grows about linearly in beta) until the 2:1-balanced tree is
    within 10% of the target. All random draws happen first, in tree order, so
    the result does not depend on the number of worker processes (workers > 1
    starts a spawn-context pool: the calling script needs a main guard)."""
    rng = np.random.default_rng(seed)
    args = []
    for _ in range(n_trees):
        target = float(np.exp(rng.uniform(np.log(size_lo), np.log(size_hi))))
        semi = rng.uniform(0.05, 0.2, 3)
        R = random_rotation(rng)
        c = rng.uniform(0.25, 0.75, 3)
        ntri = int(rng.integers(tri_lo, tri_hi + 1))
        args.append((target, semi, R, c, ntri, lmin))
    workers = min(workers or 1, n_trees)
    if workers <= 1:
        return [_batch_tree(a) for a in args]
    import multiprocessing as mp
    with mp.get_context("spawn").Pool(workers) as pool:
        return pool.map(_batch_tree, args, chunksize=1)


def two_boxes(n_face: int, domain=(8.0, 2.0, 2.0)):
    """Two bluff boxes 1.0 x 0.25 x 0.3 with 0.03 fillets, one behind the other
    along x with a gap of 0.5, centred in y and z of an 8 x 2 x 2 domain (plus
    the non-dyadic offset); 24 n_face^2 triangles."""
    half = (0.5, 0.125, 0.15)
    c0 = np.array([3.0, domain[1] / 2, domain[2] / 2]) + np.asarray(BODY_OFFSET)
    c1 = c0 + np.array([1.0 + 0.5, 0.0, 0.0])
    return merge_surfaces([rounded_box(half, 0.03, c0, n_face), rounded_box(half, 0.03, c1, n_face)])



def rounded_box_distance(p, half, fillet, center):
    """Signed distance of points (n, 3) to a box with rounded edges and corners
    (negative inside): the inner box (half - fillet) grown by the fillet radius."""
    q = np.abs(np.asarray(p, np.float64) - np.asarray(center)) - (np.asarray(half) - fillet)
    outside = np.linalg.norm(np.maximum(q, 0.0), axis=1)
    inside = np.minimum(q.max(axis=1), 0.0)
    return outside + inside - fillet


def two_box_workload(lmin=6, lmax=11, beta=13.0, n_face=91, domain=(8.0, 2.0, 2.0)):
    """Two filleted bluff boxes (two_boxes) in an 8 x 2 x 2 domain, refined at
    their surfaces from level lmin to lmax.

    The octree root is the cube of side 8 that holds the domain; its leaves
    cover only [0, 8) x [0, 2) x [0, 2) (the domain is a quarter of the root
    in y and in z). Octants whose centre lies within beta*h of either box
    surface are split, which at the default beta gives about 10^7 octants."""
    assert domain[0] == 4 * domain[1] and domain[1] == domain[2]
    M = lmax
    half = (0.5, 0.125, 0.15)
    c0 = np.array([3.0, domain[1] / 2, domain[2] / 2]) + np.asarray(BODY_OFFSET)
    c1 = c0 + np.array([1.5, 0.0, 0.0])

    def refine(cx, cy, cz, h, lev):
        p = np.stack([cx, cy, cz], 1)
        d = np.minimum(np.abs(rounded_box_distance(p, half, 0.03, c0)),
                       np.abs(rounded_box_distance(p, half, 0.03, c1)))
        return (d < beta * h) & (lev < M)

    full = 1 << M
    tree = refined_octree(M, lmin, refine, ext=(full, full >> 2, full >> 2), root_len=domain[0],
                          meta={"body": "two_boxes", "beta": beta, "lmin": lmin, "lmax": lmax})
    return tree, two_boxes(n_face, domain)
