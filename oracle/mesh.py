"""Mesh derivation of the CPU reference (TEST INFRASTRUCTURE ONLY).

Plain numpy, written from the paper's description of octree meshing:

* Vertices are the corners of the leaves. A vertex that lies in the interior of
  an edge or a face of some leaf is *hanging*: it is not an independent degree
  of freedom but the linear combination of the larger edge's two end points
  (weights 1/2) or the larger face's four corners (weights 1/4). This is the
  correction operator M_e of Alg. 3, with I1d = [1/2 1/2] and I2d = I1d (x) I1d
  (Section "Matrix Assembly on Distributed Octrees", hanging-node paragraph and
  its figure).
* With 2:1 balance across faces, edges and vertices, only the midpoint of a
  leaf's edge or the centre of a leaf's face can be another leaf's corner, and
  a master is never itself hanging (asserted).
* Independent nodes are numbered by the Morton key of their integer
  coordinates (x in the lowest bit); dof = 4*node + c with c in (ux, uy, uz, p).
* The CSR pattern holds full 4x4 blocks for every node pair coupled by a non-IN
  element after constraint expansion, plus every node's diagonal block.
"""
from __future__ import annotations

import numpy as np

MORTON_BITS = 21   # per axis; 3 x 21 bits fit a uint64 key

# corner c of a leaf: offset ((c>>0)&1, (c>>1)&1, (c>>2)&1) times the side
CORNER_OFF = np.array([[(c >> 0) & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], dtype=np.int64)
# the 12 edges: (corner a, corner b) with b = a + unit step along one axis
EDGES = [(a, a | (1 << k)) for k in range(3) for a in range(8) if not (a >> k) & 1]
# the 6 faces: the four corners with bit k equal to s
FACES = [[c for c in range(8) if ((c >> k) & 1) == s] for k in range(3) for s in (0, 1)]


class Mesh:
    pass


def _vertices_and_hanging(ax, ay, az, level, max_level):
    """Corner keys of every leaf, the unique vertex keys, and the hanging
    vertices (key, up to 4 master keys, weights)."""
    M = int(max_level)
    ax = np.asarray(ax, np.int64); ay = np.asarray(ay, np.int64); az = np.asarray(az, np.int64)
    lev = np.asarray(level, np.int64)
    side = np.int64(1) << (M - lev)
    anc = np.stack([ax, ay, az], 1)
    corners = anc[:, None, :] + CORNER_OFF[None, :, :] * side[:, None, None]   # (E, 8, 3)
    ckey = morton_key(corners[..., 0], corners[..., 1], corners[..., 2])     # (E, 8)
    all_keys, inv = np.unique(ckey.ravel(), return_inverse=True)
    pos_of_key = lambda k: np.searchsorted(all_keys, k)
    in_set = lambda k: (pos_of_key(k) < all_keys.size) & (all_keys[np.minimum(pos_of_key(k), all_keys.size - 1)] == k)

    # --- hanging vertices: edge midpoints / face centres that are corners ---
    hang_key, hang_masters, hang_w = [], [], []
    big = side >= 2
    for (a, b) in EDGES:
        mid = (corners[big, a] + corners[big, b]) // 2
        k = morton_key(mid[:, 0], mid[:, 1], mid[:, 2])
        hit = in_set(k)
        hang_key.append(k[hit])
        m = np.stack([ckey[big, a][hit], ckey[big, b][hit],
                      np.full(hit.sum(), -1, np.int64).astype(np.uint64),
                      np.full(hit.sum(), -1, np.int64).astype(np.uint64)], 1)
        hang_masters.append(m)
        hang_w.append(np.tile([0.5, 0.5, 0.0, 0.0], (hit.sum(), 1)))
    for f in FACES:
        cen = (corners[big, f[0]] + corners[big, f[3]]) // 2
        k = morton_key(cen[:, 0], cen[:, 1], cen[:, 2])
        hit = in_set(k)
        hang_key.append(k[hit])
        hang_masters.append(np.stack([ckey[big, c][hit] for c in f], 1))
        hang_w.append(np.tile([0.25, 0.25, 0.25, 0.25], (hit.sum(), 1)))
    hang_key = np.concatenate(hang_key)
    hang_masters = np.concatenate(hang_masters)
    hang_w = np.concatenate(hang_w)
    # the same hanging vertex is found from every coarse leaf sharing the edge/face
    hk, first = np.unique(hang_key, return_index=True)
    hang_masters, hang_w = hang_masters[first], hang_w[first]
    # masters must be independent (requires vertex balance)
    mk = hang_masters[hang_w > 0]
    if np.isin(mk, hk).any():
        raise ValueError("chained hanging constraint: tree is not 2:1 balanced")
    return ckey, all_keys, inv, hk, hang_masters, hang_w


def independent_node_keys(ax, ay, az, level, max_level):
    """Morton keys of the independent nodes of a tree, ascending: position k
    of a key is that node's number (the numbering of the CSR rows)."""
    _, all_keys, _, hk, _, _ = _vertices_and_hanging(ax, ay, az, level, max_level)
    return all_keys[~np.isin(all_keys, hk)]


def derive_mesh(ax, ay, az, level, max_level, active=None):
    """Node table, hanging constraints, per-element masters and CSR pattern.

    active: optional bool mask of elements that contribute (non-IN); the
    pattern couples masters of active elements only.
    """
    E = np.asarray(ax).shape[0]
    ckey, all_keys, inv, hk, hang_masters, hang_w = _vertices_and_hanging(ax, ay, az, level, max_level)

    # --- independent nodes, Morton order ---
    is_hang = np.isin(all_keys, hk)
    node_keys = all_keys[~is_hang]
    n_nodes = node_keys.size
    node_id = lambda k: np.searchsorted(node_keys, k)

    # --- per vertex: up to 4 (node, weight) ---
    vm = np.full((all_keys.size, 4), -1, np.int64)
    vw = np.zeros((all_keys.size, 4))
    reg = np.nonzero(~is_hang)[0]
    vm[reg, 0] = node_id(all_keys[reg])
    vw[reg, 0] = 1.0
    hpos = np.searchsorted(all_keys, hk)
    for j in range(4):
        ok = hang_w[:, j] > 0
        vm[hpos[ok], j] = node_id(hang_masters[ok, j])
        vw[hpos[ok], j] = hang_w[ok, j]

    # --- per element: vertex -> (master, weight), master set (sorted) ---
    ev = inv.reshape(E, 8)
    em = vm[ev]          # (E, 8, 4)
    ew = vw[ev]
    flat = np.where(em >= 0, em, np.iinfo(np.int64).max).reshape(E, 32)
    flat.sort(axis=1)
    dup = np.zeros_like(flat, dtype=bool)
    dup[:, 1:] = flat[:, 1:] == flat[:, :-1]
    flat[dup] = np.iinfo(np.int64).max
    flat.sort(axis=1)
    nm = (flat != np.iinfo(np.int64).max).sum(1)
    if nm.max() > 8:
        raise ValueError("element with more than 8 distinct masters")
    masters = np.where(flat[:, :8] == np.iinfo(np.int64).max, -1, flat[:, :8]).astype(np.int64)
    # C[e, a, s] = weight of master s in vertex a
    C = np.zeros((E, 8, 8))
    for a in range(8):
        for j in range(4):
            m = em[:, a, j]
            ok = m >= 0
            # slot of m within the element's (sorted) master list
            s = (masters[ok] < m[ok, None]).sum(1)
            C[np.nonzero(ok)[0], a, s] += ew[ok, a, j]

    # --- CSR pattern ---
    act = np.ones(E, bool) if active is None else np.asarray(active, bool)
    mm = masters[act]
    pi = np.repeat(mm, 8, axis=1)
    pj = np.tile(mm, (1, 8))
    ok = (pi >= 0) & (pj >= 0)
    pairs = pi[ok] * n_nodes + pj[ok]
    diag = np.arange(n_nodes, dtype=np.int64) * (n_nodes + 1)
    pairs = np.unique(np.concatenate([pairs, diag]))
    prow = pairs // n_nodes
    pcol = pairs % n_nodes
    nrow_ptr = np.zeros(n_nodes + 1, np.int64)
    np.add.at(nrow_ptr, prow + 1, 1)
    nrow_ptr = np.cumsum(nrow_ptr)
    deg = np.diff(nrow_ptr)
    # dof rows: 4 per node, each with 4*deg entries (columns 4*n + j, ascending)
    row_len = np.repeat(4 * deg, 4)
    row_ptr = np.zeros(4 * n_nodes + 1, np.int64)
    row_ptr[1:] = np.cumsum(row_len)
    cols_node = np.repeat(pcol, 4) * 4 + np.tile(np.arange(4), pcol.size)   # per node row
    col_idx = np.empty(row_ptr[-1], np.int32)
    for c in range(4):
        # dof row 4*m + c repeats the node row's column list
        for_m = np.arange(n_nodes)
        start = row_ptr[4 * for_m + c]
        lens = 4 * deg
        seg = np.repeat(start - 4 * nrow_ptr[:-1], lens) + np.arange(cols_node.size)
        col_idx[seg] = cols_node
    # active nodes: masters of at least one active element
    node_active = np.zeros(n_nodes, bool)
    node_active[mm[mm >= 0]] = True

    ms = Mesh()
    ms.n_nodes = n_nodes
    ms.node_keys = node_keys
    ms.node_xyz_int = _decode(node_keys)
    ms.n_hanging = int(hk.size)
    ms.masters = masters.astype(np.int32)
    ms.nm = nm.astype(np.int32)
    ms.C = C
    ms.row_ptr = row_ptr
    ms.col_idx = col_idx
    ms.nnz = int(row_ptr[-1])
    ms.node_active = node_active
    ms.vertex_keys = all_keys
    ms.elem_vertex = ev
    ms.vertex_is_hanging = is_hang
    return ms


def _spread_table():
    """T[v] for 7-bit v: bit b of v moved to bit 3b, written bit by bit."""
    t = np.zeros(128, np.uint64)
    for v in range(128):
        k = 0
        for b in range(7):
            k |= ((v >> b) & 1) << (3 * b)
        t[v] = k
    return t


_SPREAD = _spread_table()


def morton_key(x, y, z):
    """Morton key of integer coordinates, x in the lowest bit.

    Bit b of x goes to key bit 3b, of y to 3b+1, of z to 3b+2 (the
    node-numbering convention of the CSR), seven bits at a time through a
    table that is itself written bit by bit.
    """
    x = np.asarray(x, np.int64); y = np.asarray(y, np.int64); z = np.asarray(z, np.int64)
    if x.size and (min(x.min(), y.min(), z.min()) < 0 or
                   max(x.max(), y.max(), z.max()) >= (1 << MORTON_BITS)):
        raise ValueError("coordinate outside the 21-bit Morton range")
    key = np.zeros(np.broadcast(x, y, z).shape, np.uint64)
    for c in range(MORTON_BITS // 7):
        for axis, v in enumerate((x, y, z)):
            key |= _SPREAD[(v >> (7 * c)) & 127] << np.uint64(21 * c + axis)
    return key


def _decode(keys):
    """Inverse of morton_key: integer (x, y, z) of each key, bit by bit."""
    k = np.asarray(keys, np.uint64)
    out = np.zeros(k.shape + (3,), np.int64)
    for b in range(MORTON_BITS):
        for axis in range(3):
            bit = ((k >> np.uint64(3 * b + axis)) & np.uint64(1)).astype(np.int64)
            out[..., axis] |= bit << b
    return out
