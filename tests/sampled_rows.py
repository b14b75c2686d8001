"""Rows of a full-size problem from the CPU reference, one window at a time.

At sizes where the reference cannot derive the whole CSR pattern in a test's
time (10^7 octants, more than 2^31 nonzeros), a sample of node rows is checked
instead. For every sampled node the reference

* numbers the nodes globally (independent node keys of the whole tree, its
  own hanging-vertex detection),
* takes the leaves around the node (every leaf that can hold the node as a
  master, and enough of their neighbours for their hanging vertices to be
  found), derives that local mesh, labels its corners against the full
  surface, runs the adaptive quadrature of its INTERCEPTED elements and
  assembles the elements that have the node as a master,
* and returns the node's four rows: global column indices, values, residual.

Only the choice of which nodes to sample may look at the library's exports;
every expected value comes from the reference.
"""
from __future__ import annotations

import numpy as np

from oracle import window as W


def reference_rows(O, tree, surf, fields, node_keys, nodes, depth=3, prm=None, log=None):
    """The reference's rows of the given global nodes.

    node_keys: the reference's global independent node keys (ascending).
    fields: global nodal fields (arrays over node_keys' order).
    Returns {node: dict(active, cols[4], vals[4], resid[4])}."""
    from oracle import mesh as OM
    index = W.LeafIndex(tree)
    pos_all = OM._decode(node_keys[np.asarray(nodes)])
    sel = set()
    for pos in pos_all:
        _, win = W.node_window(index, pos)
        sel.update(win.tolist())
    sub = W.subset(tree, np.array(sorted(sel), np.int64))
    ms0 = O.derive_mesh(sub.ax, sub.ay, sub.az, sub.level, sub.max_level)
    if surf is not None:
        mk, _, nd = O.markers(sub, ms0, surf)
        assert nd == 0
    else:
        mk = np.zeros(sub.n, np.uint8)
    ms = O.derive_mesh(sub.ax, sub.ay, sub.az, sub.level, sub.max_level, active=mk != O.IN)
    gid = np.searchsorted(node_keys, ms.node_keys)
    found = (gid < node_keys.size) & (node_keys[np.minimum(gid, node_keys.size - 1)] == ms.node_keys)
    gid = np.where(found, gid, -1)
    # elements (local ids) with a sampled node as a master
    loc_of = {int(g): i for i, g in enumerate(gid) if g >= 0}
    want = np.array([loc_of[int(n)] for n in nodes], np.int64)
    has = np.isin(ms.masters, want).any(1)
    els = np.nonzero(has & (mk != O.IN))[0]
    m_used = ms.masters[els]
    assert (gid[m_used[m_used >= 0]] >= 0).all(), "a master of an assembled element is unnumbered"
    f = {}
    for k in ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0"):
        a = np.zeros(ms.n_nodes)
        a[found] = np.asarray(fields[k])[gid[found]]
        f[k] = a
    cut = els[mk[els] == O.INTERCEPTED]
    sq = O.subquad(sub, surf, cut, depth) if cut.size else None
    if log:
        log(f"reference window: {sub.n} leaves, {els.size} elements assembled "
            f"({cut.size} INTERCEPTED, {0 if sq is None else sq['el'].size} sub-cell points)")
    V, R = O.assemble(sub, ms, f, prm=prm, mk=mk, sub=sq, depth=depth, subset=els)
    out = {}
    for n, ln in zip(nodes, want):
        rows = {"active": bool(ms.node_active[ln]), "cols": [], "vals": [], "resid": []}
        for c in range(4):
            r = 4 * ln + c
            cl = ms.col_idx[ms.row_ptr[r]:ms.row_ptr[r + 1]].astype(np.int64)
            cg = 4 * gid[cl // 4] + cl % 4
            assert (gid[cl // 4] >= 0).all()
            v = V[ms.row_ptr[r]:ms.row_ptr[r + 1]].copy()
            if not rows["active"]:
                # a node of no non-IN element: identity row (diagonal block only)
                cg = 4 * int(n) + np.arange(4)
                v = (cg == 4 * int(n) + c).astype(np.float64)
            rows["cols"].append(cg)
            rows["vals"].append(v)
            rows["resid"].append(0.0 if not rows["active"] else float(R[r]))
        out[int(n)] = rows
    return out


def compare_rows(ref, rp, nrp, ncol, vals_dev, resid_dev, tol=1e-12):
    """Library rows (row_ptr rp, node-level pattern nrp/ncol, device values and
    residual) against the reference rows. Columns bit-exact; values entrywise
    within tol of the row's 1-norm and normwise within tol over the sample;
    residual normwise within tol over the sample. Returns (value error, residual
    error, largest CSR offset checked)."""
    import torch
    dv2 = rv2 = dr2 = rr2 = 0.0
    off_max = 0
    for n, rows in ref.items():
        bc = ncol[nrp[n]:nrp[n + 1]].astype(np.int64)
        cols = (4 * bc[:, None] + np.arange(4)).ravel()
        for c in range(4):
            r = 4 * n + c
            a, b = int(rp[r]), int(rp[r + 1])
            off_max = max(off_max, b)
            assert b - a == rows["cols"][c].size, (n, c, b - a, rows["cols"][c].size)
            assert np.array_equal(cols, rows["cols"][c]), (n, c)
            g = vals_dev[a:b].double().cpu().numpy()
            v = rows["vals"][c]
            assert np.all(np.abs(g - v) <= tol * max(np.abs(v).sum(), 1e-300)), (n, c)
            dv2 += float(((g - v) ** 2).sum())
            rv2 += float((v ** 2).sum())
            if resid_dev is not None:
                x = float(resid_dev[r].item())
                dr2 += (x - rows["resid"][c]) ** 2
                rr2 += rows["resid"][c] ** 2
    ev = (dv2 / rv2) ** 0.5
    er = (dr2 / rr2) ** 0.5 if rr2 > 0 else 0.0
    assert ev <= tol and er <= tol, (ev, er)
    return ev, er, off_max
