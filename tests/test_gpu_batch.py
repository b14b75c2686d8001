"""Batched form: many independent octrees in one persistent launch (device work
queue), autotuned tile / workgroups per CU, and HIP-graph replay. Each tree's
output must equal its own single-context assembly (itself checked against the
CPU reference), and one tree is checked against the reference directly.
Matrix norms are taken over the rows of active nodes; identity rows of
inactive nodes must match exactly."""
import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_00706_amd import vms
    vms.lib()
    return torch, vms


def build(torch, vms, prec, n_trees=5, seed=1003):
    work = I.batch_workload(n_trees, seed, size_lo=2e3, size_hi=3e4, lmin=3)
    stream = torch.cuda.Stream()
    ctxs, fields, vals, resid, trees = [], [], [], [], []
    with torch.cuda.stream(stream):
        for k, (tree, surf) in enumerate(work):
            ctx = vms.vms_create(tree, surf, vms.make_params(quad_depth=3, precision=prec),
                                 stream.cuda_stream)
            sz = vms.vms_sizes(ctx)
            xyz = vms.vms_export(ctx, vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64) / \
                float(1 << tree.max_level) * tree.root_len + np.asarray(tree.origin)
            f = I.make_fields(xyz, 2000 + k)
            fields.append({n: torch.as_tensor(f[n], device="cuda") for n in f})
            dt = torch.float64 if prec == vms.VMS_FP64 else torch.float32
            vals.append(torch.zeros(sz["nnz"], dtype=dt, device="cuda"))
            resid.append(torch.zeros(sz["n_rows"], dtype=torch.float64, device="cuda"))
            ctxs.append(ctx)
            trees.append((tree, surf, f))
    masks = [active_entries(vms, c, t.n) for c, (t, _, _) in zip(ctxs, trees)]
    return stream, ctxs, fields, vals, resid, trees, masks


def active_entries(vms, ctx, n_oct):
    """Mask of the CSR entries in rows of active nodes (nodes of non-IN elements)."""
    mk = vms.vms_export(ctx, vms.VMS_EXPORT_MARKERS, n_oct)
    ma = vms.vms_export(ctx, vms.VMS_EXPORT_MASTERS, n_oct)[mk != 1]
    act = np.zeros(vms.vms_sizes(ctx)["n_nodes"], bool)
    act[ma[ma >= 0]] = True
    rp = vms.vms_export(ctx, vms.VMS_EXPORT_ROW_PTR)
    return np.repeat(np.repeat(act, 4), np.diff(rp))


def singles(torch, vms, stream, ctxs, fields, vals, resid):
    out = []
    with torch.cuda.stream(stream):
        for c, f, v, r in zip(ctxs, fields, vals, resid):
            vms.vms_assemble(c, f, v, r)
            stream.synchronize()
            out.append((v.cpu().numpy().astype(np.float64).copy(), r.cpu().numpy().copy()))
    return out


def close(a, b, tol):
    return np.linalg.norm(a - b) <= tol * max(np.linalg.norm(b), 1e-300)


def close_mat(a, b, m, tol):
    return np.array_equal(a[~m], b[~m]) and close(a[m], b[m], tol)


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 1e-6)])
def test_batch_equals_single_contexts(env, prec, tol):
    torch, vms = env
    stream, ctxs, fields, vals, resid, _, masks = build(torch, vms, prec)
    ref = singles(torch, vms, stream, ctxs, fields, vals, resid)
    with torch.cuda.stream(stream):
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        for tile, gpc in ((1, 4), (4, 8), (16, 32)):
            vms.vms_batch_set_config(b, tile, gpc)
            vms.vms_batch_assemble(b, fields, vals, resid)
            stream.synchronize()
            for (rv, rr), v, r, m in zip(ref, vals, resid, masks):
                assert close_mat(v.cpu().numpy().astype(np.float64), rv, m, tol)
                assert close(r.cpu().numpy(), rr, tol)
        ms = vms.vms_batch_autotune(b, fields, vals, resid)
        cfg = vms.vms_batch_get_config(b)
        print(f"precision {prec}: autotuned {cfg}, {ms:.3f} ms")
        vms.vms_batch_destroy(b)
    for c in ctxs:
        vms.vms_destroy(c)


def test_batch_graph_replays(env):
    """Captured graph replayed several times, with eager work and synchronisation in
    between; every replay must equal the eager batched result."""
    torch, vms = env
    stream, ctxs, fields, vals, resid, _, masks = build(torch, vms, 1, n_trees=4, seed=7)
    with torch.cuda.stream(stream):
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        eager = [(v.cpu().numpy().copy(), r.cpu().numpy().copy()) for v, r in zip(vals, resid)]
        vms.vms_batch_use_graph(b, True)
        for rep in range(4):
            for v in vals:
                v.fill_(123.0)          # eager work between replays
            stream.synchronize()
            vms.vms_batch_assemble(b, fields, vals, resid)
            stream.synchronize()
            for (ev, er), v, r, m in zip(eager, vals, resid, masks):
                assert close_mat(v.cpu().numpy().astype(np.float64), ev.astype(np.float64), m, 1e-6)
                assert close(r.cpu().numpy(), er, 1e-6)
        vms.vms_batch_destroy(b)
    for c in ctxs:
        vms.vms_destroy(c)


def test_batch_refuses_weak_bc_switched_on_later(env):
    """Weak boundary terms switched on for a context after it joined a batch:
    the batch refuses to assemble (before any launch); switched off again, the
    rebuilt records are re-read and the (graph-replayed) batch equals the single
    assemblies."""
    torch, vms = env
    stream, ctxs, fields, vals, resid, _, masks = build(torch, vms, 0, n_trees=3, seed=5)
    with torch.cuda.stream(stream):
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        vms.vms_batch_use_graph(b, True)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        vms.vms_set_weak_bc(ctxs[1], True, 4.0, (0.0, 0.0, 0.0))
        with pytest.raises(vms.VmsError) as e:
            vms.vms_batch_assemble(b, fields, vals, resid)
        assert e.value.code == vms.VMS_EUNSUPPORTED
        vms.vms_set_weak_bc(ctxs[1], False, 0.0, (0.0, 0.0, 0.0))
        for v in vals:
            v.fill_(7.0)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        got = [(v.cpu().numpy().copy(), r.cpu().numpy().copy()) for v, r in zip(vals, resid)]
        vms.vms_batch_destroy(b)
    ref = singles(torch, vms, stream, ctxs, fields, vals, resid)
    for (rv, rr), (gv, gr), m in zip(ref, got, masks):
        assert close_mat(gv, rv, m, 1e-13) and close(gr, rr, 1e-13)
    for c in ctxs:
        vms.vms_destroy(c)


def test_batch_tree_against_reference(env, oracle):
    torch, vms = env
    stream, ctxs, fields, vals, resid, trees, masks = build(torch, vms, 0, n_trees=3, seed=11)
    with torch.cuda.stream(stream):
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        vms.vms_batch_destroy(b)
    k = int(np.argmin([t.n for t, _, _ in trees]))
    tree, surf, f = trees[k]
    O = oracle
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    mk, _, _ = O.markers(tree, ms, surf)
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level, active=mk != O.IN)
    sub = O.subquad(tree, surf, np.nonzero(mk == O.INTERCEPTED)[0], 3)
    # the tree's fields are those of the reference's node positions
    assert np.array_equal(vms.vms_export(ctxs[k], vms.VMS_EXPORT_NODE_XYZ).T, ms.node_xyz_int)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << tree.max_level) * tree.root_len
    f_ref = I.make_fields(xyz + np.asarray(tree.origin), 2000 + k)
    assert all(np.array_equal(f_ref[n], f[n]) for n in f)
    V, R = O.assemble(tree, ms, f_ref, mk=mk, sub=sub, depth=3)
    v = vals[k].cpu().numpy()
    r = resid[k].cpu().numpy()
    act = np.repeat(np.repeat(ms.node_active, 4), np.diff(ms.row_ptr))
    assert np.array_equal(act, masks[k])
    assert close_mat(v, V, act, 1e-12)
    assert np.linalg.norm(r - R) <= 1e-12 * np.linalg.norm(R)
    for c in ctxs:
        vms.vms_destroy(c)


@pytest.mark.timeout(900)
def test_batch_full_size(env, oracle):
    """The 64-tree workload at full size (log-uniform 1e4..5e5 octants, seed
    1003), BF16x3, autotuned and replayed as a graph (the benchmark's launch):
    every tree's values and residual equal its single-context assembly bit for
    bit;
    the fixed queue order gives the same outputs bit for bit as the eq. (Wpart)
    order; sampled rows of the largest tree match the CPU reference within the
    mixed form's bar; a constant state gives a zero residual in every tree."""
    import os
    import time
    import sampled_rows as SR
    torch, vms = env
    t0 = time.perf_counter()
    work = I.batch_workload(64, 1003, workers=min(16, os.cpu_count() or 1))
    print(f"64 trees, {sum(t.n for t, _ in work)} octants ({time.perf_counter() - t0:.1f} s)", flush=True)
    big = int(np.argmax([t.n for t, _ in work]))
    stream = torch.cuda.Stream()
    ctxs, fields, vals, resid, ident, host_f = [], [], [], [], [], []
    with torch.cuda.stream(stream):
        for k, (tree, surf) in enumerate(work):
            ctx = vms.vms_create(tree, surf, vms.make_params(quad_depth=3, precision=vms.VMS_MIXED_BF16),
                                 stream.cuda_stream)
            sz = vms.vms_sizes(ctx)
            xyz = vms.vms_export(ctx, vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64) / \
                float(1 << tree.max_level) * tree.root_len + np.asarray(tree.origin)
            f = I.make_fields(xyz, 3000 + k)
            if k == big:
                host_f = f
            fields.append({n: torch.as_tensor(f[n], device="cuda") for n in f})
            vals.append(torch.zeros(sz["nnz"], dtype=torch.float32, device="cuda"))
            resid.append(torch.zeros(sz["n_rows"], dtype=torch.float64, device="cuda"))
            # CSR places of the rows of inactive nodes (one diagonal block each)
            mk = vms.vms_export(ctx, vms.VMS_EXPORT_MARKERS, tree.n)
            ma = vms.vms_export(ctx, vms.VMS_EXPORT_MASTERS, tree.n)[mk != 1]
            act = np.zeros(sz["n_nodes"], bool)
            act[ma[ma >= 0]] = True
            rp = vms.vms_export(ctx, vms.VMS_EXPORT_ROW_PTR)
            first = rp[4 * np.nonzero(~act)[0]]
            ident.append(torch.as_tensor((first[:, None] + np.arange(16)).ravel(), device="cuda"))
            ctxs.append(ctx)
        print(f"contexts ({time.perf_counter() - t0:.1f} s)", flush=True)
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        vms.vms_batch_autotune(b, fields, vals, resid)
        print(f"autotuned: {vms.vms_batch_get_config(b)}", flush=True)
        vms.vms_batch_use_graph(b, True)
        for _ in range(2):
            vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        got = [(v.clone(), r.clone()) for v, r in zip(vals, resid)]
        # the fixed queue order: the same outputs bit for bit
        vms.vms_batch_set_order(b, False)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        assert all(torch.equal(gv, v) and torch.equal(gr, r) for (gv, gr), v, r in zip(got, vals, resid))
        vms.vms_batch_set_order(b, True)
        for c, f, v, r in zip(ctxs, fields, vals, resid):
            vms.vms_assemble(c, f, v, r)
        stream.synchronize()
        worst_j = worst_r = 0.0
        bitwise = True
        for (gv, gr), v, r, idx in zip(got, vals, resid, ident):
            assert torch.equal(gv[idx], v[idx])
            bitwise &= bool(torch.equal(gv, v) and torch.equal(gr, r))
            ej = (torch.linalg.vector_norm((gv - v).double()) /
                  (torch.linalg.vector_norm(v.double()) ** 2 - float((v[idx].double() ** 2).sum())) ** 0.5).item()
            er = (torch.linalg.vector_norm(gr - r) / torch.linalg.vector_norm(r)).item()
            worst_j, worst_r = max(worst_j, ej), max(worst_r, er)
        print(f"batch vs single contexts: worst J {worst_j:.2e}, worst R {worst_r:.2e}, "
              f"bit for bit: {bitwise}", flush=True)
        # the same per-item arithmetic and the same summation order: equal bits
        assert bitwise
        # sampled rows of the largest tree against the reference (BF16 bar)
        tree, surf = work[big]
        keys = oracle._mesh.independent_node_keys(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
        assert np.array_equal(vms.vms_export(ctxs[big], vms.VMS_EXPORT_NODE_XYZ).T, oracle._mesh._decode(keys))
        rp = vms.vms_export(ctxs[big], vms.VMS_EXPORT_ROW_PTR)
        mk = vms.vms_export(ctxs[big], vms.VMS_EXPORT_MARKERS, tree.n)
        ma = vms.vms_export(ctxs[big], vms.VMS_EXPORT_MASTERS, tree.n)
        cutm = ma[mk == 2].ravel()
        rng = np.random.default_rng(1)
        nodes = np.unique(np.concatenate([rng.choice(keys.size, 24, replace=False),
                                          rng.choice(cutm[cutm >= 0], 8, replace=False)]))
        rows = SR.reference_rows(oracle, tree, surf, host_f, keys, nodes, depth=3)
        ev, er, _ = SR.compare_rows(rows, rp, vms.vms_export(ctxs[big], vms.VMS_EXPORT_NODE_ROW_PTR),
                                    vms.vms_export(ctxs[big], vms.VMS_EXPORT_NODE_COL), got[big][0],
                                    got[big][1], tol=1e-5)
        print(f"largest tree ({tree.n} octants): {nodes.size} sampled rows against the reference: "
              f"values {ev:.2e}, residual {er:.2e}", flush=True)
        # constant state: zero residual in every tree (graph replay)
        for f in fields:
            for n, v in (("ux", 0.7), ("uy", -0.3), ("uz", 0.2), ("p", 0.0), ("ux0", 0.7), ("uy0", -0.3),
                         ("uz0", 0.2)):
                f[n].fill_(v)
        vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        rmax = max(r.abs().max().item() for r in resid)
        print(f"constant state: max |R| {rmax:.2e}")
        assert rmax < 1e-6
        vms.vms_batch_destroy(b)
    for c in ctxs:
        vms.vms_destroy(c)
