"""The learned in-out workload's geometry: two filleted bluff boxes (1.0 x 0.25
x 0.3, fillet 0.03, gap 0.5) in an 8 x 2 x 2 domain, which fills a quarter of
the octree root in y and in z.

* A small tree of the same geometry (coarser surface): labels, sub-cell
  entries, node coordinates and CSR indices bit-exact against the CPU
  reference; FP64 values to 1e-12, BF16 to 1e-5.
* Full size (levels 6-11, about 10^7 octants, 198,744 triangles, more than
  2^31 CSR nonzeros): node numbering equal to the reference's own numbering of
  the whole tree; sampled node rows (random ones, rows whose CSR offsets pass
  2^31, nodes of INTERCEPTED elements, inactive nodes) against the reference's
  windowed assembly: columns bit-exact, values and residual within 1e-12;
  properties that hold at any size (a constant state has
  zero residual; the CSR product equals the matrix-free Jacobian action;
  inactive rows are identity rows), BF16 within 1e-5 of FP64 over the rows of
  active nodes, and the learned filter (trained on 4M exact distances) giving
  the exact labels of the kept sub-cell points, themselves checked against the
  reference on a subsample.
"""
import time

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


def phys(tree, ijk):
    return ijk.astype(np.float64) / float(1 << tree.max_level) * tree.root_len + np.asarray(tree.origin)


def test_two_boxes_small_against_reference(env, oracle):
    torch, vms = env
    O = oracle
    tree, surf = I.two_box_workload(lmin=3, lmax=7, beta=2.0, n_face=6)
    assert I.is_watertight(surf)
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    mk, _, nd = O.markers(tree, ms, surf)
    assert nd == 0
    msa = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level, active=mk != O.IN)
    cut = np.nonzero(mk == O.INTERCEPTED)[0]
    sub = O.subquad(tree, surf, cut, 3)
    # fields at the reference's node positions (domain scale: the 2 x 2 cross-section)
    f = I.make_fields(phys(tree, msa.node_xyz_int), 1001, shortest_side=2.0)
    V, R = O.assemble(tree, msa, f, mk=mk, sub=sub, depth=3)
    act = np.repeat(np.repeat(msa.node_active, 4), np.diff(msa.row_ptr))
    for prec, tol in ((vms.VMS_FP64, 1e-12), (vms.VMS_MIXED_BF16, 1e-5)):
        asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
        assert np.array_equal(asm.export(vms.VMS_EXPORT_MARKERS), mk)
        assert np.array_equal(asm.export(vms.VMS_EXPORT_NODE_XYZ).T, msa.node_xyz_int)
        assert np.array_equal(asm.export(vms.VMS_EXPORT_ROW_PTR), msa.row_ptr)
        assert np.array_equal(asm.export(vms.VMS_EXPORT_COL_IDX), msa.col_idx)
        g = asm.export(vms.VMS_EXPORT_SUBGP)
        for k in ("el", "key", "lvl", "xyz"):
            assert np.array_equal(g[k], sub[k]), k
        asm.set_fields(f)
        asm.assemble()
        torch.cuda.synchronize()
        vals = asm.vals.cpu().numpy().astype(np.float64)
        res = asm.resid.cpu().numpy()
        assert np.array_equal(vals[~act], V[~act])  # identity rows of inactive nodes
        ej = np.linalg.norm(vals[act] - V[act]) / np.linalg.norm(V[act])
        er = np.linalg.norm(res - R) / np.linalg.norm(R)
        print(f"{tree.n} octants, {cut.size} INTERCEPTED, {sub['el'].size} sub-cell points, "
              f"precision {prec}: J {ej:.2e} R {er:.2e}")
        assert ej <= tol and er <= tol
        asm.close()


def _sq_norm(a, chunk=1 << 27):
    return sum(float((a[i:i + chunk].double() ** 2).sum()) for i in range(0, a.numel(), chunk))


def _sq_diff(a, b, chunk=1 << 27):
    return sum(float(((a[i:i + chunk].double() - b[i:i + chunk]) ** 2).sum())
               for i in range(0, a.numel(), chunk))


@pytest.mark.timeout(1000)
def test_two_boxes_full_size(env, oracle, monkeypatch):
    torch, vms = env
    from paper_2009_00706_amd.learned import LearnedFilter
    t0 = time.perf_counter()
    tree, surf = I.two_box_workload()
    print(f"workload: {tree.n} octants, {surf.tris.shape[0]} triangles "
          f"({time.perf_counter() - t0:.1f} s)", flush=True)
    assert 0.9e7 < tree.n < 1.1e7 and surf.tris.shape[0] == 198744
    monkeypatch.setenv("VMS_SETUP_LOG", "1")  # set-up stages on stderr as they finish

    # ---- FP64: properties at full size
    t0 = time.perf_counter()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    sz, st = asm.sizes, vms.vms_stats(asm.ctx)
    n, nnz = sz["n_nodes"], sz["nnz"]
    print(f"FP64 context ({time.perf_counter() - t0:.1f} s): {sz}, stats {st}", flush=True)
    assert nnz > 2 ** 31
    mk = asm.export(vms.VMS_EXPORT_MARKERS)
    ma = asm.export(vms.VMS_EXPORT_MASTERS)[mk != 1]
    active = np.zeros(n, bool)
    active[ma[ma >= 0]] = True
    inact = np.nonzero(~active)[0]
    rp = asm.export(vms.VMS_EXPORT_ROW_PTR)
    const = {"ux": np.full(n, 0.7), "uy": np.full(n, -0.3), "uz": np.full(n, 0.2), "p": np.zeros(n)}
    const.update({"ux0": const["ux"], "uy0": const["uy"], "uz0": const["uz"]})
    asm.set_fields(const)
    asm.assemble()
    torch.cuda.synchronize()
    rmax = asm.resid.abs().max().item()
    print(f"constant state: max |R| {rmax:.2e}", flush=True)
    assert rmax < 1e-15
    # the reference numbers the nodes of the whole tree itself; fields live at
    # its node positions
    t1 = time.perf_counter()
    keys = oracle._mesh.independent_node_keys(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    kxyz = oracle._mesh._decode(keys)
    assert np.array_equal(asm.export(vms.VMS_EXPORT_NODE_XYZ).T, kxyz)
    print(f"reference node numbering equal ({time.perf_counter() - t1:.1f} s)", flush=True)
    f = I.make_fields(phys(tree, kxyz), 1001, shortest_side=2.0)
    del kxyz
    asm.set_fields(f)
    t1 = time.perf_counter()
    asm.assemble()
    torch.cuda.synchronize()
    print(f"FP64 assembly {1e3 * (time.perf_counter() - t1):.0f} ms (first call)", flush=True)
    ref, rref = asm.vals, asm.resid.clone()
    # ---- sampled rows against the reference (selection may use the exports)
    import sampled_rows as SR
    rng = np.random.default_rng(0)
    act_idx = np.nonzero(active)[0]
    high = act_idx[rp[4 * act_idx] > 2 ** 31]
    cutm = ma[mk[mk != 1] == 2].ravel()
    cutm = cutm[cutm >= 0]
    nodes = np.unique(np.concatenate([rng.choice(act_idx, 24, replace=False),
                                      rng.choice(high, 24, replace=False),
                                      rng.choice(cutm, 10, replace=False),
                                      rng.choice(inact, 4, replace=False)]))
    t1 = time.perf_counter()
    rows = SR.reference_rows(oracle, tree, surf, f, keys, nodes, depth=3,
                             log=lambda m: print(m, flush=True))
    nrp = asm.export(vms.VMS_EXPORT_NODE_ROW_PTR)
    ncol = asm.export(vms.VMS_EXPORT_NODE_COL)
    ev, er, omax = SR.compare_rows(rows, rp, nrp, ncol, ref, rref)
    print(f"{nodes.size} sampled node rows against the reference ({time.perf_counter() - t1:.1f} s): "
          f"values {ev:.2e}, residual {er:.2e}, CSR offsets up to {omax} (2^31 = {2 ** 31})", flush=True)
    assert omax > 2 ** 31
    del nrp, ncol, keys
    # identity rows: a sample of inactive nodes' rows hold a single 1 on the diagonal
    for node in rng.choice(inact, min(64, inact.size), replace=False):
        for c in range(4):
            r = 4 * int(node) + c
            row = ref[int(rp[r]):int(rp[r + 1])]
            assert int((row != 0).sum()) == 1 and float(row.sum()) == 1.0
    # the CSR product (more than 2^31 entries) against the matrix-free action
    gen = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn(4 * n, dtype=torch.float64, device="cuda", generator=gen)
    y_csr = asm.spmv(x)
    y_mf = asm.jacobian_action(x)
    torch.cuda.synchronize()
    ep = (torch.linalg.vector_norm(y_csr - y_mf) / torch.linalg.vector_norm(y_mf)).item()
    print(f"CSR product vs matrix-free action: {ep:.2e}", flush=True)
    assert ep <= 1e-12
    del x, y_csr, y_mf
    asm.close()
    asm.vals = asm.resid = None  # ref and rref hold them until the comparison is done

    # ---- BF16 form against FP64: the inactive rows (one 1 each) are exact in
    # both, so the active-row norms follow from the full ones
    asm2 = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=vms.VMS_MIXED_BF16))
    asm2.set_fields(f)
    asm2.assemble()
    torch.cuda.synchronize()
    ref_sq = _sq_norm(ref) - 4 * inact.size
    ej = (_sq_diff(asm2.vals, ref) / ref_sq) ** 0.5
    er = (torch.linalg.vector_norm(asm2.resid - rref) / torch.linalg.vector_norm(rref)).item()
    print(f"BF16 vs FP64 (active rows): J {ej:.2e} R {er:.2e}", flush=True)
    assert ej <= 1e-5 and er <= 1e-5
    del ref, rref
    pts = asm2.export(vms.VMS_EXPORT_SUBGP)["xyz"]
    asm2.close()
    torch.cuda.empty_cache()

    # ---- learned filter on the kept sub-cell points
    t0 = time.perf_counter()
    lf = LearnedFilter(surf, trunc=0.05, seed=0, sigma=1.0)
    loss = lf.train(4_000_000, steps=8000, batch=8192, lr=3e-3)
    lo, hi = surf.verts.min(0), surf.verts.max(0)
    held = I.sdf_sample_points(surf, lo - 0.2, hi + 0.2, 2_000_000, 21, near_frac=0.9, near_dist=0.02)
    lf.calibrate(held, grid=(48, 8, 8))
    torch.cuda.synchronize()
    print(f"learned filter trained and calibrated in {time.perf_counter() - t0:.1f} s "
          f"(loss {loss:.2e})", flush=True)
    exact = lf.classify(pts, learned=False)
    learned = lf.classify(pts, learned=True)
    torch.cuda.synchronize()
    assert torch.equal(exact, learned)
    sample = np.sort(rng.choice(pts.shape[0], 1000, replace=False))
    refl, _ = oracle.label_points(surf, pts[sample])
    assert np.array_equal(exact.cpu().numpy()[sample], refl)
    tt = {}
    for mode in (False, True):
        lf.classify(pts, learned=mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(3):
            lf.classify(pts, learned=mode)
        torch.cuda.synchronize()
        tt[mode] = (time.perf_counter() - t1) / 3
    print(f"{pts.shape[0]} kept sub-cell points: exact {1e3 * tt[False]:.1f} ms, "
          f"learned {1e3 * tt[True]:.1f} ms ({tt[False] / tt[True]:.2f}x)", flush=True)
    lf.close()
