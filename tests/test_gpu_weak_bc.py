"""Weak (Nitsche) boundary terms, eq. (weakbc), on the GPU against the CPU
reference.

* Surface points (element, reference coordinates, weights, normals):
  bit-exact (the host builds them with the reference's arithmetic).
* Residual and Jacobian with the terms on: FP64 entrywise 1e-12 of each row's
  1-norm and normwise 1e-12 over the rows of active nodes (identity rows
  exact); residual-only and matrix-free Jacobian action consistent with it;
  BF16x3 within 1e-5.
* Properties at full size: u = u_prev = g constant, p = 0 gives a zero
  residual; switching the terms off again restores the plain assembly
  bit for bit.
"""
import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12
G = (0.1, 0.0, -0.2)
CB = 4.0


@pytest.fixture(scope="module")
def vms():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_00706_amd import vms as V
    V.lib()
    return V


def node_xyz(asm, tree):
    return asm.export(1).T.astype(np.float64) / float(1 << tree.max_level) * tree.root_len + \
        np.asarray(tree.origin)


def case():
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    return I.sphere_refined_octree(c, 0.2, 3, 5, 1.5), I.icosphere(2, 0.2, c)


@pytest.fixture(scope="module")
def reference(oracle):
    tree, surf = case()
    O = oracle
    ms0 = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    mk, _, _ = O.markers(tree, ms0, surf)
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level, active=mk != O.IN)
    sub = O.subquad(tree, surf, np.nonzero(mk == O.INTERCEPTED)[0], 3)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << tree.max_level)
    f = I.make_fields(xyz, 1001)
    V, R = O.assemble(tree, ms, f, mk=mk, sub=sub, depth=3)
    Vs, Rs, sp = O.weak_bc(tree, ms, surf, mk, f, c_b=CB, g=G)
    return tree, surf, ms, mk, sub, f, V + Vs, R + Rs, sp


def check(vals, V, res, R, ms):
    rid = np.repeat(np.arange(ms.row_ptr.size - 1), np.diff(ms.row_ptr))
    act = np.repeat(np.repeat(ms.node_active, 4), np.diff(ms.row_ptr))
    assert np.array_equal(vals[~act], V[~act])
    rown = np.zeros(ms.row_ptr.size - 1)
    np.add.at(rown, rid, np.abs(V))
    err = np.abs(vals - V)
    assert np.all(err <= TOL * rown[rid]), (err / np.maximum(rown[rid], 1e-300)).max()
    assert np.linalg.norm((vals - V)[act]) <= TOL * np.linalg.norm(V[act])
    assert np.linalg.norm(res - R) <= TOL * np.linalg.norm(R)


def test_surface_points_bit_exact(vms, reference):
    tree, surf, ms, mk, sub, f, V, R, sp = reference
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    asm.set_weak_bc(True, CB, G)
    g = asm.export(vms.VMS_EXPORT_SURFGP)
    assert g["el"].size == sp["el"].size > 0
    for k in ("el", "xi", "w", "n"):
        assert np.array_equal(g[k], sp[k]), k
    assert vms.vms_stats(asm.ctx)["n_surfgp"] == sp["el"].size
    asm.close()


def test_weak_bc_fp64_residual_jacobian_and_action(vms, reference):
    import torch
    tree, surf, ms, mk, sub, f, V, R, sp = reference
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    asm.set_weak_bc(True, CB, G)
    asm.set_fields(f)
    asm.assemble()
    torch.cuda.synchronize()
    vals, res = asm.vals.cpu().numpy(), asm.resid.cpu().numpy()
    check(vals, V, res, R, ms)
    # residual-only assembly
    asm.apply()
    r2 = asm.resid.cpu().numpy()
    assert np.linalg.norm(r2 - R) <= TOL * np.linalg.norm(R)
    # matrix-free action and the CSR product against the reference J x
    x = np.random.default_rng(9).normal(size=asm.sizes["n_rows"])
    xt = torch.as_tensor(x, device="cuda")
    rid = np.repeat(np.arange(ms.row_ptr.size - 1), np.diff(ms.row_ptr))
    y_ref = np.zeros(ms.row_ptr.size - 1)
    np.add.at(y_ref, rid, V * x[ms.col_idx])
    act = np.repeat(ms.node_active, 4)
    for y in (asm.jacobian_action(xt).cpu().numpy(), asm.spmv(xt).cpu().numpy()):
        assert np.array_equal(y[~act], y_ref[~act])
        assert np.linalg.norm((y - y_ref)[act]) <= TOL * np.linalg.norm(y_ref[act])
    asm.close()


def test_weak_bc_bf16_form(vms, reference):
    import torch
    tree, surf, ms, mk, sub, f, V, R, sp = reference
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=vms.VMS_MIXED_BF16))
    asm.set_weak_bc(True, CB, G)
    asm.set_fields(f)
    asm.assemble()
    torch.cuda.synchronize()
    vals = asm.vals.cpu().numpy().astype(np.float64)
    act = np.repeat(np.repeat(ms.node_active, 4), np.diff(ms.row_ptr))
    ej = np.linalg.norm((vals - V)[act]) / np.linalg.norm(V[act])
    er = np.linalg.norm(asm.resid.cpu().numpy() - R) / np.linalg.norm(R)
    print(f"bf16 with weak terms: J {ej:.2e} R {er:.2e}")
    assert ej <= 1e-5 and er <= 1e-5
    asm.close()


def test_weak_bc_full_size_properties(vms):
    """Sphere workload: u = u_prev = g, p = 0 gives R = 0 with the surface
    terms on; switching them off restores the plain matrix bit for bit."""
    import torch
    tree, surf = I.sphere_workload()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    n = asm.sizes["n_nodes"]
    fc = {"ux": np.full(n, G[0]), "uy": np.full(n, G[1]), "uz": np.full(n, G[2]), "p": np.zeros(n)}
    fc.update({"ux0": fc["ux"], "uy0": fc["uy"], "uz0": fc["uz"]})
    asm.set_fields(I.make_fields(node_xyz(asm, tree), 1001))
    asm.assemble()
    plain = asm.vals.clone()
    asm.set_weak_bc(True, CB, G)
    st = vms.vms_stats(asm.ctx)
    assert st["n_surfgp"] == 3 * surf.tris.shape[0]
    asm.assemble()
    assert not torch.equal(asm.vals, plain)
    asm.set_fields(fc)
    asm.assemble()
    torch.cuda.synchronize()
    assert asm.resid.abs().max().item() < 1e-15
    asm.set_weak_bc(False)
    asm.set_fields(I.make_fields(node_xyz(asm, tree), 1001))
    asm.assemble()
    assert torch.equal(asm.vals, plain)
    asm.close()


def test_element_weights_match_reference(vms, oracle, reference):
    """eq. (Wpart) weights from the library equal the reference's, bit for
    bit, with the surface terms off and on."""
    tree, surf, ms, mk, sub, f, V, R, sp = reference
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    r = 3.7
    w0 = vms.vms_element_weights(asm.ctx, tree.n, r)
    assert np.array_equal(w0, oracle.element_weights(tree, mk, sub, None, r))
    asm.set_weak_bc(True, CB, G)
    w1 = vms.vms_element_weights(asm.ctx, tree.n, r)
    assert np.array_equal(w1, oracle.element_weights(tree, mk, sub, sp, r))
    assert np.all(w1[mk == 0] == 1.0) and np.all(w1[mk == 1] == 0.0)
    asm.close()
