"""Parity of the matrix-free Jacobian action and of the CSR product.

* vms_apply_jacobian (y = J(U) x without the matrix) against the reference's
  directional derivative of the residual (itself pinned against the
  column-by-column Jacobian): FP64 normwise and max-norm 1e-12 on a uniform
  mesh, a hanging mesh and a cut mesh with sub-cell points (ragged items);
  mixed contexts (FP32 point work) normwise 1e-5.
* vms_spmv with the GPU-assembled values against the reference's Jacobian
  times x (1e-12), and at the full sphere size against the matrix-free action
  (the same J, two formulations; 1e-12).
* Properties: x = 0 gives y = 0; inactive rows give y = x; the rest state with
  a constant velocity direction gives rho h^3/dt c on interior momentum rows.

Norms are taken over the rows of active nodes: the identity rows of inactive
nodes (y = x, O(1)) are checked exactly and would otherwise dominate them.
"""
import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def reference_mesh(O, tree, surf, depth):
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    mk = np.zeros(tree.n, np.uint8)
    sub = None
    if surf is not None:
        mk, _, _ = O.markers(tree, ms, surf)
        ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level, active=mk != O.IN)
        sub = O.subquad(tree, surf, np.nonzero(mk == O.INTERCEPTED)[0], depth)
    return ms, mk, sub


def ref_fields(vms, asm, tree, ms, seed):
    """Fields at the reference's node positions (the library's must be the same)."""
    assert np.array_equal(asm.export(vms.VMS_EXPORT_NODE_XYZ).T, ms.node_xyz_int)
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << tree.max_level) * tree.root_len
    return I.make_fields(xyz + np.asarray(tree.origin), seed)


def close(y, y_ref, tol, act):
    """act: rows of active nodes (compared to tol); the others must match exactly."""
    assert np.array_equal(y[~act], y_ref[~act])
    y, y_ref = y[act], y_ref[act]
    assert np.linalg.norm(y - y_ref) <= tol * np.linalg.norm(y_ref), \
        np.linalg.norm(y - y_ref) / np.linalg.norm(y_ref)
    assert np.abs(y - y_ref).max() <= tol * np.abs(y_ref).max()


def active_rows(vms, asm):
    mk = asm.export(vms.VMS_EXPORT_MARKERS)
    ma = asm.export(vms.VMS_EXPORT_MASTERS)[mk != 1]
    act = np.zeros(asm.sizes["n_nodes"], bool)
    act[ma[ma >= 0]] = True
    return np.repeat(act, 4)


CASES = {
    "uniform16": (lambda: (I.uniform_octree(4), None), 3),
    "hanging": (lambda: (I.sphere_refined_octree((0.5 + I.BODY_OFFSET[0], 0.5, 0.5), 0.3, 2, 5, 1.5),
                         None), 3),
    "cut": (lambda: (I.sphere_refined_octree(tuple(0.5 + o for o in I.BODY_OFFSET), 0.2, 3, 5, 1.5),
                     I.icosphere(2, 0.2, tuple(0.5 + o for o in I.BODY_OFFSET))), 3),
    "cut_depth1": (lambda: (I.sphere_refined_octree(tuple(0.5 + o for o in I.BODY_OFFSET), 0.25, 2, 4, 1.0),
                            I.icosphere(2, 0.25, tuple(0.5 + o for o in I.BODY_OFFSET))), 1),
}


@pytest.mark.parametrize("case", list(CASES))
def test_jacobian_action_fp64_against_reference(vms, oracle, case):
    mk_tree, depth = CASES[case]
    tree, surf = mk_tree()
    torch = pytest.importorskip("torch")
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=depth))
    ms, mk, sub = reference_mesh(oracle, tree, surf, depth)
    f = ref_fields(vms, asm, tree, ms, 1001)
    asm.set_fields(f)
    n = asm.sizes["n_rows"]
    x = np.random.default_rng(3).normal(size=n)
    y = asm.jacobian_action(torch.as_tensor(x, device="cuda")).cpu().numpy()
    y_ref = oracle.jacobian_apply(tree, ms, f, x, mk=mk, sub=sub, depth=depth)
    act = np.repeat(ms.node_active, 4)
    assert np.array_equal(act, active_rows(vms, asm))
    print(f"{case}: {tree.n} octants, rel err "
          f"{np.linalg.norm((y - y_ref)[act]) / np.linalg.norm(y_ref[act]):.2e}")
    close(y, y_ref, TOL, act)
    inact = np.nonzero(~ms.node_active)[0]
    if surf is not None:
        assert inact.size > 0
    for c in range(4):
        assert np.array_equal(y[4 * inact + c], x[4 * inact + c])
    asm.close()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_jacobian_action_mixed_contexts(vms, oracle, prec):
    """Mixed contexts evaluate the point work in FP32: normwise 1e-5."""
    tree, surf = CASES["cut"][0]()
    torch = pytest.importorskip("torch")
    p = vms.VMS_MIXED_BF16 if prec == "bf16" else vms.VMS_MIXED_FP16
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=p))
    ms, mk, sub = reference_mesh(oracle, tree, surf, 3)
    f = ref_fields(vms, asm, tree, ms, 1001)
    asm.set_fields(f)
    x = np.random.default_rng(4).normal(size=asm.sizes["n_rows"])
    y = asm.jacobian_action(torch.as_tensor(x, device="cuda")).cpu().numpy()
    y_ref = oracle.jacobian_apply(tree, ms, f, x, mk=mk, sub=sub, depth=3)
    act = np.repeat(ms.node_active, 4)
    err = np.linalg.norm((y - y_ref)[act]) / np.linalg.norm(y_ref[act])
    print(f"{prec}: rel err {err:.2e}")
    assert err <= 1e-5
    assert np.array_equal(y[~act], x[~act])
    asm.close()


def test_spmv_against_reference_jacobian(vms, oracle):
    """The CSR product with the GPU-assembled Jacobian equals the reference's
    Jacobian times x, and the matrix-free action."""
    tree, surf = CASES["cut"][0]()
    torch = pytest.importorskip("torch")
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    ms, mk, sub = reference_mesh(oracle, tree, surf, 3)
    f = ref_fields(vms, asm, tree, ms, 1001)
    asm.set_fields(f)
    asm.assemble()
    x = np.random.default_rng(6).normal(size=asm.sizes["n_rows"])
    xt = torch.as_tensor(x, device="cuda")
    y = asm.spmv(xt).cpu().numpy()
    V, _ = oracle.assemble(tree, ms, f, mk=mk, sub=sub, depth=3, resid=False)
    rid = np.repeat(np.arange(ms.row_ptr.size - 1), np.diff(ms.row_ptr))
    y_ref = np.zeros(ms.row_ptr.size - 1)
    np.add.at(y_ref, rid, V * x[ms.col_idx])
    act = np.repeat(ms.node_active, 4)
    close(y, y_ref, TOL, act)
    close(asm.jacobian_action(xt).cpu().numpy(), y_ref, TOL, act)
    # the product is reproducible bit for bit (fixed summation order)
    assert np.array_equal(asm.spmv(xt).cpu().numpy(), y)
    asm.close()


def test_matrix_free_equals_spmv_full_size(vms):
    """Sphere workload (~194k octants, 4M sub-cell points): the matrix-free
    action and the product with the assembled matrix agree to 1e-12, in FP64;
    x = 0 gives y = 0 exactly."""
    torch = pytest.importorskip("torch")
    tree, surf = I.sphere_workload()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    asm.set_fields(I.make_fields(node_xyz(asm, tree), 1001))
    asm.assemble()
    x = torch.as_tensor(np.random.default_rng(7).normal(size=asm.sizes["n_rows"]), device="cuda")
    y1 = asm.jacobian_action(x)
    y2 = asm.spmv(x)
    act = torch.as_tensor(active_rows(vms, asm), device="cuda")
    assert torch.equal(y1[~act], y2[~act]) and torch.equal(y1[~act], x[~act])
    err = (torch.linalg.vector_norm((y1 - y2)[act]) / torch.linalg.vector_norm(y2[act])).item()
    print(f"full size: rel diff {err:.2e}")
    assert err <= TOL
    z = asm.jacobian_action(torch.zeros_like(x))
    assert torch.count_nonzero(z).item() == 0
    asm.close()


def test_rest_state_constant_direction_closed_form(vms):
    """u = u_prev = 0, p = 0, x = constant velocity on the 16^3 mesh: interior
    momentum rows rho h^3/dt c, interior continuity rows 0."""
    torch = pytest.importorskip("torch")
    tree = I.uniform_octree(4)
    rho, dt = 1.0, 0.01
    asm = vms.Assembler(tree, None, vms.make_params(quad_depth=3, rho=rho, dt=dt))
    n = asm.sizes["n_nodes"]
    z = np.zeros(n)
    asm.set_fields({"ux": z, "uy": z, "uz": z, "p": z, "ux0": z, "uy0": z, "uz0": z})
    cvel = np.array([0.7, -1.1, 0.4])
    x = np.zeros(4 * n)
    for k in range(3):
        x[k::4] = cvel[k]
    y = asm.jacobian_action(torch.as_tensor(x, device="cuda")).cpu().numpy()
    ijk = asm.export(vms.VMS_EXPORT_NODE_XYZ).T
    inner = np.nonzero(np.all((ijk > 0) & (ijk < (1 << tree.max_level)), axis=1))[0]
    h = 1.0 / 16
    for k in range(3):
        np.testing.assert_allclose(y[4 * inner + k], rho * h ** 3 / dt * cvel[k], rtol=1e-13)
    assert np.abs(y[4 * inner + 3]).max() < 1e-15
    asm.close()
