"""Triquadratic (27-node) elements on the GPU against the CPU reference.

The 16^3 uniform mesh of the paper's matrix-assembly comparison (and of the
uniform workload): node coordinates, CSR row pointers and column indices
bit-exact; Jacobian values (entrywise within 1e-12 of the row's 1-norm) and the
residual (normwise) within 1e-12; a second call reproduces the bits; a
constant state gives a zero residual; a tree with hanging nodes is refused.
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


def test_q2_uniform_16cube_parity(env, oracle):
    torch, vms = env
    from oracle import q2 as Q
    t = I.uniform_octree(4)
    m = Q.derive_q2_mesh(t)
    q = vms.vms_q2_create(t)
    sz = vms.vms_q2_sizes(q)
    assert sz["n_nodes"] == m.n_nodes == 33 ** 3 and sz["nnz"] == m.nnz
    assert np.array_equal(vms.vms_q2_export(q, vms.VMS_EXPORT_NODE_XYZ).T, m.node_xyz_half)
    assert np.array_equal(vms.vms_q2_export(q, vms.VMS_EXPORT_ROW_PTR), m.row_ptr)
    assert np.array_equal(vms.vms_q2_export(q, vms.VMS_EXPORT_COL_IDX), m.col_idx)
    f = I.make_fields(Q.node_xyz(t, m), 1000)
    fd = {k: torch.as_tensor(f[k], device="cuda") for k in f}
    vals = torch.zeros(sz["nnz"], dtype=torch.float64, device="cuda")
    res = torch.zeros(sz["n_rows"], dtype=torch.float64, device="cuda")
    vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / 5 * 1e3
    g, gr = vals.cpu().numpy(), res.cpu().numpy()
    V, R = Q.assemble(t, m, f)
    rid = np.repeat(np.arange(4 * m.n_nodes), np.diff(m.row_ptr))
    rownorm = np.zeros(4 * m.n_nodes)
    np.add.at(rownorm, rid, np.abs(V))
    ej = np.linalg.norm(g - V) / np.linalg.norm(V)
    ee = np.max(np.abs(g - V) / rownorm[rid])
    er = np.linalg.norm(gr - R) / np.linalg.norm(R)
    print(f"Q2 16^3 ({t.n} elements, {m.n_nodes} nodes, nnz {m.nnz}): J {ej:.2e} (entrywise {ee:.2e}), "
          f"R {er:.2e}; {ms:.2f} ms per assembly, {t.n / ms * 1e3:.3e} elements/s")
    assert ej <= 1e-12 and ee <= 1e-12 and er <= 1e-12
    # bitwise reproducible
    v2, r2 = vals.clone(), res.clone()
    vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    assert torch.equal(v2, vals) and torch.equal(r2, res)
    # constant state: zero residual
    n = m.n_nodes
    for k, v in (("ux", 0.3), ("uy", -0.7), ("uz", 0.2), ("p", 0.0), ("ux0", 0.3), ("uy0", -0.7), ("uz0", 0.2)):
        fd[k] = torch.full((n,), v, dtype=torch.float64, device="cuda")
    vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    assert res.abs().max().item() < 1e-15
    vms.vms_q2_destroy(q)


def test_q2_refuses_hanging_nodes(env):
    torch, vms = env
    c = (0.5 + I.BODY_OFFSET[0], 0.5, 0.5)
    t = I.sphere_refined_octree(c, 0.3, 2, 3, 1.0)
    with pytest.raises(vms.VmsError) as e:
        vms.vms_q2_create(t)
    assert e.value.code == vms.VMS_EMESH
