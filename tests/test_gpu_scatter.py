"""Atomic scatter of the element matrices (vms_set_scatter), the alternative
measured beside the record-and-gather scatter.

* FP64 on a cut, hanging mesh: CSR values within 1e-12 of the CPU reference
  (entrywise against each row's 1-norm and normwise over the rows of active
  nodes), within 1e-13 of the record scatter (only the order of the additions
  differs), identity rows of inactive nodes exact, residual identical.
* BF16x3: within 1e-6 of the record scatter of the same form (FP32 sums).
* Error paths: unknown mode, weak boundary terms on either side of the switch.
"""
import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vms():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_00706_amd import vms as V
    V.lib()
    return V


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
    return tree, surf, ms, f, V, R


def rows(ms):
    rid = np.repeat(np.arange(ms.row_ptr.size - 1), np.diff(ms.row_ptr))
    act = np.repeat(np.repeat(ms.node_active, 4), np.diff(ms.row_ptr))
    return rid, act


def run(vms, tree, surf, f, prec, mode):
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
    asm.set_fields(f)
    vms.vms_set_scatter(asm.ctx, mode)
    asm.vals.fill_(np.nan)
    asm.assemble(flags=vms.VMS_RELABEL)
    v1 = asm.vals.cpu().numpy().copy()
    r1 = asm.resid.cpu().numpy().copy()
    asm.assemble(flags=0)     # a second call overwrites (the values are zeroed first)
    v2 = asm.vals.cpu().numpy().copy()
    asm.close()
    return v1, r1, v2


def test_atomic_fp64_against_reference_and_records(vms, reference):
    tree, surf, ms, f, V, R = reference
    print(f"[scatter] fp64: {tree.n} octants, nnz {V.size}", flush=True)
    va, ra, va2 = run(vms, tree, surf, f, vms.VMS_FP64, vms.VMS_SCATTER_ATOMIC)
    vr, rr, _ = run(vms, tree, surf, f, vms.VMS_FP64, vms.VMS_SCATTER_RECORDS)
    rid, act = rows(ms)
    rown = np.zeros(ms.row_ptr.size - 1)
    np.add.at(rown, rid, np.abs(V))
    for v in (va, va2):
        assert np.isfinite(v).all()
        assert np.array_equal(v[~act], V[~act])            # identity rows of inactive nodes
        err = np.abs(v - V)
        assert np.all(err <= 1e-12 * rown[rid]), (err / np.maximum(rown[rid], 1e-300)).max()
        assert np.linalg.norm((v - V)[act]) <= 1e-12 * np.linalg.norm(V[act])
        assert np.all(np.abs(v - vr) <= 1e-13 * rown[rid])
    assert np.array_equal(ra, rr)                          # the residual keeps its records
    assert np.linalg.norm(ra - R) <= 1e-12 * np.linalg.norm(R)


def test_atomic_bf16_against_records(vms, reference):
    tree, surf, ms, f, V, R = reference
    va, ra, _ = run(vms, tree, surf, f, vms.VMS_MIXED_BF16, vms.VMS_SCATTER_ATOMIC)
    vr, rr, _ = run(vms, tree, surf, f, vms.VMS_MIXED_BF16, vms.VMS_SCATTER_RECORDS)
    rid, act = rows(ms)
    rown = np.zeros(ms.row_ptr.size - 1)
    np.add.at(rown, rid, np.abs(V))
    assert np.array_equal(va[~act], vr[~act])
    assert np.all(np.abs(va.astype(np.float64) - vr) <= 1e-6 * rown[rid])
    assert np.linalg.norm((va.astype(np.float64) - V)[act]) <= 1e-5 * np.linalg.norm(V[act])
    assert np.array_equal(ra, rr)


def test_scatter_mode_errors(vms):
    tree, surf = case()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    with pytest.raises(vms.VmsError) as e:
        vms.vms_set_scatter(asm.ctx, 7)
    assert e.value.code == vms.VMS_EINVAL
    asm.set_weak_bc(True, 4.0, (0.0, 0.0, 0.0))
    with pytest.raises(vms.VmsError) as e:
        vms.vms_set_scatter(asm.ctx, vms.VMS_SCATTER_ATOMIC)
    assert e.value.code == vms.VMS_EUNSUPPORTED
    asm.set_weak_bc(False)
    vms.vms_set_scatter(asm.ctx, vms.VMS_SCATTER_ATOMIC)
    with pytest.raises(vms.VmsError) as e:
        asm.set_weak_bc(True, 4.0, (0.0, 0.0, 0.0))
    assert e.value.code == vms.VMS_EUNSUPPORTED
    vms.vms_set_scatter(asm.ctx, vms.VMS_SCATTER_RECORDS)
    asm.set_weak_bc(True, 4.0, (0.0, 0.0, 0.0))
    asm.close()
