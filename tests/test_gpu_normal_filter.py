"""The normal-based in-out test of Alg. 5 as a certified filter in front of the
exact test of the sub-cell quadrature (VMS_INOUT_NORMAL).

* Bodies and convexity: an icosphere and the two filleted boxes are convex
  bodies, a dented icosphere is not (exact orientation of every edge's far
  vertex at vms_create).
* Labels: after a relabel in the normal mode the kept sub-cell points, the CSR
  values and the residual equal those of the exact mode bit for bit, and the
  points of a sample of INTERCEPTED elements equal the CPU reference's; on
  convex bodies the filter decides a share of the candidates, on a non-convex
  body none (every point goes to the exact test).
"""
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


def dented(subdiv, r, c, depth):
    """Icosphere with vertex 0 pushed towards the centre by depth x r: the
    faces around it form a dent (not convex), the surface stays closed."""
    s = I.icosphere(subdiv, r, c)
    v = s.verts.copy()
    v[0] = np.asarray(c) + (v[0] - np.asarray(c)) * (1.0 - depth)
    return I.Surface(v, s.tris.copy(), {"kind": "dented icosphere"})


def compare_modes(torch, vms, oracle, tree, surf, f, n_sample=30):
    ex = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    nm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, inout_mode=vms.VMS_INOUT_NORMAL))
    for a in (ex, nm):
        a.set_fields(f)
        a.assemble(flags=vms.VMS_RELABEL)
    torch.cuda.synchronize()
    vms.vms_sizes(nm.ctx)                     # raises on a kept-point count changed by the relabel
    ge, gn = ex.export(vms.VMS_EXPORT_SUBGP), nm.export(vms.VMS_EXPORT_SUBGP)
    for k in ("el", "key", "lvl", "xyz"):
        assert np.array_equal(ge[k], gn[k]), k
    assert torch.equal(ex.vals, nm.vals) and torch.equal(ex.resid, nm.resid)
    rs = vms.vms_relabel_stats(nm.ctx)
    decided = 1.0 - rs["exact_in_last_relabel"] / rs["candidates"]
    mk = ex.export(vms.VMS_EXPORT_MARKERS)
    cut = np.nonzero(mk == 2)[0]
    pick = np.sort(np.random.default_rng(5).choice(cut, min(n_sample, cut.size), replace=False))
    ref = oracle.subquad(tree, surf, pick, 3)
    sel = np.isin(gn["el"], pick)
    for k in ("el", "key", "lvl", "xyz"):
        assert np.array_equal(gn[k][sel], ref[k]), k
    comps = vms.vms_components(nm.ctx)
    ex.close()
    nm.close()
    return decided, rs, comps


def fields(vms, tree, surf):
    a = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    xyz = a.export(vms.VMS_EXPORT_NODE_XYZ).T / float(1 << tree.max_level)
    a.close()
    return I.make_fields(xyz * tree.root_len + np.asarray(tree.origin), 1000)


def test_convex_sphere(env, oracle):
    torch, vms = env
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    s = I.icosphere(3, 0.2, c)
    tree = I.sphere_refined_octree(c, 0.2, 3, 6, 1.5)
    decided, rs, (n, convex) = compare_modes(torch, vms, oracle, tree, s, fields(vms, tree, s))
    print(f"[normal] sphere: {tree.n} octants, {rs['candidates']} candidates, decided {decided:.3f}", flush=True)
    assert n == 1 and convex.all()
    assert decided > 0.2


def test_two_convex_boxes(env, oracle):
    torch, vms = env
    tree, s = I.two_box_workload(lmin=3, lmax=7, beta=2.0, n_face=6)
    f = fields(vms, tree, s)
    decided, rs, (n, convex) = compare_modes(torch, vms, oracle, tree, s, f)
    print(f"[normal] two boxes: {tree.n} octants, {rs['candidates']} candidates, decided {decided:.3f}",
          flush=True)
    assert n == 2 and convex.all()
    assert decided > 0.2


def test_non_convex_body_goes_to_the_exact_test(env, oracle):
    torch, vms = env
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    s = dented(3, 0.2, c, 0.3)
    assert I.is_watertight(s)
    tree = I.sphere_refined_octree(c, 0.2, 3, 6, 1.5)
    decided, rs, (n, convex) = compare_modes(torch, vms, oracle, tree, s, fields(vms, tree, s))
    print(f"[normal] dented sphere: decided {decided:.3f}", flush=True)
    assert n == 1 and not convex.any()
    assert decided == 0.0


def test_convex_and_non_convex_bodies(env, oracle):
    """Two bodies, one convex and one dented: elements cut by the convex one
    use the filter, those cut by the dented one do not; labels stay exact."""
    torch, vms = env
    c0 = np.array([0.3, 0.5, 0.5]) + I.BODY_OFFSET
    c1 = np.array([0.7, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.merge_surfaces([I.icosphere(3, 0.12, c0), dented(3, 0.12, c1, 0.3)])
    tree = I.sphere_refined_octree(tuple((c0 + c1) / 2), 0.3, 3, 6, 1.5)
    decided, rs, (n, convex) = compare_modes(torch, vms, oracle, tree, s, fields(vms, tree, s))
    print(f"[normal] convex + dented: decided {decided:.3f}", flush=True)
    assert n == 2 and convex.tolist() == [True, False]
    assert 0.0 < decided
