"""Overlapped schedule of the matrix assembly (vms_set_overlap): the relabel,
the INTERCEPTED items and the surface terms on the context's second stream
beside the summation of the blocks without their records. Outputs must equal
those of the in-order schedule bit for bit (same records, same per-block
summation order), with relabelling, with and without the weak boundary terms,
in FP64 and in the mixed forms; the timing layout of each schedule adds up.
The parity of the (default) overlapped schedule against the CPU reference is
what the other GPU parity tests check."""
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


def case():
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    return I.sphere_refined_octree(c, 0.2, 3, 6, 1.5), I.icosphere(3, 0.2, c)


def fields(vms, asm, tree, seed):
    xyz = asm.export(vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64) / float(1 << tree.max_level)
    return I.make_fields(xyz * tree.root_len + np.asarray(tree.origin), seed)


def outputs(torch, vms, asm, overlap, flags):
    vms.vms_set_overlap(asm.ctx, overlap)
    asm.vals.fill_(np.nan)
    asm.resid.fill_(np.nan)
    asm.assemble(flags=flags)
    torch.cuda.synchronize()
    return asm.vals.cpu().numpy().copy(), asm.resid.cpu().numpy().copy()


@pytest.mark.parametrize("prec", ["fp64", "bf16", "fp16"])
@pytest.mark.parametrize("weak", [False, True])
def test_overlapped_equals_in_order(env, prec, weak):
    torch, vms = env
    tree, surf = case()
    p = {"fp64": vms.VMS_FP64, "bf16": vms.VMS_MIXED_BF16, "fp16": vms.VMS_MIXED_FP16}[prec]
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=p))
    if weak:
        asm.set_weak_bc(True, 4.0, (0.1, 0.0, -0.2))
    asm.set_fields(fields(vms, asm, tree, 1001))
    st = vms.vms_stats(asm.ctx)
    assert st["n_intercepted"] > 0
    print(f"[overlap] {prec} weak={weak}: {tree.n} octants, {st['n_intercepted']} intercepted", flush=True)
    v0, r0 = outputs(torch, vms, asm, False, vms.VMS_RELABEL)
    v1, r1 = outputs(torch, vms, asm, True, vms.VMS_RELABEL)
    v2, r2 = outputs(torch, vms, asm, True, 0)
    assert np.isfinite(v0).all() and np.isfinite(r0).all()
    for v, r in ((v1, r1), (v2, r2)):
        assert np.array_equal(v.view(np.uint8), v0.view(np.uint8))
        assert np.array_equal(r.view(np.uint8), r0.view(np.uint8))
    vms.vms_sizes(asm.ctx)  # no relabel changed a kept-point count
    asm.close()


def test_timing_layouts(env):
    """In order: the five stages tile the call. Overlapped: relabel and late
    items run on the second stream inside the span after the OUT kernel."""
    torch, vms = env
    tree, surf = case()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    asm.set_fields(fields(vms, asm, tree, 7))
    vms.vms_set_timing(asm.ctx, True)
    for ov in (False, True):
        vms.vms_set_overlap(asm.ctx, ov)
        for _ in range(2):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(asm.stream)
            asm.assemble(flags=vms.VMS_RELABEL)
            b.record(asm.stream)
            b.synchronize()
            ms = np.array(vms.vms_last_timing(asm.ctx))
            wall = a.elapsed_time(b)
        print(f"[overlap] overlap={ov}: stages {np.round(ms, 3).tolist()}, call {wall:.3f} ms", flush=True)
        assert (ms >= 0).all() and ms[2] > 0 and ms[3] > 0 and ms[4] > 0
        dev = ms[1] + ms[2] + ms[4] if ov else ms.sum()
        assert dev <= wall * 1.05 + 0.05
        if ov:
            assert ms[0] + ms[3] <= ms[4] * 1.05 + 0.05   # the side stream ends before the join
    asm.close()


def test_no_surface_has_no_second_stream_work(env):
    """A tree without a body has no late blocks: the overlapped setting takes
    the in-order path (the timing layout shows it)."""
    torch, vms = env
    tree = I.uniform_octree(3)
    asm = vms.Assembler(tree, None, vms.make_params())
    asm.set_fields(fields(vms, asm, tree, 3))
    vms.vms_set_timing(asm.ctx, True)
    v1, r1 = outputs(torch, vms, asm, True, 0)
    ms = np.array(vms.vms_last_timing(asm.ctx))
    v0, r0 = outputs(torch, vms, asm, False, 0)
    assert ms[0] == 0 or ms[0] < 0.05
    assert np.array_equal(v1, v0) and np.array_equal(r1, r0)
    asm.close()
