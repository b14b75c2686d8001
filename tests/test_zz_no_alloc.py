"""The allocation-free exact in-out entry point (inout_classify_static, the
surface staged in the library's static device array) against inout_classify
on the same inputs: labels bit-exact, on two calls in a row with the second
one smaller (fewer points, a smaller surface), so that the second call reuses
an array that still holds the first call's staging. A surface too large for
the array is refused before any launch."""
import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu


def _points(surf, n, seed):
    rng = np.random.default_rng(seed)
    lo, hi = surf.verts.min(0), surf.verts.max(0)
    pad = 0.2 * (hi - lo)
    p = rng.uniform(lo - pad, hi + pad, size=(n, 3))
    # a share of the points close to the surface (near vertices, both sides)
    k = n // 3
    v = surf.verts[rng.integers(0, surf.verts.shape[0], k)]
    p[:k] = v + rng.normal(scale=1e-3 * (hi - lo).max(), size=(k, 3))
    return p


def test_static_scratch_matches_inout_classify():
    import torch
    from paper_2009_00706_amd import vms
    assert torch.cuda.is_available()
    vms.lib()
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    cases = [(I.icosphere(4, 0.3, c), 200_000, 1), (I.icosphere(2, 0.2, c), 30_001, 2)]
    for surf, n, seed in cases:
        p = _points(surf, n, seed)
        px, py, pz = (torch.as_tensor(np.ascontiguousarray(p[:, k]), device="cuda") for k in range(3))
        ref = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
        got = torch.full((n,), 9, dtype=torch.uint8, device="cuda")
        print(f"surface {surf.n_tri} triangles, {n} points", flush=True)
        vms.inout_classify(surf, px, py, pz, ref)
        vms.inout_classify_static(surf, px, py, pz, got)
        torch.cuda.synchronize()
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        assert set(np.unique(r)) <= {0, 1}
        assert 0 < r.sum() < n
        assert np.array_equal(g, r)


def test_static_scratch_rejects_a_surface_above_its_size():
    import torch
    from paper_2009_00706_amd import vms
    c = tuple(0.5 + o for o in I.BODY_OFFSET)
    big = I.icosphere(7, 0.3, c)              # 327,680 triangles: about 40 MB of staging
    px = torch.zeros(4, dtype=torch.float64, device="cuda")
    lab = torch.full((4,), 5, dtype=torch.uint8, device="cuda")
    with pytest.raises(vms.VmsError) as e:
        vms.inout_classify_static(big, px, px, px, lab)
    assert e.value.code == vms.VMS_EOVERFLOW
    torch.cuda.synchronize()
    assert (lab.cpu().numpy() == 5).all()      # nothing was launched
