"""Learned in-out filter on the GPU: gradients and Adam against the FP64
reference network, FP16-MFMA inference, exact signed-distance sampler, and
bit-exact labels of the filtered classification (with the gain it brings)."""
import time

import numpy as np
import pytest

from paper_2009_00706_amd import inputs as I

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, 0.0])
HI = np.array([1.0, 1.0, 1.0])


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available()
    from paper_2009_00706_amd import vms
    vms.lib()
    return torch, vms


def dev_xyz(torch, pts):
    x = torch.as_tensor(np.ascontiguousarray(pts, np.float64), device="cuda")
    return x[:, 0].contiguous(), x[:, 1].contiguous(), x[:, 2].contiguous()


def test_gradient_and_adam_match_reference(env):
    torch, vms = env
    from oracle import mlp as M
    th = M.init_params(7).astype(np.float32)
    B = M.fourier_matrix(7, 2.0).astype(np.float32)
    rng = np.random.default_rng(3)
    x = rng.uniform(LO, HI, (1000, 3))
    sdf = rng.normal(0, 0.05, 1000)
    T = 0.05
    h = vms.vms_mlp_create(LO, HI, th, B, T)
    px, py, pz = dev_xyz(torch, x)
    g = torch.zeros(M.N_PARAMS, dtype=torch.float32, device="cuda")
    loss = vms.vms_mlp_grad(h, px, py, pz, torch.as_tensor(sdf, device="cuda"), g)
    ref_loss, ref_g = M.loss_and_grad(th.astype(np.float64), x, sdf, LO, HI, B.astype(np.float64), T)
    gg = g.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(gg - ref_g) / np.linalg.norm(ref_g)
    print(f"gradient rel err {err:.2e}, loss {loss:.6e} vs {ref_loss:.6e}")
    assert err <= 1e-5
    assert abs(loss - ref_loss) <= 1e-6 * ref_loss
    # one Adam step from zero moments
    vms.vms_mlp_adam_step(h, g, 1e-3)
    t1 = vms.vms_mlp_get_params(h).astype(np.float64)
    ref_t1, _, _ = M.adam_step(th.astype(np.float64), gg, np.zeros_like(gg), np.zeros_like(gg), 1, 1e-3)
    assert np.abs(t1 - ref_t1).max() <= 1e-6
    vms.vms_mlp_destroy(h)


def test_fp16_inference_close_to_reference(env):
    torch, vms = env
    from oracle import mlp as M
    th = M.init_params(11).astype(np.float32)
    B = M.fourier_matrix(11, 2.0).astype(np.float32)
    h = vms.vms_mlp_create(LO, HI, th, B, 0.05)
    rng = np.random.default_rng(5)
    x = rng.uniform(LO, HI, (5000, 3))
    px, py, pz = dev_xyz(torch, x)
    pred = torch.empty(5000, dtype=torch.float32, device="cuda")
    vms.vms_mlp_predict(h, px, py, pz, pred)
    ref = M.forward(th.astype(np.float64), x, LO, HI, B.astype(np.float64))
    err = np.abs(pred.cpu().numpy() - ref)
    print(f"fp16 inference max abs err {err.max():.2e} (output scale {np.abs(ref).max():.2e})")
    assert err.max() <= 2e-2 * max(1.0, np.abs(ref).max())
    vms.vms_mlp_destroy(h)


def test_exact_sdf_sampler(env, oracle):
    torch, vms = env
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.icosphere(3, 0.2, c)
    pts = I.sdf_sample_points(s, LO, HI, 3000, 2, near_dist=0.1)
    hio = vms.inout_prepare(s)
    px, py, pz = dev_xyz(torch, pts)
    out = torch.empty(3000, dtype=torch.float64, device="cuda")
    T = 0.08
    vms.vms_sdf_sample(hio, px, py, pz, T, out)
    got = out.cpu().numpy()
    d = np.minimum(oracle.unsigned_distance(s, pts), T)
    lab, _ = oracle.label_points(s, pts)
    ref = np.where(lab == 1, -d, d)
    assert np.array_equal(np.signbit(got) | (got == 0), (lab == 1) | (d == 0))
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-15)
    vms.inout_release(hio)


def test_learned_labels_bit_exact_and_gain(env, oracle):
    """Train on exact distances, calibrate the margin on held-out points drawn like
    the queries, then classify new points: labels equal the exact ones; report the
    fraction decided by the network and the throughput against the exact test."""
    torch, vms = env
    from paper_2009_00706_amd.learned import LearnedFilter
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.icosphere(4, 0.1, c)
    lf = LearnedFilter(s, trunc=0.05, seed=0, sigma=1.0)
    loss = lf.train(1_000_000, steps=8000, batch=8192, lr=3e-3)
    # queries: points within a few element sizes of the surface, as sub-cell points are
    held = I.sdf_sample_points(s, LO, HI, 200_000, 11, near_frac=0.9, near_dist=0.02)
    m, err = lf.calibrate(held)
    q = I.sdf_sample_points(s, LO, HI, 1_000_000, 12, near_frac=0.9, near_dist=0.02)
    exact = lf.classify(q, learned=False)
    learned = lf.classify(q, learned=True)
    torch.cuda.synchronize()
    assert torch.equal(exact, learned)
    ref, _ = oracle.label_points(s, q[:20000])
    assert np.array_equal(exact[:20000].cpu().numpy(), ref)
    # gain: fraction decided by the network and time per classification
    pred = lf.predict(q).cpu().numpy()
    decided = float(np.mean(np.abs(pred) >= m))
    tt = {}
    for mode in (False, True):
        for _ in range(2):
            lf.classify(q, learned=mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            lf.classify(q, learned=mode)
        torch.cuda.synchronize()
        tt[mode] = (time.perf_counter() - t0) / 5
    print(f"train loss {loss:.3e}, margin {m:.3e}, decided by network {decided:.3f}, "
          f"exact {tt[False]*1e3:.2f} ms, learned {tt[True]*1e3:.2f} ms, gain {tt[False]/tt[True]:.2f}x")
    assert decided > 0.5
    lf.close()


def test_learned_filter_inside_the_assembly(env, oracle):
    """The learned filter in front of the exact test of the sub-cell quadrature
    (vms_params.inout_mode / vms_set_inout): a surface much finer than the
    elements (81,920 triangles, many background triangles per element). The
    relabelled sub-cell points, the CSR values and the residual equal those of
    the exact mode bit for bit, and the points of a sample of INTERCEPTED
    elements equal the reference's. The relabel time is reported for several
    thresholds on the element's background-triangle count (the network is used
    only at or above it) and the best one is kept: where the network loses, it
    is switched off."""
    torch, vms = env
    from paper_2009_00706_amd.learned import LearnedFilter
    c = np.array([0.5, 0.5, 0.5]) + I.BODY_OFFSET
    s = I.icosphere(6, 0.2, c)
    tree = I.sphere_refined_octree(tuple(c), 0.2, 3, 6, 1.5)
    lf = LearnedFilter(s, trunc=0.05, seed=0, sigma=1.0)
    loss = lf.train(1_000_000, steps=8000, batch=8192, lr=3e-3)
    held = I.sdf_sample_points(s, LO, HI, 2_000_000, 11, near_frac=0.9, near_dist=0.03)
    m, _ = lf.calibrate(held, grid=(16, 16, 16))
    print(f"{tree.n} octants, {s.n_tri} triangles: train loss {loss:.2e}, margin {m:.2e}", flush=True)
    prm = vms.make_params(quad_depth=3)
    ex = vms.Assembler(tree, s, prm)
    ln = vms.Assembler(tree, s, vms.make_params(quad_depth=3, inout_mode=vms.VMS_INOUT_LEARNED))
    vms.vms_set_inout(ln.ctx, vms.VMS_INOUT_LEARNED, lf.net, 0)
    xyz = ex.export(vms.VMS_EXPORT_NODE_XYZ).T / float(1 << tree.max_level)
    f = I.make_fields(xyz, 1000)
    for a in (ex, ln):
        a.set_fields(f)
        a.assemble(flags=vms.VMS_RELABEL)
    torch.cuda.synchronize()
    vms.vms_sizes(ln.ctx)                     # raises on a kept-point count changed by the relabel
    ge, gl = ex.export(vms.VMS_EXPORT_SUBGP), ln.export(vms.VMS_EXPORT_SUBGP)
    for k in ("el", "key", "lvl", "xyz"):
        assert np.array_equal(ge[k], gl[k]), k
    assert torch.equal(ex.vals, ln.vals) and torch.equal(ex.resid, ln.resid)
    rs = vms.vms_relabel_stats(ln.ctx)
    decided = 1.0 - rs["exact_in_last_relabel"] / rs["candidates"]
    print(f"{rs['candidates']} candidate points, decided by the network: {decided:.3f}", flush=True)
    assert decided > 0.2
    # the reference's points on a sample of INTERCEPTED elements
    mk = ex.export(vms.VMS_EXPORT_MARKERS)
    cut = np.nonzero(mk == 2)[0]
    pick = np.sort(np.random.default_rng(3).choice(cut, min(40, cut.size), replace=False))
    ref = oracle.subquad(tree, s, pick, 3)
    sel = np.isin(gl["el"], pick)
    for k in ("el", "key", "lvl", "xyz"):
        assert np.array_equal(gl[k][sel], ref[k]), k
    # relabel time by threshold on the background-triangle count
    vms.vms_set_timing(ln.ctx, True)
    vms.vms_set_timing(ex.ctx, True)

    def relabel_ms(a):
        for _ in range(2):
            a.assemble(flags=vms.VMS_RELABEL)
        t = []
        for _ in range(5):
            a.assemble(flags=vms.VMS_RELABEL)
            t.append(vms.vms_last_timing(a.ctx)[0])
        return float(np.median(t))

    t_exact = relabel_ms(ex)
    times = {}
    for tb in (0, 16, 32, 64, 128, 1 << 30):
        # each new threshold rebuilds the element lists of the learned relabel,
        # which runs on the second stream of the overlapped schedule: the
        # outputs must stay those of the exact mode after every rebuild
        vms.vms_set_inout(ln.ctx, vms.VMS_INOUT_LEARNED, lf.net, tb)
        times[tb] = relabel_ms(ln)
        torch.cuda.synchronize()
        vms.vms_sizes(ln.ctx)
        assert torch.equal(ex.vals, ln.vals) and torch.equal(ex.resid, ln.resid), tb
    best = min(times, key=times.get)
    print(f"relabel: exact {t_exact:.3f} ms; learned by threshold "
          + ", ".join(f"{k}: {v:.3f}" for k, v in times.items())
          + f"; best threshold {best} ({t_exact / times[best]:.2f}x)", flush=True)
    # with the threshold above every element the learned mode is the exact one
    assert times[1 << 30] <= 1.1 * t_exact + 0.01
    ex.close()
    ln.close()
    lf.close()
