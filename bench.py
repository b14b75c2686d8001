"""Benchmark of the VMS assembly + in-out hot path on one MI355X.

One step = vms_assemble with relabelling: adaptive sub-cell quadrature of every
INTERCEPTED element with an exact in-out test of each candidate point, then the
residual and Jacobian of every non-IN element summed from element records into
the CSR and the residual (identity rows included). Inputs are resident in HBM
before the timed region. Prints one JSON line.

Workloads:
  twoboxes  (default) two filleted bluff boxes 1.0 x 0.25 x 0.3 (fillet 0.03,
            gap 0.5, 198,744 triangles) in an 8 x 2 x 2 domain, octree levels
            6-11 refined at the surfaces (10.2M octants, 3.37e9 CSR nonzeros),
            sub-cell quadrature depth 3. FP64 headline; the BF16 and FP16 forms
            and the learned + mixed form (network trained on 4M exact distances
            in front of the exact in-out test) timed on the same inputs.
  sphere    immersed sphere r = 0.1 (icosphere, 5120 triangles) at the unit
            cube's centre, octree levels 5-8 refined at the surface (194,328
            octants, hanging nodes), sub-cell quadrature depth 3.
  precision the sphere at levels 6-10 (2.1M octants).
  uniform16 16^3 uniform octants, no body.
  batch64   64 independent octrees (log-uniform 1e4..5e5 octants, one ellipsoid
            body each) assembled by one persistent launch, autotuned, replayed
            as a captured graph; BF16 form by default. Labels are computed at
            context creation; a step is the assembly.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# algorithmic work per quadrature point: the dense B^T D B contraction,
# (16x4x32 + 32x4x32) multiply-adds x 2 = 12,288 flop; an OUT element has 8
# points, an INTERCEPTED element its kept sub-cell points
FLOP_PER_POINT = 12288
PEAK_FP64_TFLOPS = 78.6     # FP64 vector and FP64 MFMA
PEAK_FP32_TFLOPS = 157.3    # FP32 vector (the mixed forms' per-point and stage-1 work)
PEAK_HBM_GBS = 8000.0       # HBM3E
BATCH_SEED = 1003           # seed of the 64-tree batch workload


_T0 = time.perf_counter()


def log(msg):
    """Progress on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="twoboxes",
                    choices=["sphere", "uniform16", "precision", "twoboxes", "batch64", "q2uniform16"])
    ap.add_argument("--precision", default=None, choices=["fp64", "bf16", "fp16"])
    ap.add_argument("--n-trees", type=int, default=64)
    ap.add_argument("--no-forms", action="store_true", help="skip the BF16/FP16 comparison")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned + mixed step")
    ap.add_argument("--no-scatter", action="store_true", help="skip the atomic-scatter comparison")
    ap.add_argument("--no-normal", action="store_true", help="skip the normal-based filter comparison")
    ap.add_argument("--no-classify", action="store_true", help="skip the standalone in-out classification rate")
    ap.add_argument("--learned-standalone", action="store_true",
                    help="also time the learned filter on the kept sub-cell points outside the assembly")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1500, help="leaves drawn for the oracle sample")
    ap.add_argument("--cpu-workers", type=int, default=16,
                    help="processes of the all-core oracle run (the GPU's share of host cores)")
    ap.add_argument("--cost-model", default="none", choices=["precision", "small", "none"],
                    help="workload on which the eq. (Wpart) cost model predicts the kernel time")
    ap.add_argument("--no-jv", action="store_true",
                    help="skip the Jacobian-product section (matrix-free action and CSR product)")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--traffic", default=os.path.join(ROOT, "profiles", "traffic.json"))
    return ap.parse_args()


def copy_calibration(mib):
    import torch
    n = mib * (1 << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 8, "bytes_written": n * 8, "launches": 3}))


def workload(name):
    from paper_2009_00706_amd import inputs as I
    if name == "uniform16":
        return I.uniform_octree(4), None, {
            "workload": "uniform 16^3 octants on the unit cube (4096 OUT elements, 4913 nodes)",
            "octants": 4096}
    if name == "precision":
        tree, surf = I.sphere_workload(lmin=6, lmax=10, beta=3.0)
        return tree, surf, {
            "workload": "immersed sphere r=0.1 (icosphere 4, 5120 triangles), octree levels 6-10 "
                        f"refined at the surface ({tree.n} octants), sub-cell quadrature depth 3",
            "octants": tree.n}
    if name == "twoboxes":
        tree, surf = I.two_box_workload()
        return tree, surf, {
            "workload": "two filleted bluff boxes 1.0x0.25x0.3 (fillet 0.03, gap 0.5, "
                        f"{surf.tris.shape[0]} triangles) in an 8x2x2 domain, octree levels 6-11 "
                        f"refined at the surfaces ({tree.n} octants), sub-cell quadrature depth 3",
            "octants": tree.n, "shortest_side": 2.0, "learned_train_samples": 4_000_000}
    tree, surf = I.sphere_workload()
    return tree, surf, {
        "workload": "immersed sphere r=0.1 (icosphere 4, 5120 triangles), octree levels 5-8 "
                    f"refined at the surface ({tree.n} octants), sub-cell quadrature depth 3",
        "octants": tree.n}


def node_xyz(vms, ctx, tree):
    return vms.vms_export(ctx, vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64) / \
        float(1 << tree.max_level) * tree.root_len + np.asarray(tree.origin)


# the sources of the element kernel: the recorded traffic holds for this text only
KERNEL_SOURCES = ("assemble2.hip", "kernels.h", "geom.h", "vms_point.h")


def traffic_for(path, workload, precision):
    """HBM bytes per launch of the dominant kernel from the recorded counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy calibration); None when no
    record exists or the kernel source changed since the counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    try:
        tr = json.load(open(path))
        src = b"".join(open(os.path.join(ROOT, "paper_2009_00706_amd", "csrc", f), "rb").read()
                       for f in KERNEL_SOURCES)
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(src).hexdigest()[:16]
    for e in tr.get("entries", []):
        if e.get("workload") == workload and e.get("precision") == precision and \
                e.get("kernel_source_sha256_16") == sha:
            return e.get("bytes_per_launch")
    return None


def _cpu_info():
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


_BASE = {}


def _baseline_work(_=None):
    """The timed oracle work of the CPU baseline (sub-cell quadrature with exact
    labels of the sampled INTERCEPTED elements, then the residual and Jacobian
    of every sampled element); returns its wall time."""
    from oracle import core as O
    b = _BASE
    t0 = time.perf_counter()
    sq = O.subquad(b["sub"], b["surf"], b["cut"], 3) if b["cut"].size else None
    O.assemble(b["sub"], b["ms"], b["f"], mk=b["mk"], sub=sq, depth=3, subset=b["els"])
    return time.perf_counter() - t0


def cpu_baseline(tree, surf, n_sample, shortest_side=1.0, workers=16, seed=0):
    """The CPU reference as it stands, on a bounded sample of the workload: leaves
    drawn at random (seed 0), IN ones dropped (exact corner labels), each
    assembled in the window of leaves around it (its neighbours decide its
    hanging corners). Timed: the sub-cell quadrature with exact labels of the
    INTERCEPTED ones and the residual and Jacobian of all, once in one process,
    then the same work in `workers` processes at once (all cores). Set-up (the
    windows' meshes, corner labels, fields at the window's nodes) is not timed,
    as the GPU's set-up is not. Runs before the GPU is touched (forks)."""
    import multiprocessing as mp
    from oracle import core as O
    from oracle import window as W
    from paper_2009_00706_amd import inputs as I
    rng = np.random.default_rng(seed)
    pick = np.sort(rng.choice(tree.n, min(tree.n, n_sample), replace=False))
    index = W.LeafIndex(tree)
    sel = set(pick.tolist())
    for e in pick:
        sel.update(W.element_window(index, e).tolist())
    L = np.array(sorted(sel), np.int64)
    sub = W.subset(tree, L)
    ms = O.derive_mesh(sub.ax, sub.ay, sub.az, sub.level, sub.max_level)
    loc = np.searchsorted(L, pick)
    mk = np.zeros(sub.n, np.uint8)
    if surf is not None:
        # exact labels of the sampled elements' corners decide their markers
        cv = ms.elem_vertex[loc].ravel()
        vx = O.vertex_xyz(sub, ms)
        lab, _ = O.label_points(surf, vx[cv])
        cnt = lab.reshape(-1, 8).astype(np.int64).sum(1)
        mk[loc] = np.where(cnt == 8, O.IN, np.where(cnt == 0, O.OUT, O.INTERCEPTED))
    keep = loc[mk[loc] != O.IN]
    xyz = ms.node_xyz_int.astype(np.float64) / float(1 << sub.max_level) * sub.root_len + \
        np.asarray(sub.origin)
    f = I.make_fields(xyz, 1001, shortest_side)
    _BASE.update(sub=sub, surf=surf, ms=ms, mk=mk, f=f, els=keep,
                 cut=keep[mk[keep] == O.INTERCEPTED])
    n = int(keep.size)
    n_cut = int(_BASE["cut"].size)
    O.lib()
    t1 = _baseline_work()
    workers = max(1, min(workers, os.cpu_count() or 1))
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        times = pool.map(_baseline_work, range(workers))
        tall = time.perf_counter() - t0
    _BASE.clear()
    model, ncpu = _cpu_info()
    return {"value": workers * n / tall, "unit": "elements/s", "cores": workers, "kind": "oracle",
            "single_core_value": n / t1, "single_core_s": t1, "all_core_wall_s": tall,
            "cpu_model": model, "nproc": ncpu,
            "sample": f"{n - n_cut} OUT + {n_cut} INTERCEPTED elements of this workload (leaves drawn at "
                      f"random, seed {seed}, IN ones dropped), each in its window of neighbouring leaves; "
                      f"timed: sub-cell quadrature with exact labels + residual and Jacobian; "
                      f"{t1:.1f} s in one process; the same work in {workers} processes at once "
                      f"({tall:.1f} s wall, value = {workers} x sample / wall)"}


def active_rows(vms, asm):
    """Rows of active nodes (nodes of non-IN elements); the others are identity rows."""
    mk = asm.export(vms.VMS_EXPORT_MARKERS)
    ma = asm.export(vms.VMS_EXPORT_MASTERS)[mk != 1]
    act = np.zeros(asm.sizes["n_nodes"], bool)
    act[ma[ma >= 0]] = True
    return np.repeat(act, 4)


def run_single(torch, vms, tree, surf, f, prec, steps, warmup, flags, params=None, prepare=None,
               atomic=False):
    """Time `steps` whole steps of one context; returns numbers and the outputs.
    params: vms_params (default: depth 3 at precision prec); prepare(asm) runs
    after the fields are set and before the warm-up."""
    t_setup = time.perf_counter()
    asm = vms.Assembler(tree, surf, params or vms.make_params(quad_depth=3, precision=prec))
    setup_s = time.perf_counter() - t_setup
    asm.set_fields(f)
    extra = prepare(asm) if prepare else None
    st = vms.vms_stats(asm.ctx)
    n_active = st["n_out"] + st["n_intercepted"]
    vms.vms_set_timing(asm.ctx, True)
    for _ in range(warmup):
        asm.assemble(flags=flags)
    torch.cuda.synchronize()
    stage = np.zeros((steps, 5))
    t0 = time.perf_counter()
    for k in range(steps):
        asm.assemble(flags=flags)
        stage[k] = vms.vms_last_timing(asm.ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same step in order (every stage alone on the context stream): the
    # isolated stage times and what the overlapped schedule gains
    vms.vms_set_overlap(asm.ctx, False)
    n_io = min(steps, 5)
    asm.assemble(flags=flags)
    torch.cuda.synchronize()
    stage_io = np.zeros((n_io, 5))
    t2 = time.perf_counter()
    for k in range(n_io):
        asm.assemble(flags=flags)
        stage_io[k] = vms.vms_last_timing(asm.ctx)
    torch.cuda.synchronize()
    ms_io = 1e3 * (time.perf_counter() - t2) / n_io
    vms.vms_set_overlap(asm.ctx, True)
    # steady state (labels cached), for context
    t1 = time.perf_counter()
    for _ in range(steps):
        asm.assemble(flags=0)
    torch.cuda.synchronize()
    steady = n_active * steps / (time.perf_counter() - t1)
    asm.assemble(flags=flags)
    torch.cuda.synchronize()
    relabel = vms.vms_relabel_stats(asm.ctx) if surf is not None else None
    vms.vms_sizes(asm.ctx)   # raises if a relabel changed an element's kept-point count
    # device time of each timed step: the stages on the context stream (the
    # relabel and INTERCEPTED stages of an overlapped step ran beside the last)
    over = overlapped(st) and not atomic
    dev = stage[:, 1] + stage[:, 2] + stage[:, 4] if over else stage.sum(1)
    out = {"elapsed": elapsed, "value": n_active * steps / elapsed, "ms_step": 1e3 * elapsed / steps,
           "step_device_ms": {"p10": float(np.percentile(dev, 10)), "p50": float(np.median(dev)),
                              "p90": float(np.percentile(dev, 90))},
           "stage": stage.mean(0), "stage_in_order": stage_io.mean(0), "ms_step_in_order": ms_io,
           "overlapped": over, "steady": steady, "setup_s": setup_s, "stats": st,
           "sizes": asm.sizes, "n_active": n_active, "relabel": relabel, "extra": extra,
           "vals": asm.vals, "resid": asm.resid, "inactive": inactive_entries(torch, vms, asm)}
    asm.close()
    return out


def overlapped(st):
    """Whether vms_assemble (matrix, overlap on) takes the overlapped schedule."""
    return st["n_intercepted"] > 0 or st.get("n_surfgp", 0) > 0


def stage_dict(avg, over=False):
    if over:
        return {"relabel_beside": float(avg[0]), "args": float(avg[1]), "out_elements": float(avg[2]),
                "intercepted_elements_beside": float(avg[3]), "after_out_elements": float(avg[4]),
                "note": "overlapped step: relabel and INTERCEPTED items on the second stream, beside "
                        "the span after the OUT kernel (gather of the other blocks, then the late "
                        "blocks and the residual); device step = args + OUT + that span"}
    return {"relabel": float(avg[0]), "args": float(avg[1]), "out_elements": float(avg[2]),
            "intercepted_elements": float(avg[3]), "csr_gather": float(avg[4])}


def schedule_info(m):
    return {"stage_ms_in_order": stage_dict(m["stage_in_order"]), "ms_per_step_in_order": m["ms_step_in_order"],
            "overlap_speedup": m["ms_step_in_order"] / m["ms_step"]}


def train_filter(torch, surf, n_train):
    """The learned in-out filter: network trained by the library's kernels on
    exact clamped distances, per-cell margins calibrated on held-out points
    drawn like the sub-cell quadrature's candidates (near the surface)."""
    from paper_2009_00706_amd import inputs as I
    from paper_2009_00706_amd.learned import LearnedFilter
    t0 = time.perf_counter()
    lf = LearnedFilter(surf, trunc=0.05, seed=0, sigma=1.0)
    loss = lf.train(n_train, steps=8000, batch=8192, lr=3e-3)
    lo, hi = surf.verts.min(0) - 0.2, surf.verts.max(0) + 0.2
    held = I.sdf_sample_points(surf, lo, hi, 2_000_000, 21, near_frac=0.9, near_dist=0.02)
    ext = hi - lo
    grid = tuple(int(max(4, round(32 * e / ext.max()))) for e in ext)
    margin, _ = lf.calibrate(held, grid=grid)
    torch.cuda.synchronize()
    return lf, {"train_samples": n_train, "train_loss": loss, "global_margin": margin,
                "margin_grid": list(grid), "train_and_calibrate_s": time.perf_counter() - t0}


def normal_filter(torch, vms, tree, surf, f, reps=7):
    """The normal-based test of Alg. 5 as a certified filter (VMS_INOUT_NORMAL)
    against the exact test alone: relabel time (in-order schedule, HIP events),
    share of the candidate points the filter decides, bodies and convexity."""
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    asm.set_fields(f)
    vms.vms_set_timing(asm.ctx, True)
    vms.vms_set_overlap(asm.ctx, False)
    out = {}
    for name, mode in (("exact", vms.VMS_INOUT_EXACT), ("normal", vms.VMS_INOUT_NORMAL)):
        vms.vms_set_inout(asm.ctx, mode)
        for _ in range(2):
            asm.assemble(flags=vms.VMS_RELABEL)
        t = []
        for _ in range(reps):
            asm.assemble(flags=vms.VMS_RELABEL)
            t.append(vms.vms_last_timing(asm.ctx)[0])
        rs = vms.vms_relabel_stats(asm.ctx)
        out[name] = {"relabel_ms": float(np.median(t)),
                     "decided_by_filter": 1.0 - rs["exact_in_last_relabel"] / max(rs["candidates"], 1)}
    n, convex = vms.vms_components(asm.ctx)
    vms.vms_sizes(asm.ctx)   # raises if a relabel changed a kept-point count
    asm.close()
    out["bodies"] = int(n)
    out["convex"] = [bool(x) for x in convex]
    out["speedup"] = out["exact"]["relabel_ms"] / out["normal"]["relabel_ms"]
    return out


def classify_rate(torch, vms, tree, surf, reps=5):
    """Exact in-out tests per second of the standalone classification
    (inout_classify_prepared: bin grid of the surface, ray parity along x with exact
    predicates) on the workload's kept sub-cell points, against the labels of
    the adaptive quadrature (all OUT), HIP events on the handle's stream."""
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    xyz = asm.export(vms.VMS_EXPORT_SUBGP)["xyz"]
    asm.close()
    n = int(xyz.shape[0])
    cols = [torch.as_tensor(np.ascontiguousarray(xyz[:, k]), device="cuda") for k in range(3)]
    del xyz
    lab = torch.full((n,), 7, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()   # the copies and the fill ran on torch's stream
    stream = torch.cuda.Stream()
    h = vms.inout_prepare(surf, stream.cuda_stream)
    try:
        vms.inout_classify_prepared(h, *cols, lab)
        stream.synchronize()
        all_out = bool((lab == 0).all())
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            vms.inout_classify_prepared(h, *cols, lab)
        b.record(stream)
        b.synchronize()
        ms = a.elapsed_time(b) / reps
    finally:
        vms.inout_release(h)
    return {"points": n, "exact_tests_per_s": n / (ms * 1e-3), "ms_per_call": ms,
            "labels_all_out": all_out,
            "note": "the kept sub-cell points of the workload, classified one by one without their "
                    "elements (the quadrature's own tests are the top-level inout_tests_per_s)"}


def learned_threshold(torch, vms, asm, lf, thresholds=(0, 16, 32, 64, 128, 1 << 30), reps=5):
    """Relabel time of the learned mode for each threshold on the element's
    background-triangle count (the network is used at or above it), and of the
    exact mode; the fastest setting is kept (the network is switched off where
    it loses). The relabel is timed alone (in-order schedule)."""
    vms.vms_set_timing(asm.ctx, True)
    vms.vms_set_overlap(asm.ctx, False)

    def relabel_ms():
        for _ in range(2):
            asm.assemble(flags=vms.VMS_RELABEL)
        t = []
        for _ in range(reps):
            asm.assemble(flags=vms.VMS_RELABEL)
            t.append(vms.vms_last_timing(asm.ctx)[0])
        return float(np.median(t))

    vms.vms_set_inout(asm.ctx, vms.VMS_INOUT_EXACT)
    t_exact = relabel_ms()
    times = {}
    for tb in thresholds:
        vms.vms_set_inout(asm.ctx, vms.VMS_INOUT_LEARNED, lf.net, tb)
        times[tb] = relabel_ms()
        times[tb] = {"relabel_ms": times[tb], "decided_by_network": None}
        rs = vms.vms_relabel_stats(asm.ctx)
        times[tb]["decided_by_network"] = 1.0 - rs["exact_in_last_relabel"] / max(rs["candidates"], 1)
    best = min(times, key=lambda k: times[k]["relabel_ms"])
    vms.vms_set_inout(asm.ctx, vms.VMS_INOUT_LEARNED, lf.net, best)
    vms.vms_set_overlap(asm.ctx, True)
    return {"exact_relabel_ms": t_exact, "by_min_bt": {str(k): v for k, v in times.items()},
            "min_bt": best, "gain_vs_exact_relabel": t_exact / times[best]["relabel_ms"]}


def learned_inout(torch, vms, tree, surf, n_train=1_000_000):
    """In-out classification of the workload's kept sub-cell points with and
    without the learned filter (network trained by the library's kernels on
    exact clamped distances, per-cell margins): labels must agree exactly."""
    from paper_2009_00706_amd import inputs as I
    from paper_2009_00706_amd.learned import LearnedFilter
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    pts = asm.export(vms.VMS_EXPORT_SUBGP)["xyz"]
    asm.close()
    t0 = time.perf_counter()
    lf = LearnedFilter(surf, trunc=0.05, seed=0, sigma=1.0)
    lf.train(n_train, steps=8000, batch=8192, lr=3e-3)
    lo, hi = surf.verts.min(0) - 0.1, surf.verts.max(0) + 0.1
    held = I.sdf_sample_points(surf, lo, hi, 2_000_000, 11, near_frac=0.9, near_dist=0.02)
    lf.calibrate(held, grid=(16, 16, 16))
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    exact = lf.classify(pts, learned=False)
    learned = lf.classify(pts, learned=True)
    torch.cuda.synchronize()
    same = bool(torch.equal(exact, learned))
    tt = {}
    for mode in (False, True):
        lf.classify(pts, learned=mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            lf.classify(pts, learned=mode)
        torch.cuda.synchronize()
        tt[mode] = (time.perf_counter() - t1) / 5
    # general queries drawn like the training set (90% within 0.02 of the surface)
    q = I.sdf_sample_points(surf, lo, hi, 2_000_000, 12, near_frac=0.9, near_dist=0.02)
    qe, ql = lf.classify(q, learned=False), lf.classify(q, learned=True)
    torch.cuda.synchronize()
    q_same = bool(torch.equal(qe, ql))
    tq = {}
    for mode in (False, True):
        lf.classify(q, learned=mode)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            lf.classify(q, learned=mode)
        torch.cuda.synchronize()
        tq[mode] = (time.perf_counter() - t1) / 5
    lf.close()
    return {"points": int(pts.shape[0]), "labels_equal": same,
            "exact_tests_per_s": pts.shape[0] / tt[False], "learned_tests_per_s": pts.shape[0] / tt[True],
            "gain": tt[False] / tt[True], "train_and_calibrate_s": train_s,
            "queries": {"points": int(q.shape[0]), "labels_equal": q_same,
                        "exact_tests_per_s": q.shape[0] / tq[False],
                        "learned_tests_per_s": q.shape[0] / tq[True], "gain": tq[False] / tq[True],
                        "sample": "90% within 0.02 of the surface, the rest uniform in its box grown by 0.1"},
            "note": "kept sub-cell points of the workload; exact: ray parity along x with exact predicates; "
                    "learned: FP16-MFMA network, exact test inside the per-cell margin"}


def inactive_entries(torch, vms, asm):
    """CSR positions of the rows of inactive nodes: each such node has only its
    diagonal block, so its 16 entries are contiguous from its first row."""
    act = active_rows(vms, asm)[::4]
    rp = asm.export(vms.VMS_EXPORT_ROW_PTR)
    first = rp[4 * np.nonzero(~act)[0]]
    return torch.as_tensor((first[:, None] + np.arange(16)).ravel(), device=asm.vals.device)


def _sq_sum(a, b=None, chunk=1 << 27):
    """sum of squares of a (or of a - b), in float64, chunk by chunk on the device"""
    s = 0.0
    for i in range(0, a.numel(), chunk):
        d = a[i:i + chunk].double() if b is None else a[i:i + chunk].double() - b[i:i + chunk].double()
        s += float((d * d).sum())
    return s


def form_errors(torch, m, r):
    """Normwise errors of a mixed form against FP64 over the rows of active
    nodes; the identity rows of inactive nodes must agree exactly."""
    ina = r["inactive"]
    mi, ri = m["vals"][ina].double(), r["vals"][ina].double()
    assert torch.equal(mi, ri)
    ref_all, diff_all = _sq_sum(r["vals"]), _sq_sum(m["vals"], r["vals"])
    ref_act = ref_all - float((ri * ri).sum())
    er = (torch.linalg.vector_norm(m["resid"] - r["resid"]) / torch.linalg.vector_norm(r["resid"])).item()
    return {"rel_err_jacobian": (diff_all / ref_act) ** 0.5,
            "rel_err_jacobian_all_entries": (diff_all / ref_all) ** 0.5, "rel_err_residual": er}


def jacobian_products(torch, vms, tree, surf, f, prec, reps=20):
    """The two ways to apply the Jacobian inside a Krylov solver: the
    matrix-free action (no matrix) and the CSR product with the assembled
    matrix; device time per product with HIP events on the context stream."""
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
    asm.set_fields(f)
    x = torch.as_tensor(np.random.default_rng(5).normal(size=asm.sizes["n_rows"]), device="cuda")
    y1, y2 = torch.empty_like(x), torch.empty_like(x)

    def timed(fn):
        for _ in range(3):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(asm.stream)
        for _ in range(reps):
            fn()
        b.record(asm.stream)
        b.synchronize()
        return a.elapsed_time(b) / reps

    t_asm = timed(lambda: asm.assemble())
    t_mf = timed(lambda: asm.jacobian_action(x, y1))
    t_sp = timed(lambda: asm.spmv(x, y2))
    act = torch.as_tensor(active_rows(vms, asm), device=x.device)
    assert torch.equal(y1[~act], y2[~act])  # identity rows
    diff = (torch.linalg.vector_norm((y1 - y2)[act]) / torch.linalg.vector_norm(y2[act])).item()
    nnz, n_rows, n_nodes = asm.sizes["nnz"], asm.sizes["n_rows"], asm.sizes["n_nodes"]
    vb = 8 if prec == vms.VMS_FP64 else 4
    # algorithmic bytes of one product: values, block columns, block-row offsets,
    # x and y once each
    sp_bytes = nnz * vb + (nnz // 16) * 4 + (n_nodes + 1) * 8 + 2 * n_rows * 8
    gbs = sp_bytes / (t_sp * 1e-3) / 1e9
    asm.close()
    return {"matrix_free_ms": t_mf, "spmv_ms": t_sp, "assembly_ms": t_asm,
            "rel_diff_matrix_free_vs_spmv": diff,  # over the rows of active nodes
            "products_before_assembly_pays": t_asm / max(t_mf - t_sp, 1e-9),
            "spmv_roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                              "frac": gbs / PEAK_HBM_GBS, "bytes_per_launch": sp_bytes,
                              "kernel": "k_bspmv"},
            "note": "y = J x: matrix-free = residual integrand differentiated along x at every "
                    "quadrature point (taus frozen), no matrix; spmv = block-CSR product with the "
                    "assembled values; assembly_ms = one steady-state vms_assemble"}


def newton_step(torch, vms, tree, surf, f, prec, rtol=1e-6):
    """Newton's linear step J dx = -R after one assembly: Dirichlet rows at the
    nodes of IN elements, then BiCGStab (the paper's method, its tolerance
    1e-6) and GMRES(50), block-Jacobi preconditioned; wall time of the solve."""
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
    asm.set_fields(f)
    asm.assemble()
    asm.apply_dirichlet()
    b = -asm.resid
    out = {}
    for name, method in (("bicgstab", vms.VMS_KSP_BCGS), ("gmres50", vms.VMS_KSP_GMRES)):
        asm.solve(b, method=method, restart=50, max_iter=3000, rtol=rtol)  # warm-up (workspace)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, it, rr = asm.solve(b, method=method, restart=50, max_iter=3000, rtol=rtol)
        ms = 1e3 * (time.perf_counter() - t0)
        chk = (torch.linalg.vector_norm(b - asm.spmv(x)) / torch.linalg.vector_norm(b)).item()
        out[name] = {"steps": it, "ms": ms, "ms_per_step": ms / max(it, 1), "rel_residual": rr,
                     "rel_residual_by_spmv": chk}
    out["dirichlet_nodes"] = int(vms.vms_dirichlet_nodes(asm.ctx).size)
    out["note"] = ("rtol 1e-6 on the true residual; a BiCGStab step has two products with the "
                   "matrix, a GMRES step one; preconditioner: inverted 4x4 diagonal node blocks")
    asm.close()
    return out


def weak_bc_cost(torch, vms, tree, surf, f, prec, reps=20):
    """Cost of the weak (Nitsche) boundary terms of eq. (weakbc): steady-state
    assembly with and without them (HIP events on the context stream)."""
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
    asm.set_fields(f)
    vms.vms_set_timing(asm.ctx, True)
    vms.vms_set_overlap(asm.ctx, False)   # isolated stage times

    def timed():
        for _ in range(3):
            asm.assemble()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st = np.zeros(5)
        a.record(asm.stream)
        for _ in range(reps):
            asm.assemble()
        b.record(asm.stream)
        b.synchronize()
        for _ in range(reps):
            asm.assemble()
            st += np.array(vms.vms_last_timing(asm.ctx))
        return a.elapsed_time(b) / reps, st / reps

    t0, s0 = timed()
    asm.set_weak_bc(True, 4.0, (0.0, 0.0, 0.0))
    n_s = vms.vms_stats(asm.ctx)["n_surfgp"]
    t1, s1 = timed()
    asm.close()
    return {"surface_points": int(n_s), "assembly_ms_without": t0, "assembly_ms_with": t1,
            "surface_kernel_ms": float(s1[3] - s0[3]), "stage_ms_without": s0.tolist(),
            "stage_ms_with": s1.tolist(),
            "note": "steady-state vms_assemble (no relabel, in-order schedule); the surface kernel runs after the "
                    "INTERCEPTED items, its time is the difference of that stage; c_b = 4, g = 0"}


def cost_model(torch, vms, st, wb, workload_name):
    """eq. (Wpart) measured on this GPU: T_v (per volume quadrature point, both
    assembly kernels) and T_s (per surface point of the weak boundary terms)
    from the calibration workload, then the assembly-kernel time of another
    workload predicted from its element weights, 8 T_v sum_e W(e), and
    measured."""
    from paper_2009_00706_amd import inputs as I
    s0, s1 = np.array(wb["stage_ms_without"]), np.array(wb["stage_ms_with"])
    n_v = 8 * st["n_out"] + st["n_subgp"]
    t_v = (s0[2] + s0[3]) * 1e-3 / n_v
    t_s = (s1[3] - s0[3]) * 1e-3 / max(wb["surface_points"], 1)
    r = t_s / t_v
    tree, surf = I.sphere_workload(lmin=6, lmax=10, beta=3.0) if workload_name == "precision" \
        else I.sphere_workload(lmin=4, lmax=7, beta=4.0)
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3))
    mh_xyz = asm.export(vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64) / float(1 << tree.max_level)
    asm.set_fields(I.make_fields(mh_xyz * tree.root_len + np.asarray(tree.origin), 1001))
    asm.set_weak_bc(True, 4.0, (0.0, 0.0, 0.0))
    vms.vms_set_timing(asm.ctx, True)
    vms.vms_set_overlap(asm.ctx, False)   # isolated kernel times
    for _ in range(3):
        asm.assemble()
    stg = np.zeros(5)
    for _ in range(10):
        asm.assemble()
        stg += np.array(vms.vms_last_timing(asm.ctx))
    stg /= 10
    w = vms.vms_element_weights(asm.ctx, tree.n, r)
    asm.close()
    pred = 8.0 * t_v * w.sum() * 1e3
    meas = stg[2] + stg[3]
    return {"T_v_ns": t_v * 1e9, "T_s_ns": t_s * 1e9, "ts_over_tv": r,
            "calibration": "this workload, FP64: both assembly kernels without, and the surface "
                           "kernel with, the weak boundary terms",
            "prediction": {"workload": ("sphere r=0.1, levels 6-10 (" if workload_name == "precision"
                                        else "sphere r=0.1, levels 4-7 (") + f"{tree.n} octants), "
                                        "FP64, weak boundary terms on",
                           "sum_weights": float(w.sum()), "predicted_ms": pred, "measured_ms": meas,
                           "rel_error": (pred - meas) / meas}}


PEAK_MFMA_16_TFLOPS = 2500.0  # dense BF16 / FP16 matrix cores


def roofline_of(m, prec, vms, traffic):
    """Roofline of the dominant assembly kernel (the one with the larger
    isolated time): FP64 against the FP64 peak; the mixed forms against the
    dense BF16/FP16 matrix-core peak of their contraction, with the FP32 vector
    figure beside it (their per-point work and operand splits run on the FP32
    VALU). The OUT kernel runs alone on the context stream in either schedule:
    its time is that of the timed steps. The INTERCEPTED kernel of an
    overlapped step shares the GPU with the gather: its time is that of the
    in-order steps."""
    avg, io, st = m["stage"], m["stage_in_order"], m["stats"]
    if io[3] > io[2]:
        k_ms, n_pts, kname = io[3], st["n_subgp"], "k_asm2 (INTERCEPTED elements, sub-cell points)"
        sched = "in-order steps"
    else:
        k_ms, n_pts, kname = avg[2], 8 * st["n_out"], "k_asm2 (OUT elements)"
        sched = "timed steps"
    if prec == vms.VMS_FP64:
        rf = roofline(k_ms, n_pts, PEAK_FP64_TFLOPS, traffic, kname)
    else:
        rf = roofline(k_ms, n_pts, PEAK_MFMA_16_TFLOPS, traffic, kname)
        rf["frac_of_fp32_vector_peak"] = rf["achieved"] / PEAK_FP32_TFLOPS
    rf["kernel_ms_from"] = sched
    return rf


def roofline(k_ms, n_pts, peak, traffic, kname):
    achieved = FLOP_PER_POINT * n_pts / (k_ms * 1e-3) / 1e12
    return {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": traffic, "kernel": kname, "kernel_ms": k_ms,
            "points_per_launch": int(n_pts), "flop_per_point": FLOP_PER_POINT}


def main_single(args):
    from paper_2009_00706_amd import inputs as I
    tree, surf, cfg = workload(args.workload)
    log(f"workload {args.workload}: {tree.n} octants")
    # the CPU baseline forks worker processes: it runs before the GPU is touched
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(tree, surf, args.cpu_sample, cfg.get("shortest_side", 1.0), args.cpu_workers)
        log(f"cpu baseline: {cpu['value']:.1f} elements/s on {cpu['cores']} cores "
            f"({cpu['single_core_value']:.1f} on one)")

    import torch
    from paper_2009_00706_amd import vms
    pname = args.precision or "fp64"
    prec = {"fp64": vms.VMS_FP64, "bf16": vms.VMS_MIXED_BF16, "fp16": vms.VMS_MIXED_FP16}[pname]
    mh = vms.vms_mesh_create(tree)
    xyz = vms.vms_mesh_export(mh, vms.VMS_EXPORT_NODE_XYZ).T.astype(np.float64)
    vms.vms_mesh_destroy(mh)
    f = I.make_fields(xyz / float(1 << tree.max_level) * tree.root_len + np.asarray(tree.origin),
                      1001, cfg.get("shortest_side", 1.0))
    del xyz
    flags = vms.VMS_RELABEL if surf is not None else 0
    log("fields ready; timing the headline form")
    r = run_single(torch, vms, tree, surf, f, prec, args.steps, args.warmup, flags)
    st, avg = r["stats"], r["stage"]
    log(f"{pname}: {r['ms_step']:.2f} ms per step")
    out = {
        "metric": "VMS elements assembled/s + in-out tests/s; learned+mixed vs FP64 at err<=1e-5",
        "value": r["value"],
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == vms.VMS_FP64 else ("f32+bf16" if prec == 1 else "f32+f16"),
        "data": "synthetic",
        "config": dict(cfg, n_nodes=r["sizes"]["n_nodes"], nnz=r["sizes"]["nnz"],
                       n_out=st["n_out"], n_intercepted=st["n_intercepted"],
                       n_subgp=st["n_subgp"], precision=pname),
        "inout_tests_per_s": (st["n_labelled"] / (r["stage_in_order"][0] * 1e-3))
                             if r["stage_in_order"][0] > 0 else None,
        "steady_state_elements_per_s": r["steady"],
        "step_device_ms": r["step_device_ms"],
        "stage_ms": stage_dict(avg, r["overlapped"]),
        **schedule_info(r),
        "setup_s": r["setup_s"],
        "roofline": roofline_of(r, prec, vms, traffic_for(args.traffic, args.workload, pname)),
    }
    if prec == vms.VMS_FP64 and not args.no_forms:
        forms, keep = {}, {}
        for name, p in (("bf16", vms.VMS_MIXED_BF16), ("fp16", vms.VMS_MIXED_FP16)):
            m = run_single(torch, vms, tree, surf, f, p, args.steps, args.warmup, flags)
            log(f"{name}: {m['ms_step']:.2f} ms per step")
            # matrix error over the rows of active nodes: the identity rows of
            # inactive nodes are exact in every form and would dominate the norm
            forms[name] = dict({"value": m["value"], "ms_per_step": m["ms_step"],
                                "speedup_vs_fp64": m["value"] / r["value"]},
                               **form_errors(torch, m, r))
            forms[name]["stage_ms"] = stage_dict(m["stage"], m["overlapped"])
            forms[name].update(schedule_info(m))
            forms[name]["roofline"] = roofline_of(m, p, vms, traffic_for(args.traffic, args.workload, name))
            keep[name] = (m["vals"], m["resid"], p)
            del m
        out["forms"] = forms
        out["forms_note"] = ("mixed forms on the same inputs and step; errors are normwise against "
                             "this FP64 GPU result (itself within 1e-12 of the CPU reference)")
        best = max(forms, key=lambda k: forms[k]["value"])
        for k in list(keep):
            if k != best:
                del keep[k]
        if surf is not None and not args.no_learned:
            log(f"learned + {best}: training the filter")
            out["learned_mixed"] = learned_mixed(torch, vms, tree, surf, f, cfg, args, flags, r,
                                                 best, keep[best])
        keep.clear()
        torch.cuda.empty_cache()
    if not args.no_scatter and prec == vms.VMS_FP64:
        out["atomic_scatter"] = atomic_scatter(torch, vms, tree, surf, f, args, flags, r,
                                               out.get("forms", {}))
    del r["vals"]
    torch.cuda.empty_cache()
    if not args.no_jv:
        log("Jacobian products")
        out["jacobian_action"] = jacobian_products(torch, vms, tree, surf, f, prec)
        log("Newton step")
        out["newton_step"] = newton_step(torch, vms, tree, surf, f, prec)
    if surf is not None and not args.no_jv:
        log("weak boundary terms")
        out["weak_bc"] = weak_bc_cost(torch, vms, tree, surf, f, prec)
        if prec == vms.VMS_FP64 and args.cost_model != "none":
            out["cost_model"] = cost_model(torch, vms, st, out["weak_bc"], args.cost_model)
    if surf is not None and not args.no_normal:
        log("normal-based filter")
        out["normal_filter"] = normal_filter(torch, vms, tree, surf, f)
    if surf is not None and not args.no_classify:
        log("standalone in-out classification")
        out["inout_classify"] = classify_rate(torch, vms, tree, surf)
    if surf is not None and args.learned_standalone:
        out["learned_inout"] = learned_inout(torch, vms, tree, surf,
                                             cfg.get("learned_train_samples", 1_000_000))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


def atomic_scatter(torch, vms, tree, surf, f, args, flags, r, forms):
    """The atomic scatter (vms_set_scatter), timed like the headline step in
    FP64 and in the faster mixed form, with its errors against the FP64 record
    scatter (in FP64 only the order of the additions differs)."""
    names = {"fp64": vms.VMS_FP64, "bf16": vms.VMS_MIXED_BF16, "fp16": vms.VMS_MIXED_FP16}
    cand = ["fp64"] + ([max(forms, key=lambda k: forms[k]["value"])] if forms else [])
    out = {}
    for name in cand:
        m = run_single(torch, vms, tree, surf, f, names[name], args.steps, args.warmup, flags,
                       prepare=lambda asm: vms.vms_set_scatter(asm.ctx, vms.VMS_SCATTER_ATOMIC), atomic=True)
        rec_ms = r["ms_step"] if name == "fp64" else forms[name]["ms_per_step"]
        st = m["stage"]
        out[name] = dict({"value": m["value"], "ms_per_step": m["ms_step"],
                          "speedup_vs_record_scatter": rec_ms / m["ms_step"],
                          "stage_ms": {"relabel": float(st[0]), "zero_fill": float(st[1]),
                                       "out_elements_with_atomics": float(st[2]),
                                       "intercepted_elements_with_atomics": float(st[3]),
                                       "identity_rows_and_residual": float(st[4])}},
                         **form_errors(torch, m, r))
        log(f"atomic scatter {name}: {m['ms_step']:.2f} ms per step")
        del m
        torch.cuda.empty_cache()
    out["note"] = ("values zeroed, then hardware atomic adds from the element kernels (no records, no "
                   "gather); summation order not fixed; errors against the FP64 record scatter")
    return out


def learned_mixed(torch, vms, tree, surf, f, cfg, args, flags, r, best, ref):
    """The learned + mixed step: the faster mixed form with the learned in-out
    filter in the relabel (threshold on the background-triangle count chosen by
    measurement). Its labels must be the exact ones: the CSR values and the
    residual equal the plain mixed form's bit for bit."""
    lf, info = train_filter(torch, surf, cfg.get("learned_train_samples", 1_000_000))
    p = ref[2]
    chosen = {}

    def prep(asm):
        chosen.update(learned_threshold(torch, vms, asm, lf))

    params = vms.make_params(quad_depth=3, precision=p, inout_mode=vms.VMS_INOUT_LEARNED)
    m = run_single(torch, vms, tree, surf, f, p, args.steps, args.warmup, flags, params=params,
                   prepare=prep)
    same = bool(torch.equal(m["vals"], ref[0]) and torch.equal(m["resid"], ref[1]))
    err = form_errors(torch, m, r)
    lf.close()
    rs = m["relabel"]
    return dict({"form": best, "value": m["value"], "ms_per_step": m["ms_step"],
                 "speedup_vs_fp64": m["value"] / r["value"],
                 "outputs_equal_to_the_exact_labels_form": same,
                 "decided_by_network": 1.0 - rs["exact_in_last_relabel"] / max(rs["candidates"], 1),
                 "stage_ms": stage_dict(m["stage"], m["overlapped"]), **schedule_info(m),
                 "threshold": chosen, "filter": info}, **err)


def main_batch(args):
    from paper_2009_00706_amd import inputs as I
    pname = args.precision or "bf16"
    t0 = time.perf_counter()
    work = I.batch_workload(args.n_trees, BATCH_SEED, workers=min(16, os.cpu_count() or 1))
    gen_s = time.perf_counter() - t0
    log(f"{len(work)} trees generated")
    cpu = None
    if not args.no_cpu_baseline:   # forks: before the GPU is touched
        big = max(range(len(work)), key=lambda k: work[k][0].n)
        cpu = cpu_baseline(work[big][0], work[big][1], args.cpu_sample, 1.0, args.cpu_workers)
        cpu["sample"] += f" (the largest tree of the batch, {work[big][0].n} octants)"
    import torch
    from paper_2009_00706_amd import vms
    prec = {"fp64": vms.VMS_FP64, "bf16": vms.VMS_MIXED_BF16, "fp16": vms.VMS_MIXED_FP16}[pname]
    stream = torch.cuda.Stream()
    ctxs, fields, vals, resid = [], [], [], []
    n_active = n_pts = n_oct = n_sub = 0
    t1 = time.perf_counter()
    with torch.cuda.stream(stream):
        for k, (tree, surf) in enumerate(work):
            ctx = vms.vms_create(tree, surf, vms.make_params(quad_depth=3, precision=prec),
                                 stream.cuda_stream)
            sz = vms.vms_sizes(ctx)
            st = vms.vms_stats(ctx)
            f = I.make_fields(node_xyz(vms, ctx, tree), 3000 + k)
            fields.append({n: torch.as_tensor(f[n], device="cuda") for n in f})
            dt = torch.float64 if prec == vms.VMS_FP64 else torch.float32
            vals.append(torch.zeros(sz["nnz"], dtype=dt, device="cuda"))
            resid.append(torch.zeros(sz["n_rows"], dtype=torch.float64, device="cuda"))
            ctxs.append(ctx)
            n_active += st["n_out"] + st["n_intercepted"]
            n_pts += 8 * st["n_out"] + st["n_subgp"]
            n_sub += st["n_subgp"]
            n_oct += tree.n
        setup_s = time.perf_counter() - t1
        log("contexts ready; autotuning")
        b = vms.vms_batch_create(ctxs, stream.cuda_stream)
        tune_ms = vms.vms_batch_autotune(b, fields, vals, resid)
        cfgb = vms.vms_batch_get_config(b)
        # kernel time of the persistent launch (eager), for the roofline; the
        # same with the fixed queue order (sub-cell items first, one each)
        order_ms = {}
        for by_w in (False, True):
            vms.vms_batch_set_order(b, by_w)
            kms = []
            for _ in range(4):
                vms.vms_batch_assemble(b, fields, vals, resid)
                kms.append(vms.vms_batch_last_timing(b))
            kms = np.array(kms[1:]).mean(0)
            order_ms["wpart_weighted" if by_w else "fixed"] = float(kms[1])
        vms.vms_batch_use_graph(b, True)
        for _ in range(args.warmup):
            vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        ts = time.perf_counter()
        for _ in range(args.steps):
            vms.vms_batch_assemble(b, fields, vals, resid)
        stream.synchronize()
        elapsed = time.perf_counter() - ts
        vms.vms_batch_destroy(b)
    sizes = sorted(t.n for t, _ in work)
    out = {
        "metric": "VMS elements assembled/s + in-out tests/s; learned+mixed vs FP64 at err<=1e-5",
        "value": n_active * args.steps / elapsed,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == vms.VMS_FP64 else ("f32+bf16" if prec == 1 else "f32+f16"),
        "data": "synthetic",
        "config": {"workload": f"{args.n_trees} independent octrees, log-uniform 1e4..5e5 octants "
                               f"(seed {BATCH_SEED}), one ellipsoid body each (2k-20k triangles), one persistent "
                               "launch replayed as a graph, sub-cell quadrature depth 3",
                   "octants": n_oct, "active_elements": n_active, "quadrature_points": n_pts,
                   "n_subgp": n_sub, "tree_sizes_min_median_max": [sizes[0], sizes[len(sizes) // 2],
                                                                   sizes[-1]],
                   "precision": pname, "autotuned": cfgb, "autotune_best_ms": tune_ms},
        "stage_ms": {"args": float(kms[0]), "persistent_assembly": float(kms[1]),
                     "csr_gather": float(kms[2])},
        "queue_order_persistent_ms": order_ms,
        "queue_note": ("units of about `tile` eq. (Wpart) element weights, heaviest first, against the "
                       "fixed order (every sub-cell item a unit of its own, all first, then runs of "
                       "`tile` OUT elements); same tile and workgroups per CU"),
        "setup_s": {"generate": gen_s, "contexts": setup_s},
        "roofline": roofline(float(kms[1]), n_pts,
                             PEAK_FP64_TFLOPS if prec == vms.VMS_FP64 else PEAK_MFMA_16_TFLOPS,
                             traffic_for(args.traffic, "batch64", pname),
                             "k_asm_batch (persistent, all trees)"),
    }
    if cpu is not None:
        out["cpu_baseline"] = cpu
    for c in ctxs:
        vms.vms_destroy(c)
    print(json.dumps(out))


# algorithmic work per Q2 quadrature point: the dense contraction with B 4 x 27
# and D 16 x 16: (16 x 4 x 27 x 4 + 16 x 27 x 27 x 4) multiply-adds x 2
FLOP_PER_POINT_Q2 = 2 * (16 * 4 * 27 * 4 + 16 * 27 * 27 * 4)


def main_q2(args):
    """Triquadratic elements on the uniform 16^3 cube (the paper's quadratic
    row of its matrix-assembly table): 27 Gauss points per element."""
    from oracle import core as O
    from oracle import q2 as Q
    from paper_2009_00706_amd import inputs as I
    tree = I.uniform_octree(4)
    m = Q.derive_q2_mesh(tree)
    f = I.make_fields(Q.node_xyz(tree, m), 1000)
    cpu = None
    if not args.no_cpu_baseline:
        import ctypes as C
        n = min(tree.n, 1500 if args.cpu_sample >= 1500 else args.cpu_sample)
        V = np.zeros(m.nnz)
        R = np.zeros(4 * m.n_nodes)
        xi, w = Q.points()
        c = O._c
        el = c(m.el_node[:n], np.int32)
        h = np.full(n, m.h)
        fl = {k: c(f[k], np.float64) for k in f}
        prm = O.params()
        t0 = time.perf_counter()
        Q._lib().or_q2_assemble(C.byref(prm), n, O._p(el), O._p(h), 27, O._p(c(xi, np.float64)),
                                O._p(c(w, np.float64)), *(O._p(fl[k]) for k in
                                                          ("ux", "uy", "uz", "p", "ux0", "uy0", "uz0")),
                                O._p(m.row_ptr), O._p(m.col_idx), O._p(V), O._p(R))
        dt = time.perf_counter() - t0
        cpu = {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
               "sample": f"the first {n} of the {tree.n} elements, residual and complex-step Jacobian, "
                         f"{dt:.1f} s in one process"}
        log(f"cpu baseline {n / dt:.1f} elements/s")
    import torch
    from paper_2009_00706_amd import vms
    q = vms.vms_q2_create(tree)
    sz = vms.vms_q2_sizes(q)
    fd = {k: torch.as_tensor(f[k], device="cuda") for k in f}
    vals = torch.zeros(sz["nnz"], dtype=torch.float64, device="cuda")
    res = torch.zeros(sz["n_rows"], dtype=torch.float64, device="cuda")
    for _ in range(args.warmup):
        vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        vms.vms_q2_assemble(q, fd, vals, res)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    kt = np.array([(vms.vms_q2_assemble(q, fd, vals, res), vms.vms_q2_last_timing(q))[1]
                   for _ in range(5)]).mean(0)
    vms.vms_q2_destroy(q)
    ms = 1e3 * el / args.steps
    out = {"metric": "VMS elements assembled/s + in-out tests/s; learned+mixed vs FP64 at err<=1e-5",
           "value": tree.n * args.steps / el, "unit": "elements/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "triquadratic (27-node) elements on the uniform 16^3 unit cube, 27 Gauss "
                                  "points per element, no body", "octants": tree.n,
                      "n_nodes": sz["n_nodes"], "nnz": sz["nnz"]},
           "stage_ms": {"element_kernel": float(kt[0]), "gathers": float(kt[1])},
           "roofline": {"bound": "alu", "achieved": FLOP_PER_POINT_Q2 * 27 * tree.n / (kt[0] * 1e-3) / 1e12,
                        "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                        "frac": FLOP_PER_POINT_Q2 * 27 * tree.n / (kt[0] * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                        "traffic": None, "kernel": "k_q2", "kernel_ms": float(kt[0]),
                        "points_per_launch": 27 * tree.n, "flop_per_point": FLOP_PER_POINT_Q2}}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    if args.workload == "batch64":
        main_batch(args)
    elif args.workload == "q2uniform16":
        main_q2(args)
    else:
        main_single(args)


if __name__ == "__main__":
    main()
