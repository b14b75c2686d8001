"""Benchmark of the VMS assembly + in-out hot path on one MI355X.

One step = vms_assemble with relabelling: adaptive sub-cell quadrature of every
INTERCEPTED element with an exact in-out test of each candidate point, then
the residual and Jacobian of every non-IN element scattered into the CSR
(zeroing and identity rows included). Inputs are resident in HBM before the
timed region. Prints one JSON line.

Workload (default): immersed sphere r = 0.1 (icosphere, 5120 triangles) at the
unit cube's centre, octree levels 5-8 refined at the surface (194,328 octants,
hanging nodes), sub-cell quadrature depth 3, FP64.
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

# algorithmic work per quadrature point: the dense B^T D B
# contraction, (16x4x32 + 32x4x32) multiply-adds x 2 = 12,288 flop; an OUT
# element has 8 points, an INTERCEPTED element its kept sub-cell points
FLOP_PER_POINT = 12288
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="sphere", choices=["sphere", "uniform16"])
    ap.add_argument("--precision", default="fp64", choices=["fp64", "bf16", "fp16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1500, help="elements in the oracle sample")
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
    tree, surf = I.sphere_workload()
    return tree, surf, {
        "workload": "immersed sphere r=0.1 (icosphere 4, 5120 triangles), octree levels 5-8 "
                    f"refined at the surface ({tree.n} octants), sub-cell quadrature depth 3",
        "octants": tree.n}


def cpu_baseline(tree, surf, fields, n_sample):
    """The CPU reference as it stands, single-threaded, on a bounded sample."""
    from oracle import core as O
    ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level)
    mk = np.zeros(tree.n, np.uint8)
    if surf is not None:
        mk, _, _ = O.markers(tree, ms, surf)
        ms = O.derive_mesh(tree.ax, tree.ay, tree.az, tree.level, tree.max_level, active=mk != O.IN)
    rng = np.random.default_rng(0)
    outs = np.nonzero(mk == O.OUT)[0]
    cut = np.nonzero(mk == O.INTERCEPTED)[0]
    n_cut = min(cut.size, max(1, n_sample * cut.size // max(1, outs.size + cut.size)))
    s_cut = np.sort(rng.choice(cut, n_cut, replace=False)) if cut.size else cut
    s_out = np.sort(rng.choice(outs, min(outs.size, n_sample - n_cut), replace=False))
    t0 = time.perf_counter()
    sub = O.subquad(tree, surf, s_cut, 3) if s_cut.size else None
    O.assemble(tree, ms, fields, mk=mk, sub=sub, depth=3, subset=np.concatenate([s_out, s_cut]))
    dt = time.perf_counter() - t0
    n = s_out.size + s_cut.size
    return {"value": n / dt, "unit": "elements/s", "cores": 1, "kind": "oracle",
            "sample": f"{s_out.size} OUT + {s_cut.size} INTERCEPTED elements drawn at random "
                      f"(seed 0) from the same workload, sub-cell quadrature and exact labels "
                      f"of the INTERCEPTED ones included, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    if args.copy_calib:
        copy_calibration(args.copy_calib)
        return
    import torch
    from paper_2009_00706_amd import inputs as I
    from paper_2009_00706_amd import vms

    prec = {"fp64": vms.VMS_FP64, "bf16": vms.VMS_MIXED_BF16, "fp16": vms.VMS_MIXED_FP16}[args.precision]
    tree, surf, cfg = workload(args.workload)
    t_setup = time.perf_counter()
    asm = vms.Assembler(tree, surf, vms.make_params(quad_depth=3, precision=prec))
    setup_s = time.perf_counter() - t_setup
    xyz = asm.export(vms.VMS_EXPORT_NODE_XYZ).T / float(1 << tree.max_level)
    f = I.make_fields(xyz, 1001)
    asm.set_fields(f)
    st = vms.vms_stats(asm.ctx)
    n_active = st["n_out"] + st["n_intercepted"]
    flags = vms.VMS_RELABEL if surf is not None else 0
    vms.vms_set_timing(asm.ctx, True)
    stream = asm.stream
    for _ in range(args.warmup):
        asm.assemble(flags=flags)
    torch.cuda.synchronize()
    # ---- timed region: K whole steps, per-stage HIP events on the context stream
    stage = np.zeros((args.steps, 4))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        asm.assemble(flags=flags)
        stage[k] = vms.vms_last_timing(asm.ctx)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    value = n_active * args.steps / elapsed
    # ---- steady state (labels cached), for context
    t1 = time.perf_counter()
    for _ in range(args.steps):
        asm.assemble(flags=0)
    torch.cuda.synchronize()
    steady = n_active * args.steps / (time.perf_counter() - t1)
    sizes = asm.sizes
    avg = stage.mean(0)
    # dominant kernel: the assembly kernel with the larger time
    if avg[3] > avg[2]:
        k_ms, n_pts, kname = avg[3], st["n_subgp"], "k_asm_f64 (INTERCEPTED elements, sub-cell points)"
    else:
        k_ms, n_pts, kname = avg[2], 8 * st["n_out"], "k_asm_f64 (OUT elements)"
    achieved = FLOP_PER_POINT * n_pts / (k_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(args.traffic):
        try:
            tr = json.load(open(args.traffic))
            if tr.get("workload") == args.workload and tr.get("precision") == args.precision:
                traffic = tr.get("bytes_per_launch")
        except Exception:
            traffic = None
    out = {
        "metric": "VMS elements assembled/s + in-out tests/s; learned+mixed vs FP64 at err<=1e-5",
        "value": value,
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == vms.VMS_FP64 else ("f32+bf16" if prec == 1 else "f32+f16"),
        "data": "synthetic",
        "config": dict(cfg, n_nodes=sizes["n_nodes"], nnz=sizes["nnz"], n_out=st["n_out"],
                       n_intercepted=st["n_intercepted"], n_subgp=st["n_subgp"],
                       precision=args.precision),
        "inout_tests_per_s": (st["n_labelled"] / (avg[0] * 1e-3)) if avg[0] > 0 else None,
        "steady_state_elements_per_s": steady,
        "stage_ms": {"relabel": avg[0], "zero": avg[1], "out_elements": avg[2],
                     "intercepted_elements": avg[3]},
        "setup_s": setup_s,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "kernel": kname, "kernel_ms": k_ms, "points_per_launch": n_pts,
                     "flop_per_point": FLOP_PER_POINT},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(tree, surf, f, args.cpu_sample)
    asm.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
