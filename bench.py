"""Benchmark: BAL time steps on the stacked-boxes workload (one MI355X).

One "step" is one bal_step: a whole backward-Euler time step through every
kernel of the path (candidates, distances, element and contact Hessians with
projection, assembly, warm start, PCG, CCD, line search, dual updates).

Workload: 8 randomly rotated cubes of 16^3 cells x 5 tets (163,840 tets,
39,304 vertices) stacked with 5 mm gaps above a ground plane, E = 1e6 Pa,
nu = 0.45, h = 1/30 s, dhat = 1e-3 m, Newton and PCG tolerances 1e-4.
The headline value is seconds per time step in mixed precision over the
workload's 10 steps (the cubes fall, collide and stack: the early steps are
contact-light, the later ones carry thousands of active pairs and most of
the Newton and PCG iterations); the FP64 form runs the same steps for
comparison.  The roofline object covers the
dominant kernel (the PCG block SpMV), timed with HIP events on the scene's
stream inside the timed steps.  The CPU baseline times the FP64 oracle on a
bounded sample of the same workload (its first Newton iteration) and
scales it by the GPU's Newton iterations per step.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
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

HBM_PEAK_GBS = 8000.0


def recorded_traffic(kernel):
    """HBM-side bytes per launch of `kernel` from the PMC summary committed
    under profiles/ (FETCH_SIZE and WRITE_SIZE scaled by a copy of known
    size), or None when the kernel's source has changed since the counters
    were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            if not line.startswith("traffic-record: "):
                continue
            rec = json.loads(line[len("traffic-record: "):])
            if rec.get("kernel") != kernel:
                continue
            src = os.path.join(ROOT, rec["source"])
            if not os.path.exists(src):
                return None
            if hashlib.sha256(open(src, "rb").read()).hexdigest() != rec["source_sha256"]:
                return None
            return rec
    return None


def run_precision(sc, precision, steps, warmup, stream, replay=True):
    """Times `steps` steps after `warmup` steps (PCG replayed as HIP graphs),
    then, with `replay`, replays the same steps from the same state with
    kernel timing on (every PCG SpMV bracketed by HIP events on the scene's
    stream) for the SpMV roofline."""
    import torch
    from paper_2407_00046_amd import Scene
    g = Scene(sc, precision=precision, newton_rtol=1e-4, pcg_rtol=1e-4, device=0, stream=stream)
    for _ in range(warmup):
        g.step(allow=(0, -7))
    x_w, v_w = g.get_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for _ in range(steps):
        stats.append(g.step(allow=(0, -7)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    x_end, _ = g.get_state()
    print(f"[bench] {precision}: {steps} steps in {wall:.1f} s", flush=True)
    timed = []
    if replay:
        g.set_state(x_w, v_w)
        g.set_kernel_timing(True)
        timed = [g.step(allow=(0, -7)) for _ in range(steps)]
        g.set_kernel_timing(False)
    newton = sum(s["newton_iters"] for s in stats)
    pcg = sum(s["pcg_iters"] for s in stats)
    warm = sum(s["warm_iters"] for s in stats)
    sec_pcg = sum(s["sec_pcg"] for s in stats)
    spmv_ms = sum(s["spmv_ms"] for s in timed)
    spmv_n = sum(s["spmv_launches"] for s in timed)
    out = dict(
        s_per_step=wall / steps,
        newton_iters_per_step=newton / steps,
        pcg_iters_per_step=pcg / steps,
        warm_iters_per_step=warm / steps,
        pcg_iters_per_s=(pcg + warm) / sec_pcg if sec_pcg > 0 else None,
        sec_pcg_per_step=sec_pcg / steps,
        sec_hessian_per_step=sum(s["sec_hessian"] for s in stats) / steps,
        sec_ccd_per_step=sum(s["sec_ccd"] for s in stats) / steps,
        sec_collision_per_step=sum(s["sec_collision"] for s in stats) / steps,
        sec_linesearch_per_step=sum(s["sec_linesearch"] for s in stats) / steps,
        graph_launches_per_step=sum(s["graph_launches"] for s in stats) / steps,
        n_active_max=max(s["n_active_max"] for s in stats),
        converged_steps=sum(s["converged"] for s in stats),
        timed_replay_same_iters=([s["pcg_iters"] for s in timed] == [s["pcg_iters"] for s in stats]) if replay
        else None,
        spmv_launches=spmv_n,
        spmv_ms_avg=spmv_ms / spmv_n if spmv_n > 0 else None,
        spmv_bytes=(timed or stats)[-1]["spmv_bytes"],
    )
    if spmv_n > 0 and spmv_ms > 0:
        out["spmv_gbs"] = out["spmv_bytes"] / (out["spmv_ms_avg"] * 1e-3) / 1e9
    g.close()
    return out, x_end


def copy_peak_gbs(stream, mib=2048, reps=20):
    """Streaming-copy bandwidth (read + write bytes) of a device-to-device copy."""
    import torch
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def spmv_r1(stream, n=128, reps=50):
    """Block SpMV on the 128^3-cell grid (2.1M nodes, 12.7M off-diagonal block
    pairs): large enough that the matrix does not fit the on-chip caches, so
    the figure is an HBM figure.  Values are Neo-Hookean Hessians at a
    randomly perturbed state plus M/h^2."""
    import scenes
    from paper_2407_00046_amd import Scene
    sc = scenes.spmv_grid(n)
    x = np.asarray(sc["x0"])
    out = {"workload": sc["name"], "n_nodes": int(x.shape[0]), "n_tets": int(sc["tets"].shape[0])}
    for prec in ("mixed", "fp64"):
        g = Scene(sc, precision=prec, device=0, stream=stream)
        g.linearize(x, sigma=0.0)
        ms, by = g.spmv_benchmark(reps=reps)
        g.close()
        out[prec] = dict(ms_per_launch=ms, bytes_per_launch=by, gbs=by / (ms * 1e-3) / 1e9,
                         frac=by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS)
        print(f"[bench] spmv {sc['name']} {prec}: {ms * 1e3:.1f} us, {out[prec]['gbs']:.0f} GB/s", flush=True)
    return out


def cpu_baseline(sc, gpu_newton_per_step):
    import torch
    from oracle import OracleScene, Params
    o = OracleScene(sc, Params(newton_rtol=1e-4, max_newton=1, pair_mode="kdtree", verbose=True))
    t0 = time.perf_counter()
    o.step()
    sec = time.perf_counter() - t0
    return dict(value=sec * gpu_newton_per_step, unit="s/step", cores=torch.get_num_threads(), kind="oracle",
                sample=f"first Newton iteration of step 1 of the same workload ({sec:.1f} s), "
                       f"scaled by the GPU's {gpu_newton_per_step:.1f} Newton iterations per step")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (the workload has 10)")
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cells", type=int, default=16)
    ap.add_argument("--no-r1", action="store_true", help="skip the 128^3-grid SpMV roofline")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding of this path is a "
              "design note, not a build.", file=sys.stderr)
        sys.exit(2)
    import torch
    import scenes
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.init()
    stream = torch.cuda.current_stream().cuda_stream
    sc = scenes.stacked_boxes(n_cubes=8, cells=args.cells, seed=0)
    print(f"[bench] workload {sc['name']}: {sc['tets'].shape[0]} tets, {sc['rest_pos'].shape[0]} vertices", flush=True)
    mixed, xm = run_precision(sc, "mixed", args.steps, args.warmup, stream)
    print(f"[bench] mixed: {mixed['s_per_step']:.3f} s/step", flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64, xf = run_precision(sc, "fp64", args.steps, args.warmup, stream, replay=False)
        print(f"[bench] fp64: {fp64['s_per_step']:.3f} s/step", flush=True)
        L = np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0))
        mixed["eps_x_vs_fp64"] = float(np.linalg.norm(xm - xf, axis=1).max() / L)
    r1 = None
    if not args.no_r1:
        r1 = spmv_r1(stream)
        r1["copy_peak_gbs"] = copy_peak_gbs(stream)
        print(f"[bench] streaming copy: {r1['copy_peak_gbs']:.0f} GB/s", flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(sc, mixed["newton_iters_per_step"])
        print(f"[bench] cpu oracle sample: {cpu['sample']}", flush=True)
    ach = mixed.get("spmv_gbs")
    roof = None
    if ach:
        kern = "k_cg_dir_spmv<float,float>"
        rec = recorded_traffic(kern)
        roof = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                    traffic=rec["bytes_per_launch"] if rec else None, kernel=kern,
                    bytes_per_launch=mixed["spmv_bytes"], avg_launch_ms=mixed["spmv_ms_avg"])
        if rec:
            roof["traffic_note"] = (f"PMC on the same kernel source: {rec['bytes_per_launch']} B per launch vs "
                                    f"{rec['algorithmic_bytes_probe']} B algorithmic on the probe's matrix")
    line = dict(
        metric="s/timestep & PCG iters/s, mixed vs FP64 at 1e-4 tol; BSR SpMV HBM GB/s",
        value=mixed["s_per_step"], unit="s/step", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=1e3 * mixed["s_per_step"], higher_is_better=False, scaling="weak", vs_baseline=None,
        dtype="mixed f32/f64", data="synthetic",
        config=dict(workload=sc["name"], n_tets=int(sc["tets"].shape[0]), n_verts=int(sc["rest_pos"].shape[0]),
                    precision="mixed", dt=sc["dt"], dhat=sc["dhat"], newton_rtol=1e-4, pcg_rtol=1e-4),
        roofline=roof, cpu_baseline=cpu, spmv_hbm=r1, mixed=mixed, fp64=fp64,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
