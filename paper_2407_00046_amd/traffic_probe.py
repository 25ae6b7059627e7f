"""HBM traffic probe for the PCG block SpMV (run under rocprofv3 --pmc).

Launches, on one GPU:
  1. a plain device-to-device copy of a known size (torch.Tensor.copy_),
     whose FETCH_SIZE / WRITE_SIZE calibrate the counters;
  2. one time step of the stacked-boxes workload (the benchmark's), then a
     linearization at the resulting state (contact blocks included) and a
     64-iteration PCG solve through bal_solve, so the k_cg_spmv dispatches
     run on a matrix of the benchmark's shape.

With --workload grid, step 2 is replaced by block SpMVs on the 128^3-cell
grid (2,146,689 nodes) in FP32 and FP64 storage.

Usage (one counter group per run):
  rocprofv3 --pmc FETCH_SIZE -d OUT -o run -- python3 paper_2407_00046_amd/traffic_probe.py [--workload grid]
  rocprofv3 --pmc WRITE_SIZE -d OUT -o run -- python3 paper_2407_00046_amd/traffic_probe.py [--workload grid]
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--copy-mib", type=int, default=512)
    ap.add_argument("--cells", type=int, default=16)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--iters", type=int, default=64)
    ap.add_argument("--workload", default="boxes", choices=["boxes", "grid"],
                    help="boxes: one step of the stacked boxes then PCG; grid: products on the 128^3 grid")
    args = ap.parse_args()
    import torch
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import scenes
    from paper_2407_00046_amd import Scene
    n = args.copy_mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(f"[probe] copy of {args.copy_mib} MiB done", flush=True)
    if args.workload == "grid":
        sc = scenes.spmv_grid(128)
        for prec in ("mixed", "fp64"):
            g = Scene(sc, precision=prec, device=0)
            g.linearize(np.asarray(sc["x0"]), sigma=0.0)
            ms, by = g.spmv_benchmark(reps=5)
            g.close()
            print(f"[probe] grid {prec}: k_spmv {ms * 1e3:.1f} us/launch, {by:.0f} B algorithmic per SpMV", flush=True)
        return
    sc = scenes.stacked_boxes(n_cubes=8, cells=args.cells, seed=0)
    g = Scene(sc, precision=args.precision, newton_rtol=1e-4, pcg_rtol=1e-4, device=0)
    st = g.step(allow=(0, -7))  # one step of the workload: the matrix below carries its contact blocks
    xb, _ = g.get_state()
    x = np.concatenate([xb, sc["obs_pos"]])
    _, _, n_active = g.linearize(x, sigma=st["sigma"])
    rng = np.random.default_rng(0)
    rhs = rng.normal(size=(g.n_all, 3))
    z, it, rel = g.solve(rhs, mode=0, rtol=1e-30, max_iters=args.iters)
    ms, by = g.spmv_benchmark(reps=8)
    print(f"[probe] {n_active} active pairs; PCG {it} iterations; k_spmv {ms * 1e3:.2f} us/launch, "
          f"{by:.0f} B algorithmic per SpMV", flush=True)


if __name__ == "__main__":
    main()
