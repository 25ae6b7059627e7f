"""Benchmark: BAL time steps on the stacked-boxes workload (one MI355X).

One "step" is one bal_step: a whole backward-Euler time step through every
kernel of the path (candidates, distances, element and contact Hessians with
projection, assembly, warm start, PCG, CCD, line search, dual updates).

Workload: 8 randomly rotated cubes of 16^3 cells x 5 tets (163,840 tets,
39,304 vertices) stacked with 5 mm gaps above a ground plane, E = 1e6 Pa,
nu = 0.45, h = 1/30 s, dhat = 1e-3 m, Newton and PCG tolerances 1e-4, the
workload's 10 steps (the cubes fall, collide and stack: the early steps are
contact-light, the later ones carry thousands of active pairs and most of
the Newton and PCG iterations).  K timed steps walk those 10 steps in order
and start again from the initial state after the tenth.

The headline value is seconds per time step in FP64 (the paper's precision).
Mixed precision runs each of the same steps from the FP64 trajectory's state
at its start, so both precisions are timed on identical states, and the
one-step position error of mixed against FP64 is reported per step.  The
roofline object covers the dominant kernel (the FP64 PCG block SpMV), timed
with HIP events on the scene's stream over a replay of the timed steps.  The
CPU baseline times the FP64 oracle on one contact-heavy Newton iteration of
two of the cubes (face to face, 0.5 mm apart: inside dhat) and scales it by
4 and by the GPU's Newton iterations per step.

Other modes (one JSON line each):
  --large       one frame of the large chain net (1,762,560 tets) in FP64 and mixed
  --ablations   the stacked boxes with warm_start = 0 and with use_al = 0 (FP64)
  --ablations-net  the same ablations on the chain net (mixed, its first 2 steps)
  --friction CHI   the stacked boxes' FP64 steps with friction coefficient CHI
  --scale       one step of 60 tumbling blocks (8.9M tets), free and under an
                active-pair memory limit (the line search's halving, Sec. 5.2)
  --traffic boxes|grid
                the workload for PMC traffic counters (run under rocprofv3 --pmc):
                a 512 MiB streaming copy to calibrate the counters, then PCG
                products on the stacked boxes' matrix after one step (boxes) or
                block SpMVs on the 128^3-cell grid (grid)

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
METRIC = "s/timestep & PCG iters/s, mixed vs FP64 at 1e-4 tol; BSR SpMV HBM GB/s"
TOL = dict(newton_rtol=1e-4, pcg_rtol=1e-4)


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


def summarize(stats, wall):
    n = len(stats)
    pcg = sum(s["pcg_iters"] for s in stats)
    warm = sum(s["warm_iters"] for s in stats)
    sec_pcg = sum(s["sec_pcg"] for s in stats)
    return dict(
        s_per_step=wall / n,
        newton_iters_per_step=sum(s["newton_iters"] for s in stats) / n,
        pcg_iters_per_step=pcg / n,
        warm_iters_per_step=warm / n,
        pcg_iters_per_s=(pcg + warm) / sec_pcg if sec_pcg > 0 else None,
        sec_pcg_per_step=sec_pcg / n,
        sec_hessian_per_step=sum(s["sec_hessian"] for s in stats) / n,
        sec_ccd_per_step=sum(s["sec_ccd"] for s in stats) / n,
        sec_collision_per_step=sum(s["sec_collision"] for s in stats) / n,
        sec_linesearch_per_step=sum(s["sec_linesearch"] for s in stats) / n,
        n_active_max=max(s["n_active_max"] for s in stats),
        n_aug_max=max(s["n_aug_max"] for s in stats),
        converged_steps=sum(s["converged"] for s in stats),
        steps=n,
    )


def run_fp64(sc, steps, warmup, stream, **kw):
    """W untimed steps, then K timed steps walking the workload's steps from
    its initial state; then a replay of the workload's steps with kernel timing
    that also records the state at the start of each step (the replay takes
    bitwise the same steps: every reduction sums in a fixed order)."""
    import torch
    from paper_2407_00046_amd import Scene
    n_wl = int(sc["n_steps"])
    g = Scene(sc, precision="fp64", device=0, stream=stream, **TOL, **kw)
    x0, v0 = g.get_state()
    for k in range(warmup):
        if k and k % n_wl == 0:
            g.set_state(x0, v0)
        g.step(allow=(0, -7))
    g.set_state(x0, v0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        if k and k % n_wl == 0:
            g.set_state(x0, v0)
        stats.append(g.step(allow=(0, -7)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print(f"[bench] fp64: {steps} steps in {wall:.1f} s", flush=True)
    g.set_state(x0, v0)
    g.set_kernel_timing(True)
    states, timed = [(x0, v0)], []
    for k in range(min(steps, n_wl)):
        timed.append(g.step(allow=(0, -7)))
        states.append(g.get_state())
    g.set_kernel_timing(False)
    g.close()
    out = summarize(stats, wall)
    out["per_step"] = [dict(status=s["status"], newton=s["newton_iters"], pcg=s["pcg_iters"], warm=s["warm_iters"],
                            active=s["n_active_max"], sec=round(s["sec_total"], 4)) for s in stats[:n_wl]]
    spmv_ms = sum(s["spmv_ms"] for s in timed)
    spmv_n = sum(s["spmv_launches"] for s in timed)
    out["replay_same_iters"] = [s["pcg_iters"] for s in timed] == [s["pcg_iters"] for s in stats[:len(timed)]]
    out["spmv_launches"] = spmv_n
    out["spmv_ms_avg"] = spmv_ms / spmv_n if spmv_n else None
    # algorithmic bytes of each step's product launches, weighted by their launch counts
    w_bytes = sum(s["spmv_bytes"] * s["spmv_launches"] for s in timed)
    out["spmv_bytes_avg"] = w_bytes / spmv_n if spmv_n else None
    if spmv_n and spmv_ms > 0:
        out["spmv_gbs"] = w_bytes / (spmv_ms * 1e-3) / 1e9
    return out, states


def run_mixed_from(sc, states, steps, stream, **kw):
    """Mixed-precision steps, each started from the FP64 trajectory's state at
    the start of that step: the same K steps as the FP64 run, on identical
    states; eps_x[k] = max_v |x_mixed - x_fp64| / (scene diagonal) after step k."""
    import torch
    from paper_2407_00046_amd import Scene
    n_wl = len(states) - 1
    L = float(np.linalg.norm(sc["x0"].max(0) - sc["x0"].min(0)))
    g = Scene(sc, precision="mixed", device=0, stream=stream, **TOL, **kw)
    stats, eps, wall = [], [], 0.0
    for k in range(steps):
        x, v = states[k % n_wl]
        g.set_state(x, v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats.append(g.step(allow=(0, -7)))
        torch.cuda.synchronize()
        wall += time.perf_counter() - t0
        if k < n_wl:
            xm, _ = g.get_state()
            eps.append(float(np.linalg.norm(xm - states[k + 1][0], axis=1).max() / L))
    g.close()
    print(f"[bench] mixed: {steps} steps in {wall:.1f} s (each from the FP64 state)", flush=True)
    out = summarize(stats, wall)
    out["per_step"] = [dict(status=s["status"], newton=s["newton_iters"], pcg=s["pcg_iters"], warm=s["warm_iters"],
                            active=s["n_active_max"], sec=round(s["sec_total"], 4)) for s in stats[:n_wl]]
    out["eps_x_vs_fp64_per_step"] = eps
    out["eps_x_vs_fp64_max"] = max(eps) if eps else None
    return out


def stream_peak():
    from paper_2407_00046_amd import bal
    rd, cp = bal.stream_benchmark(0, 2 << 30, 20)
    return dict(read_gbs=rd, copy_gbs=cp, kernel="k_stream_read / k_stream_copy (2 GiB)")


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


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(gpu_newton_per_step, threads_one=True):
    """The FP64 oracle on one contact-heavy Newton iteration of a quarter of
    the workload: 2 of its 8 cubes, axis-aligned and face to face 0.5 mm apart
    above the ground (about 14,500 pairs inside dhat from the first iteration,
    as many as the workload's contact-heavy steps carry), timed with every host
    thread and with one; scaled by 4 for the workload's 8 cubes and by the
    GPU's Newton iterations per step."""
    import torch
    import scenes
    from oracle import OracleScene, Params
    sc = scenes.stacked_boxes(n_cubes=2, cells=16, seed=0, gap=5e-4, rotate=False)
    scale = 4.0

    def one_iteration():
        o = OracleScene(sc, Params(newton_rtol=1e-4, max_newton=1, pair_mode="kdtree", verbose=True))
        t0 = time.perf_counter()
        tr = []
        o.step(trace=tr)
        return time.perf_counter() - t0, tr[0]["n_active"]

    threads = torch.get_num_threads()
    sec, nact = one_iteration()
    sec1 = None
    if threads_one:
        torch.set_num_threads(1)
        try:
            sec1, _ = one_iteration()
        finally:
            torch.set_num_threads(threads)
    per_iter = scale * sec
    return dict(value=per_iter * gpu_newton_per_step, unit="s/step", cores=threads, kind="oracle",
                sample=(f"one Newton iteration of 2 of the 8 cubes face to face 0.5 mm apart ({nact} pairs inside "
                        f"dhat): {sec:.1f} s on {threads} threads, x4 for the 8 cubes, x the GPU's "
                        f"{gpu_newton_per_step:.1f} FP64 Newton iterations per step"),
                cpu_model=cpu_model(), sec_per_newton_iter=per_iter,
                sec_per_newton_iter_1thread=scale * sec1 if sec1 else None,
                value_1thread=scale * sec1 * gpu_newton_per_step if sec1 else None)


def roofline_of(run, kernel):
    ach = run.get("spmv_gbs")
    if not ach:
        return None
    rec = recorded_traffic(kernel)
    roof = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                traffic=rec["bytes_per_launch"] if rec else None, kernel=kernel,
                bytes_per_launch=run["spmv_bytes_avg"], avg_launch_ms=run["spmv_ms_avg"])
    if rec:
        roof["traffic_note"] = (f"PMC on the same kernel source: {rec['bytes_per_launch']} B per launch vs "
                                f"{rec['algorithmic_bytes_probe']} B algorithmic on the probe's matrix")
    return roof


def mode_traffic(which, stream):
    """Counter workload: a calibration copy of 512 MiB, then the products."""
    import scenes
    from paper_2407_00046_amd import Scene, bal
    bal.stream_benchmark(0, 512 << 20, 3)
    print("[traffic] calibration: 3 reads and 3 copies of 512 MiB (k_stream_read, k_stream_copy)", flush=True)
    if which == "grid":
        sc = scenes.spmv_grid(128)
        for prec in ("mixed", "fp64"):
            g = Scene(sc, precision=prec, device=0, stream=stream)
            g.linearize(np.asarray(sc["x0"]), sigma=0.0)
            ms, by = g.spmv_benchmark(reps=5)
            g.close()
            print(f"[traffic] grid {prec}: k_spmv {ms * 1e3:.1f} us/launch, {by:.0f} B algorithmic", flush=True)
        return
    sc = scenes.stacked_boxes(n_cubes=8, cells=16, seed=0)
    for prec in ("fp64", "mixed"):
        g = Scene(sc, precision=prec, device=0, stream=stream, **TOL)
        st = g.step(allow=(0, -7))  # one step: the matrix below carries its contact blocks
        xb, _ = g.get_state()
        x = np.concatenate([xb, sc["obs_pos"]])
        _, _, n_active = g.linearize(x, sigma=st["sigma"])
        rhs = np.random.default_rng(0).normal(size=(g.n_all, 3))
        _, it, _ = g.solve(rhs, mode=0, rtol=1e-30, max_iters=64)
        ms, by = g.spmv_benchmark(reps=8)
        g.close()
        print(f"[traffic] boxes {prec}: {n_active} active pairs; PCG {it} iterations; k_spmv {ms * 1e3:.2f} us, "
              f"{by:.0f} B algorithmic per SpMV", flush=True)


def mode_large(stream, ccd_rule):
    import scenes
    from paper_2407_00046_amd import Scene
    out = {}
    for E_net in (1e9, 1e8):
        sc = scenes.chain_net_large(E_net=E_net)
        print(f"[bench] {sc['name']} E_net {E_net:g}: {sc['tets'].shape[0]} tets, {sc['rest_pos'].shape[0]} vertices",
              flush=True)
        for prec in ("fp64", "mixed"):
            g = Scene(sc, precision=prec, device=0, stream=stream, ccd_rule=ccd_rule, **TOL)
            st = g.step(allow=(0, -7))
            g.close()
            rec = {k: st[k] for k in ("status", "converged", "newton_iters", "pcg_iters", "warm_iters", "n_active_max",
                                      "n_aug_max", "ls_retries", "sec_total", "sec_pcg", "min_dist")}
            out[f"E{E_net:g}_{prec}"] = rec
            print(f"[bench] large net E {E_net:g} {prec}: {rec}", flush=True)
    print(json.dumps(dict(metric=METRIC, workload="chain_net_large_1.76M_tets_1_frame", ccd_rule=ccd_rule,
                          results=out)), flush=True)


def mode_scale(stream, ccd_rule):
    """One step of the memory-limited scale-up workload (60 tumbling blocks,
    8.9M tets) in FP64, capped at 200 Newton iterations: device memory the
    scene holds, s/step, Newton and PCG iterations; then the same step with
    the active-pair memory limit set to a quarter of the pairs the free run
    activates, so the line search halves (Sec. 5.2)."""
    import torch
    import scenes
    from paper_2407_00046_amd import Scene
    sc = scenes.tumbling_blocks()
    print(f"[bench] {sc['name']}: {sc['tets'].shape[0]} tets, {sc['rest_pos'].shape[0]} vertices", flush=True)
    os.environ["BAL_VERBOSE"] = "1"  # the library prints a line per 25 Newton iterations of this long step
    out = {}
    limit = None
    for name in ("free", "limited"):
        # a bounded sample: the step is capped at 200 Newton iterations
        kw = dict(max_newton=200, **(dict(max_contacts=limit) if limit else {}))
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        g = Scene(sc, precision="fp64", device=0, stream=stream, ccd_rule=ccd_rule, **TOL, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = g.step(allow=(0, -6, -7))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        free1, _ = torch.cuda.mem_get_info()
        g.close()
        rec = {k: st[k] for k in ("status", "converged", "newton_iters", "pcg_iters", "warm_iters", "n_active_max",
                                  "ls_retries", "sec_pcg", "sec_hessian", "sec_ccd", "sec_collision")}
        rec.update(s_per_step=wall, device_gib=(free0 - free1) / 2 ** 30, max_contacts=limit)
        out[name] = rec
        print(f"[bench] scale {name}: {rec}", flush=True)
        limit = max(1, rec["n_active_max"] // 4)
    print(json.dumps(dict(metric=METRIC, workload=sc["name"], n_tets=int(sc["tets"].shape[0]), ccd_rule=ccd_rule,
                          results=out)), flush=True)


def mode_ablations(sc, steps, stream, ccd_rule):
    """The paper's two ablations (Sec. 6.3: plain barrier inexact Newton
    without A', and block-Jacobi PCG without the stiffness-grouped warm
    start) and the half-gap CCD margin (a departure) against the method as
    printed, FP64, the same timed steps."""
    out = {}
    for name, kw in (("bal", dict(ccd_rule=ccd_rule)), ("no_warm_start", dict(warm_start=0, ccd_rule=ccd_rule)),
                     ("no_al", dict(use_al=0, ccd_rule=ccd_rule)), ("ccd_half_gap", dict(ccd_rule="half_gap"))):
        r, _ = run_fp64(sc, steps, 0, stream, **kw)
        r.pop("per_step")
        out[name] = r
        print(f"[bench] ablation {name}: {r['s_per_step']:.3f} s/step, {r['newton_iters_per_step']:.1f} Newton, "
              f"{r['pcg_iters_per_step']:.0f} PCG + {r['warm_iters_per_step']:.0f} warm per step", flush=True)
    print(json.dumps(dict(metric=METRIC, workload=sc["name"], ablations=out)), flush=True)


def mode_friction(sc, chi, steps, stream, ccd_rule):
    """The stacked boxes' FP64 steps with fully-implicit friction (Sec. 4.1,
    coefficient chi, eps_v = dhat): the workload runs frictionless as
    configured; this measures what the friction terms cost."""
    r, _ = run_fp64(sc, steps, 0, stream, ccd_rule=ccd_rule, friction=chi)
    print(f"[bench] friction {chi}: {r['s_per_step']:.3f} s/step, {r['newton_iters_per_step']:.1f} Newton, "
          f"{r['pcg_iters_per_step']:.0f} PCG per step, {r['converged_steps']} of {r['steps']} steps converged",
          flush=True)
    print(json.dumps(dict(metric=METRIC, workload=sc["name"], friction=chi, fp64=r)), flush=True)


def mode_ablations_net(stream, ccd_rule, steps=2):
    """The two ablations on the chain net as its workload states it (mixed
    precision, tolerances 1e-4), a bounded sample of its first `steps` steps.
    Every configuration stops these steps at the 1000-iteration Newton cap,
    so the comparison is per Newton iteration: PCG and warm-start iterations
    and seconds per Newton iteration, and the steps' end states."""
    import scenes
    from paper_2407_00046_amd import Scene
    sc = scenes.chain_net()
    print(f"[bench] {sc['name']}: {sc['tets'].shape[0]} tets, {sc['rest_pos'].shape[0]} vertices", flush=True)
    out = {}
    for name, kw in (("bal", {}), ("no_warm_start", dict(warm_start=0)), ("no_al", dict(use_al=0))):
        g = Scene(sc, precision="mixed", device=0, stream=stream, ccd_rule=ccd_rule, **TOL, **kw)
        recs = []
        for _ in range(steps):
            st = g.step(allow=(0, -7))
            recs.append({k: st[k] for k in ("status", "newton_iters", "pcg_iters", "warm_iters", "n_active_max",
                                            "n_aug_max", "sec_total", "sec_pcg", "min_dist")})
        g.close()
        nn = sum(r["newton_iters"] for r in recs)
        out[name] = dict(steps=recs, newton=nn,
                         pcg_per_newton=sum(r["pcg_iters"] for r in recs) / nn,
                         warm_per_newton=sum(r["warm_iters"] for r in recs) / nn,
                         ms_per_newton=1e3 * sum(r["sec_total"] for r in recs) / nn)
        print(f"[bench] net ablation {name}: {nn} Newton, {out[name]['pcg_per_newton']:.1f} PCG + "
              f"{out[name]['warm_per_newton']:.1f} warm per Newton iteration, {out[name]['ms_per_newton']:.2f} ms "
              f"per Newton iteration", flush=True)
    print(json.dumps(dict(metric=METRIC, workload=sc["name"], precision="mixed", ccd_rule=ccd_rule,
                          sample=f"first {steps} of the workload's 5 steps", ablations=out)), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed steps (the workload has 10; more walk it again)")
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-r1", action="store_true", help="skip the 128^3-grid SpMV roofline")
    ap.add_argument("--ccd-rule", default="printed", choices=["printed", "half_gap", "literal"])
    ap.add_argument("--broad-phase", default="hash", choices=["hash", "lbvh"])
    ap.add_argument("--large", action="store_true")
    ap.add_argument("--ablations", action="store_true")
    ap.add_argument("--ablations-net", action="store_true")
    ap.add_argument("--friction", type=float, default=0.0,
                    help="run the stacked boxes' FP64 steps with this friction coefficient (a measurement mode)")
    ap.add_argument("--scale", action="store_true")
    ap.add_argument("--traffic", choices=["boxes", "grid"])
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
    if args.traffic:
        mode_traffic(args.traffic, stream)
        return
    if args.large:
        mode_large(stream, args.ccd_rule)
        return
    if args.scale:
        mode_scale(stream, args.ccd_rule)
        return
    if args.ablations_net:
        mode_ablations_net(stream, args.ccd_rule)
        return
    sc = scenes.stacked_boxes(n_cubes=8, cells=16, seed=0)
    print(f"[bench] workload {sc['name']}: {sc['tets'].shape[0]} tets, {sc['rest_pos'].shape[0]} vertices", flush=True)
    if args.ablations:
        mode_ablations(sc, args.steps, stream, args.ccd_rule)
        return
    if args.friction > 0.0:
        mode_friction(sc, args.friction, args.steps, stream, args.ccd_rule)
        return
    fp64, states = run_fp64(sc, args.steps, args.warmup, stream, ccd_rule=args.ccd_rule, broad_phase=args.broad_phase)
    print(f"[bench] fp64: {fp64['s_per_step']:.3f} s/step", flush=True)
    mixed = None
    if not args.no_mixed:
        mixed = run_mixed_from(sc, states, args.steps, stream, ccd_rule=args.ccd_rule, broad_phase=args.broad_phase)
        print(f"[bench] mixed: {mixed['s_per_step']:.3f} s/step, max one-step eps_x vs fp64 "
              f"{mixed['eps_x_vs_fp64_max']:.2e}", flush=True)
    r1 = None
    if not args.no_r1:
        r1 = spmv_r1(stream)
        r1["stream_peak"] = stream_peak()
        print(f"[bench] streaming read {r1['stream_peak']['read_gbs']:.0f} GB/s, copy "
              f"{r1['stream_peak']['copy_gbs']:.0f} GB/s", flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(fp64["newton_iters_per_step"])
        print(f"[bench] cpu oracle sample: {cpu['sample']}", flush=True)
    line = dict(
        metric=METRIC, value=fp64["s_per_step"], unit="s/step", n_gpus=1, steps=args.steps, warmup=args.warmup,
        ms_per_step=1e3 * fp64["s_per_step"], higher_is_better=False, scaling="weak", vs_baseline=None,
        dtype="f64", data="synthetic",
        config=dict(workload=sc["name"], n_tets=int(sc["tets"].shape[0]), n_verts=int(sc["rest_pos"].shape[0]),
                    workload_steps=int(sc["n_steps"]), precision="fp64", dt=sc["dt"], dhat=sc["dhat"],
                    ccd_rule=args.ccd_rule, broad_phase=args.broad_phase, **TOL),
        roofline=roofline_of(fp64, "k_cg_dir_spmv<double, double>"), cpu_baseline=cpu, spmv_hbm=r1, fp64=fp64,
        mixed=mixed,
        mixed_speedup=(fp64["s_per_step"] / mixed["s_per_step"]) if mixed else None,
    )
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
