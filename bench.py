#!/usr/bin/env python3
"""Benchmark: FitzHugh-Nagumo bidomain steps/s on a 256^3 grid with the KFBI diffusion solve.

Workload (synthetic, seeded): box [-1.2, 1.2]^3 with 256 cells per axis (255^3 unknowns per
component, coupled intra/extracellular pair); a closed thick shell (outer ellipsoid
0.9/0.7/0.6, inner wall 0.6 x ellipsoid with seeded smooth radial noise) carrying 40,960
interface nodes; sigma_i = 1, sigma_e = 2, Cm = beta = 1, dt = 0.01 (kappa = 200);
FHN theta = 0.13, H = 100, alpha = 0.25, zeta = 1; V = 1 in a ball of radius 0.25 at a
seeded mid-wall point; GMRES(50) relative tolerance 1e-8 on ||g'||.

A step is one whole Strang step (reaction, coupled KFBI Neumann solve, reaction) with all
inputs resident in HBM.  Every variant runs the same untimed steps first (default 40; the
learned variant records them and trains on them) and is then timed over the same window
(default steps 40-140).  The stimulus excites the whole shell by about step 60 and the
tissue is back at rest by about step 150, so this window holds the propagating wave; a
later window would time a resting tissue.  Variants: plain (FP64 throughout, GMRES from psi^{n-1}), mixed (FP32
matrix-vector products inside FP64 iterative refinement), learned (mixed + the learned warm
start), projected (mixed + the least-residual combination of the last 8 solutions as start).  Every solve ends at the same FP64 relative residual bound.

Prints one JSON line (see the "metric" key).  --batch and --copy-calibration run the
batched 2D workload and the counter calibration instead.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "bidomain steps/s at 256^3 (GMRES tol 1e-8), learned+mixed vs plain; HBM % peak"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--nodes", type=int, default=40960)
    ap.add_argument("--variants", default="plain,mixed,learned,projected,projected_mixed")
    ap.add_argument("--train-steps", type=int, default=40)
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--inner-tol", type=float, default=1e-4, help="mixed precision: relative tolerance of each FP32 inner solve")
    ap.add_argument("--kernel-steps", type=int, default=10, help="steps after the timed window timed per kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-run", action="store_true", help="short run for rocprofv3 (first listed variant only, no CPU baseline)")
    ap.add_argument("--batch", action="store_true",
                    help="only the batched 2D workload: 64 seeded Neumann problems of sizes 64..1024, "
                         "solved as one batch and one by one (problems/s)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time plain copies of one coupled FP64 field (the reference kernels for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def cpu_baseline(grid, co, box_solves_per_step):
    """Oracle (FP64 NumPy/SciPy, single-threaded FFT) on a bounded sample: one coupled box solve
    of the same 256^3 workload, scaled by the box solves per step of the GPU run."""
    import numpy as np

    from oracle import boxsolve
    f = np.random.default_rng(0).normal(size=(co.ncomp, grid.n ** grid.dim))
    t0 = time.perf_counter()
    boxsolve.box_solve(f, grid, co)
    dt_box = time.perf_counter() - t0
    s_per_step = dt_box * box_solves_per_step
    return {"value": 1.0 / s_per_step, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one coupled {grid.cells}^3 box solve by the oracle ({dt_box:.2f} s), scaled by "
                      f"{box_solves_per_step:.1f} box solves per step (matvecs + volume + final solve); "
                      f"interface work (<2% of a matvec) not included",
            "host_cpu": platform.processor() or platform.machine(),
            "host_cores_available": len(os.sched_getaffinity(0))}


def measured_traffic(kernel):
    """HBM bytes per launch of a dense DST pass from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size); None if the kernel
    source has changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "pmc_traffic_dst_fp64_shell256.txt")
    src = os.path.join(ROOT, "paper_2104_05024_amd", "csrc", "dst.hip")
    try:
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        for line in open(path):
            f = line.split()
            if len(f) == 5 and f[0] == "bench-traffic" and f[1] == kernel:
                if f[4] != sha:
                    return None, "counters predate the current kernel source"
                return float(f[2]), os.path.relpath(path, ROOT)
    except OSError:
        pass
    return None, "no counter summary"


def batch_bench(a, torch):
    """64 seeded 2D Neumann problems (manufactured u = e^x sin(pi y)), FP32 inner GMRES with
    FP64 refinement to 1e-10 per problem: one batch vs the problems one at a time."""
    import numpy as np

    from paper_2104_05024_amd import kfbi as K
    from paper_2104_05024_amd import workloads as W
    probs = W.batch_2d()
    t0 = time.perf_counter()
    b = K.Batch(probs)
    setup_s = time.perf_counter() - t0
    singles = [K.Problem(*p) for p in probs]
    dev = torch.device("cuda:0")
    fs, gs = [], []
    for (iface, grid, co), p in zip(probs, singles):
        pts = W.grid_points(grid)
        fs.append((np.pi ** 2 - 1 + co.kappa) * np.exp(pts[:, 0]) * np.sin(np.pi * pts[:, 1]))
        X, n = p.table("nodes_X").reshape(-1, 2), p.table("nodes_n").reshape(-1, 2)
        gs.append(n[:, 0] * np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1])
                  + n[:, 1] * np.pi * np.exp(X[:, 0]) * np.cos(np.pi * X[:, 1]))
    f = torch.tensor(np.concatenate(fs), device=dev)
    g = torch.tensor(np.concatenate(gs), device=dev)
    opts = dict(tol=1e-10, precision=1, inner_tol=1e-4)
    for _ in range(max(a.warmup, 1)):
        b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    reps = max(1, min(a.steps, 10))
    t0 = time.perf_counter()
    for _ in range(reps):
        u, psi, infos = b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    worst = max(i["rel_resid"] for i in infos)
    # the same problems one at a time through the single-problem entry point
    segs = [(f[b.goff[i]:b.goff[i] + b.N[i] ** 2].reshape(1, -1).contiguous(),
             g[b.ioff[i]:b.ioff[i] + b.M[i]].reshape(1, -1).contiguous()) for i in range(b.n)]
    for p, (fi, gi) in zip(singles, segs):
        p.solve_neumann(gi, fi, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for p, (fi, gi) in zip(singles, segs):
            p.solve_neumann(gi, fi, **opts)
    torch.cuda.synchronize()
    t_single = (time.perf_counter() - t0) / reps
    for p in singles:
        p.close()
    b.close()
    print(json.dumps({
        "metric": "batched 2D Neumann solves, problems/s (FP32 inner + FP64 refinement to 1e-10)",
        "value": round(b.n / t_batch, 2), "unit": "problems/s", "n_problems": b.n,
        "one_at_a_time_problems_per_s": round(b.n / t_single, 2), "speedup_vs_one_at_a_time": round(t_single / t_batch, 2),
        "ms_per_batch": round(1000 * t_batch, 2), "reps": reps, "max_final_rel_resid": worst,
        "mean_inner_iters": float(np.mean([i["iters"] for i in infos])),
        "setup_s": round(setup_s, 2), "data": "synthetic (seeded stars, manufactured solution)",
        "config": {"workload": "64 star-shaped 2D Neumann problems, cells in {64,...,1024}, 3-8 lobes, "
                               "amplitude 0.05-0.2, kappa 50-2000, M = 2 cells"}}))


def copy_calibration(a, torch):
    """Two plain copies of one coupled FP64 field (known bytes): the runtime's blit copy and a
    torch elementwise kernel (dst = src * 1)."""
    n = 2 * (a.cells - 1) ** 3
    src = torch.ones(n, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    out = {"bytes_read": n * 8, "bytes_written": n * 8}
    for name, fn in (("blit", lambda: dst.copy_(src)), ("elementwise", lambda: torch.mul(src, 1.0, out=dst))):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / reps
        out[name] = {"avg_s": el, "GB_per_s": 2 * n * 8 / el / 1e9}
    print(json.dumps(out))


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py runs the workload on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    if a.copy_calibration:
        copy_calibration(a, torch)
        return
    if a.batch:
        batch_bench(a, torch)
        return
    from paper_2104_05024_amd import kfbi as K
    from paper_2104_05024_amd import workloads as W

    dev = torch.device("cuda:0")
    dt = 0.01
    p = W.BidomainParams()
    iface = W.thick_shell(n_nodes=a.nodes)
    grid = W.box(3, a.cells)
    co = W.bidomain_coeffs(3, p, dt)
    t0 = time.perf_counter()
    prob = K.Problem(iface, grid, co)
    setup_s = time.perf_counter() - t0
    log(f"setup {setup_s:.1f} s: M={prob.M} crossings={prob.n_crossings} irregular={prob.n_irregular}")
    V0, q0 = W.ball_state(grid, W.stimulus_center(iface), radius=0.25)

    variants = [v for v in a.variants.split(",") if v]
    if a.profile_run:
        variants = variants[:1]
    results = {}
    kt = {}
    for name in variants:
        if name == "learned":
            try:
                bd = K.Bidomain(prob, p, tol=1e-8, precision=1, warm_start=1, inner_tol=a.inner_tol)
                bd.mlp_init(capacity=max(a.train_steps, 1), seed=3)
            except K.KfbiError as e:
                log(f"learned variant unavailable: {e}")
                continue
        elif name in ("projected", "projected_mixed"):
            bd = K.Bidomain(prob, p, tol=1e-8, precision=1 if name == "projected_mixed" else 0, warm_start=3,
                            inner_tol=a.inner_tol)
        else:
            bd = K.Bidomain(prob, p, tol=1e-8, precision=1 if name == "mixed" else 0, warm_start=0,
                            inner_tol=a.inner_tol)
        V = torch.tensor(V0, device=dev)
        q = torch.tensor(q0, device=dev)
        hist = torch.zeros(2, 2, prob.M, dtype=torch.float64, device=dev)
        # every variant times the same window of the simulation: steps n_warm .. n_warm + steps
        n_warm = max(a.warmup, a.train_steps) if "learned" in variants else a.warmup
        for i in range(n_warm):
            bd.step(V, q, hist, dt)
        if name == "learned":
            loss = bd.train(epochs=a.epochs, lr=1e-3)
            log(f"learned: trained on {a.train_steps} steps, loss {loss:.3e}")
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(a.steps):
            infos.append(bd.step(V, q, hist, dt))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        # per-kernel HIP-event timing over the next steps (event timing launches every kernel
        # directly, so it stays out of the timed window, where GMRES replays captured steps)
        prob.profile(True)
        for i in range(a.kernel_steps):
            bd.step(V, q, hist, dt)
        torch.cuda.synchronize()
        kt[name] = {k: prob.kernel_time(k) for k in ("dst_x", "dst_y", "dst_last", "dst_x_rows", "dst_y_sparse",
                                                     "dst_last_sparse", "dst_last_out", "dst_x_fhn",
                                                     "jumps", "correct", "gather")}
        prob.profile(False)
        worst = max(i["rel_resid"] for i in infos)
        results[name] = {
            "steps_per_s": a.steps / el, "ms_per_step": 1000 * el / a.steps,
            "mean_iters": float(np.mean([i["iters"] for i in infos])),
            "mean_matvecs_fp64": float(np.mean([i["matvecs_fp64"] for i in infos])),
            "mean_matvecs_fp32": float(np.mean([i["matvecs_fp32"] for i in infos])),
            "max_final_rel_resid": worst,
            "mean_start_resid": float(np.mean([i["start_resid"] for i in infos])),
            "warm_start_used": int(sum(i["warm_start_used"] for i in infos)),
            "V_max": float(V.max().item()),
        }
        log(f"{name}: {results[name]}")
        bd.close()

    head = "learned" if "learned" in results else ("mixed" if "mixed" in results else "plain")
    r = results[head]
    # roofline of the dominant FP64 pencil kernel (plain variant: every launch is FP64).  The
    # dense passes (dst_x, dst_y, dst_last) each read and write the whole coupled field.  The
    # z pass of the matrix-vector product (dst_last_sparse) reads only the z planes that hold
    # irregular nodes (the others are zero) and writes only those that hold extrapolation
    # stencil nodes; the z pass of the BIE right-hand side's volume solve (dst_last_out) reads
    # every plane and writes only the stencil planes.  The row-masked x and y passes
    # (dst_x_rows, dst_y_sparse) are not priced.  The three x passes of a step that carry the
    # reaction (dst_x_fhn) are priced per launch as the mean of: forward Euler + source (V, q
    # read, the transformed pair written), source + correction (V, q and the correction rows
    # read, the pair written) and inverse + backward Euler (the pair, V and q read, V, q written).
    ref = "plain" if "plain" in kt else head
    N = grid.n
    field_bytes = co.ncomp * N ** 3 * 8
    planes_in = len(np.unique(prob.table("irregular") // (N * N)))
    planes_out = len(np.unique(prob.table("st_lin") // (N * N)))
    rows_in = len(np.unique(prob.table("irregular") // N))
    algo_of = {"dst_x": 2.0 * field_bytes, "dst_y": 2.0 * field_bytes, "dst_last": 2.0 * field_bytes,
               "dst_last_sparse": float(co.ncomp * N * N * 8 * (planes_in + planes_out)),
               "dst_last_out": float(field_bytes + co.ncomp * N * N * 8 * planes_out),
               "dst_x_fhn": (2.0 * field_bytes + (2.0 * field_bytes + co.ncomp * rows_in * N * 8)
                             + 3.0 * field_bytes) / 3.0}
    tot = {k: us * n for k, (us, n) in kt[ref].items()}
    priced = [k for k in algo_of if kt[ref][k][1] > 0]
    dom = max(priced, key=tot.get)
    avg_us, launches = kt[ref][dom]
    algo = algo_of[dom]
    achieved = algo / (avg_us * 1e-6) / 1e9
    traffic, traffic_src = measured_traffic(dom)
    roof = {"bound": "hbm", "kernel": f"k_{dom} (FP64, {ref} variant)", "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "traffic_source": traffic_src, "algorithmic_bytes_per_launch": algo, "avg_launch_us": round(avg_us, 2),
            "z_planes_read_written_by_dst_last_sparse": [planes_in, planes_out],
            "hbm_frac_by_class": {k: round(algo_of[k] / (kt[ref][k][0] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                  for k in priced},
            "note": ("dst_last_sparse transforms every z pencil like the dense pass but moves only the "
                     "planes that hold irregular or stencil nodes, so its time is set by the transform "
                     "work in LDS and registers rather than by HBM") if dom == "dst_last_sparse" else None,
            "algorithmic_bytes_per_launch_by_class": algo_of,
            "launches": launches,
            "kernel_timing": f"HIP events on the solve stream over the {a.kernel_steps} steps after the timed window",
            "kernel_avg_us": {k: round(v[0], 2) for k, v in kt[ref].items()},
            "kernel_share_of_timed_kernels": {k: round(v / sum(tot.values()), 3) for k, v in tot.items()}}
    out = {
        "metric": METRIC, "value": round(r["steps_per_s"], 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": n_warm, "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "plain" else "f32+f64",
        "data": "synthetic (seeded thick-shell geometry and stimulus ball)",
        "config": {"workload": f"FHN bidomain on a thick shell, {a.cells}^3 grid, {prob.M} interface nodes, "
                               f"dt=0.01, GMRES(50) tol 1e-8, timed steps {n_warm}-{n_warm + a.steps}",
                   "variant": head, "cells": a.cells,
                   "interface_nodes": prob.M, "crossings": prob.n_crossings, "parallelism": "single GPU"},
        "variants": {k: {kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in results.items()},
        "untimed_steps_before_window": n_warm,
        "speedup_vs_plain": round(r["steps_per_s"] / results["plain"]["steps_per_s"], 3) if "plain" in results else None,
        "roofline": roof,
        "setup_s": round(setup_s, 2),
        "autotuned_tile_widths": {"f64": list(prob.tiles(K.KFBI_F64)), "f32": list(prob.tiles(K.KFBI_F32))},
    }
    if not a.no_cpu_baseline and not a.profile_run:
        per_step = results[ref]["mean_matvecs_fp64"] + results[ref]["mean_matvecs_fp32"] + 2
        log("cpu baseline: timing the oracle's coupled box solve ...")
        out["cpu_baseline"] = cpu_baseline(grid, co, per_step)
    prob.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
