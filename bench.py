#!/usr/bin/env python3
"""Benchmark: FitzHugh-Nagumo bidomain steps/s on a 256^3 grid with the KFBI diffusion solve.

Workload (synthetic, seeded): box [-1.2, 1.2]^3 with 256 cells per axis (255^3 unknowns per
component, coupled intra/extracellular pair); a closed thick shell (outer ellipsoid
0.9/0.7/0.6, inner wall 0.6 x ellipsoid with seeded smooth radial noise) carrying 40,960
interface nodes; sigma_i = 1, sigma_e = 2, Cm = beta = 1, dt = 0.01 (kappa = 200);
FHN theta = 0.13, H = 100, alpha = 0.25, zeta = 1; V = 1 in a ball of radius 0.25 at a
seeded mid-wall point, the same ball set to V = 1 again at step 300 (a second beat: the tissue
is excitable again about 300 steps after a beat); GMRES(50) relative tolerance 1e-8 on ||g'||.

Schedule (the same for every variant, from the same initial state): the first 200 steps
(the learned variant records them and trains its network on them afterwards), then --warmup
untimed steps, then --steps timed steps (by default 295, so the run is the 500 steps of the
workload), then steps after the window for per-kernel HIP-event timing and for the FP64
residual check by explicit products.  A step is one whole Strang step (reaction, coupled KFBI
Neumann solve, reaction) with all inputs resident in HBM.

Variants: plain (FP64, GMRES from psi^{n-1}); mixed (one GMRES whose products turn FP32 once
the residual allows, with an FP64 product certifying the result); learned (the value: start
from the least-residual combination of the last 8 solutions, one minimal-residual step along the
trained network's predicted correction, mixed precision as in mixed); projected and projected_mixed (the
learned variant without the network, in FP64 and mixed precision); mixed_ir (FP32 inner GMRES
with FP64 iterative refinement); richardson (the simple iteration, gamma = 0.8, FP64).  Every
solve ends at the same FP64 relative residual bound.

Also reported: the batched 2D workload (problems/s) and the paper's own examples in its parameter
regime (GMRES iterations per step, steps/s, the simple iteration's residual).

Prints one JSON line (see the "metric" key).  --batch and --copy-calibration run the batched
2D workload and the counter calibration alone.
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
PREFIX = 200          # the first steps of the workload: the learned variant trains on them
PACE_AT = 300         # second stimulus of the seeded ball


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500 - PREFIX - 5)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cells", type=int, default=256)
    ap.add_argument("--nodes", type=int, default=40960)
    ap.add_argument("--variants", default="plain,mixed,learned,projected,projected_mixed,mixed_ir,richardson")
    ap.add_argument("--epochs", type=int, default=150)
    ap.add_argument("--switch", type=float, default=2e-3,
                    help="mixed precision: relative residual below which the products run in FP32")
    ap.add_argument("--inner-tol", type=float, default=1e-4, help="mixed_ir: relative tolerance of each FP32 inner solve")
    ap.add_argument("--kernel-steps", type=int, default=10, help="steps after the timed window timed per kernel")
    ap.add_argument("--check-steps", type=int, default=10,
                    help="steps after those whose FP64 residual is checked by an explicit product")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="leave the batched 2D workload out of the line")
    ap.add_argument("--no-examples", action="store_true", help="leave the paper's examples out of the line")
    ap.add_argument("--profile-run", action="store_true",
                    help="short run for rocprofv3 (first listed variant only, no CPU baseline, no batch)")
    ap.add_argument("--prefix", type=int, default=PREFIX,
                    help="untimed steps before the warm-up (the workload's first 200; fewer only for profiling "
                         "runs, which then no longer time the workload's window)")
    ap.add_argument("--batch", action="store_true",
                    help="only the batched 2D workload: 64 seeded Neumann problems of sizes 64..1024, "
                         "solved as one batch and one by one (problems/s)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only time plain copies of one coupled FP64 field (the reference kernels for "
                         "scaling the FETCH_SIZE / WRITE_SIZE counters)")
    return ap.parse_args()


def cpu_baseline(iface, grid, co, p, dt, V0, q0):
    """The oracle as it stands (FP64 NumPy/SciPy, FFTs on every host core) on a bounded sample of the
    same workload: one bidomain step from the initial state (GMRES from zero, tolerance 1e-8) and
    one matrix-vector product, timed after the oracle's setup (setup excluded, stated)."""
    import numpy as np

    from oracle import bidomain as obd
    from oracle import boxsolve as obs
    from oracle import kfbi as ok
    t0 = time.perf_counter()
    o = ok.Problem(iface, grid, co)
    o.null_density()   # the coupled pair's null density: once per problem, part of the setup
    setup_s = time.perf_counter() - t0
    log(f"cpu baseline: oracle setup {setup_s:.1f} s (with the null density); timing one oracle step ...")
    t0 = time.perf_counter()
    _, _, _, _, info = obd.step(o, p, V0, q0, dt, tol=1e-8)
    step_s = time.perf_counter() - t0
    psi = np.random.default_rng(0).uniform(-1, 1, size=(2, o.M))
    t0 = time.perf_counter()
    o.apply(psi)
    apply_s = time.perf_counter() - t0
    return {"value": 1.0 / step_s, "unit": "steps/s", "cores": obs.WORKERS, "kind": "oracle step, timed",
            "sample": f"one oracle bidomain step of this workload from its initial state ({step_s:.1f} s, "
                      f"{info['iters']} GMRES iterations from zero at tolerance 1e-8) and one coupled "
                      f"matrix-vector product ({apply_s:.2f} s); oracle setup ({setup_s:.0f} s, tables and the coupled "
                      f"pair's null density) excluded; "
                      f"scipy.fft with {obs.WORKERS} workers",
            "apply_s": round(apply_s, 3), "step_s": round(step_s, 2), "setup_s": round(setup_s, 1),
            "host_cpu": platform.processor() or platform.machine(),
            "host_cores_available": len(os.sched_getaffinity(0))}


def measured_traffic(kernel):
    """HBM bytes per launch of a DST pass from the committed rocprofv3 counter summary
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


def batch_run(torch, warmup=1, reps=5, singles=True):
    """64 seeded 2D Neumann problems (manufactured u = e^x sin(pi y)), FP32 inner GMRES with
    FP64 refinement to 1e-10 per problem: one batch (each DST pass one launch over all size
    groups; also timed with one launch per group and pass), and (singles) the problems one at a
    time."""
    import numpy as np

    from paper_2104_05024_amd import kfbi as K
    from paper_2104_05024_amd import workloads as W
    probs = W.batch_2d()
    t0 = time.perf_counter()
    b = K.Batch(probs)
    setup_s = time.perf_counter() - t0
    dev = torch.device("cuda:0")
    fs, gs = [], []
    for (iface, grid, co) in probs:
        pts = W.grid_points(grid)
        fs.append((np.pi ** 2 - 1 + co.kappa) * np.exp(pts[:, 0]) * np.sin(np.pi * pts[:, 1]))
    for pr in probs:
        h = K.Problem(*pr, host_only=True)     # node positions and normals (host tables only)
        X, n = h.table("nodes_X").reshape(-1, 2), h.table("nodes_n").reshape(-1, 2)
        h.close()
        gs.append(n[:, 0] * np.exp(X[:, 0]) * np.sin(np.pi * X[:, 1])
                  + n[:, 1] * np.pi * np.exp(X[:, 0]) * np.cos(np.pi * X[:, 1]))
    f = torch.tensor(np.concatenate(fs), device=dev)
    g = torch.tensor(np.concatenate(gs), device=dev)
    opts = dict(tol=1e-10, precision=1, inner_tol=1e-4)
    for _ in range(max(warmup, 1)):
        b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        u, psi, infos = b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    # the same solves with one DST launch per size group and pass
    b.merge(False)
    b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        b.solve_neumann(g, f, **opts)
    torch.cuda.synchronize()
    t_grouped = (time.perf_counter() - t0) / reps
    b.merge(True)
    out = {"problems_per_s": round(b.n / t_batch, 1), "n_problems": b.n, "ms_per_batch": round(1000 * t_batch, 2),
           "grouped_launches_problems_per_s": round(b.n / t_grouped, 1),
           "max_final_rel_resid": max(i["rel_resid"] for i in infos),
           "mean_inner_iters": float(np.mean([i["iters"] for i in infos])), "setup_s": round(setup_s, 2),
           "cells": sorted(set(gr.cells for _, gr, _ in probs))}
    if singles:
        ps = [K.Problem(*pr) for pr in probs]
        segs = [(f[b.goff[i]:b.goff[i] + b.N[i] ** 2].reshape(1, -1).contiguous(),
                 g[b.ioff[i]:b.ioff[i] + b.M[i]].reshape(1, -1).contiguous()) for i in range(b.n)]
        for p, (fi, gi) in zip(ps, segs):
            p.solve_neumann(gi, fi, **opts)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for p, (fi, gi) in zip(ps, segs):
                p.solve_neumann(gi, fi, **opts)
        torch.cuda.synchronize()
        t_single = (time.perf_counter() - t0) / reps
        out["one_at_a_time_problems_per_s"] = round(b.n / t_single, 1)
        out["speedup_vs_one_at_a_time"] = round(t_single / t_batch, 2)
        for p in ps:
            p.close()
    b.close()
    return out


def paper_examples(torch):
    """The paper's own regime (anisotropic D_i = diag(30, 5[, 5]), D_e = diag(20, 10[, 10]), beta = 1000,
    dt = h, virtual electrode): GMRES iterations per step and steps/s for Example 1 (circle, 256^2,
    128 steps) and Example 3 (sphere, 128^3, 32 steps), for the sphere also the simple iteration
    (gamma = 0.8; the coupled pair's residual measured without its null-density component)."""
    import numpy as np

    from paper_2104_05024_amd import kfbi as K
    from paper_2104_05024_amd import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    for key, fn, cells, steps in (("example1_circle_256", W.paper_circle_example, 256, 128),
                                  ("example3_sphere_128", W.paper_sphere_example, 128, 32)):
        iface, grid, co, p, dt, stim = fn(cells)
        prob = K.Problem(iface, grid, co)
        n = grid.n ** grid.dim
        Is = torch.tensor(stim, device=dev)
        res = {"cells": cells, "interface_nodes": prob.M, "steps": steps, "dt": dt}
        runs = [("gmres", dict(), steps, False)]
        if grid.dim == 3:
            runs += [("simple_iteration", dict(method=1, gamma=0.8, max_iters=500), steps, False)]
        for tag, kw, ns, noconv in runs:
            bd = K.Bidomain(prob, p, tol=1e-8, **kw)
            V = torch.zeros(n, dtype=torch.float64, device=dev)
            q = torch.zeros_like(V)
            hist = torch.zeros(2, 2, prob.M, dtype=torch.float64, device=dev)
            bd.step(V, q, hist, dt, I_stim=Is, allow_noconv=noconv)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            infos = [bd.step(V, q, hist, dt, I_stim=Is, allow_noconv=noconv) for _ in range(ns - 1)]
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            if tag == "gmres":
                res.update(gmres_iters_per_step=round(float(np.mean([i["iters"] for i in infos])), 2),
                           steps_per_s=round((ns - 1) / el, 1), max_rel_resid=max(i["rel_resid"] for i in infos),
                           V_max=round(float(V.max().item()), 4))
            else:
                res.update(simple_iteration_iters_per_step=round(float(np.mean([i["iters"] for i in infos])), 2),
                           simple_iteration_steps_per_s=round((ns - 1) / el, 1),
                           simple_iteration_max_rel_resid=max(i["rel_resid"] for i in infos))
            bd.close()
        prob.close()
        out[key] = res
        log(f"{key}: {res}")
    return out


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


# variant -> Bidomain keyword arguments
def variant_kwargs(name, a):
    mixed = dict(precision=2, inner_tol=a.switch)
    return {
        "plain": dict(precision=0, warm_start=0),
        "mixed": dict(warm_start=0, **mixed),
        "learned": dict(warm_start=4, **mixed),
        "projected": dict(precision=0, warm_start=3),
        "projected_mixed": dict(warm_start=3, **mixed),
        "mixed_ir": dict(precision=1, warm_start=0, inner_tol=a.inner_tol),
        "richardson": dict(precision=0, warm_start=0, method=1, gamma=0.8, max_iters=400),
    }[name]


KERNELS = ("dst_x", "dst_y", "dst_last", "dst_x_rows", "dst_y_sparse", "dst_last_sparse", "dst_last_out",
           "dst_x_fhn", "dst_x_fe1", "dst_y1", "dst_last_anti", "dst_last_diff", "dst_last_comb", "dst_x_be1", "jumps",
           "correct", "gather")


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
        out = batch_run(torch, warmup=max(a.warmup, 1), reps=max(1, min(a.steps, 10)))
        print(json.dumps({"metric": "batched 2D Neumann solves, problems/s (FP32 inner + FP64 refinement to 1e-10)",
                          "value": out["problems_per_s"], "unit": "problems/s", **out,
                          "data": "synthetic (seeded stars, manufactured solution)",
                          "config": {"workload": "64 star-shaped 2D Neumann problems, cells in {64,...,1024}, "
                                                 "3-8 lobes, amplitude 0.05-0.2, kappa 50-2000, M = 2 cells"}}))
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
    ball = torch.tensor(V0 > 0.5, device=dev)
    tissue = torch.tensor(prob.table("inside").astype(bool), device=dev)
    n_tissue = float(tissue.sum())

    variants = [v for v in a.variants.split(",") if v]
    if a.profile_run:
        variants = variants[:1]
    t_win0 = a.prefix + a.warmup
    results, kt = {}, {}
    for name in variants:
        bd = K.Bidomain(prob, p, tol=1e-8, **variant_kwargs(name, a))
        if name == "learned":
            bd.mlp_init(capacity=max(a.prefix, 1), seed=3)
        V = torch.tensor(V0, device=dev)
        q = torch.tensor(q0, device=dev)
        hist = torch.zeros(2, 2, prob.M, dtype=torch.float64, device=dev)
        step_no = 0

        def step(v=name):
            nonlocal step_no
            if step_no == PACE_AT:
                V[ball] = 1.0
            step_no += 1
            return bd.step(V, q, hist, dt)

        for _ in range(a.prefix):
            step()
        if name == "learned":
            loss = bd.train(epochs=a.epochs, lr=1e-3)
            log(f"learned: network trained on steps 1-{a.prefix}, loss {loss:.3e}")
        for _ in range(a.warmup):
            step()
        exc0 = float(((V > 0.5) & tissue).sum()) / n_tissue
        infos = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            infos.append(step())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        exc1 = float(((V > 0.5) & tissue).sum()) / n_tissue
        # per-kernel HIP-event timing over the next steps (event timing launches every kernel
        # directly, so it stays out of the timed window, where GMRES replays captured steps)
        prob.profile(True)
        for _ in range(a.kernel_steps):
            step()
        torch.cuda.synchronize()
        kt[name] = {k: prob.kernel_time(k) for k in KERNELS}
        prob.profile(False)
        # the FP64 residual of the following solves by explicit products
        bd.true_resid(True)
        checks = [step() for _ in range(a.check_steps)]
        bd.true_resid(False)
        results[name] = {
            "steps_per_s": a.steps / el, "ms_per_step": 1000 * el / a.steps,
            "mean_iters": float(np.mean([i["iters"] for i in infos])),
            "mean_matvecs_fp64": float(np.mean([i["matvecs_fp64"] for i in infos])),
            "mean_matvecs_fp32": float(np.mean([i["matvecs_fp32"] for i in infos])),
            "max_final_rel_resid": max(i["rel_resid"] for i in infos),
            "max_true_rel_resid": max(i["true_resid"] for i in checks) if checks else None,
            "mean_start_resid": float(np.mean([i["start_resid"] for i in infos])),
            "start_used": int(sum(i["warm_start_used"] & 1 for i in infos)),
            "learned_step_tried": int(sum((i["warm_start_used"] >> 2) & 1 for i in infos)),
            "learned_step_taken": int(sum((i["warm_start_used"] >> 1) & 1 for i in infos)),
            "fp64_checks": int(sum(i["outer"] for i in infos)) if name in ("mixed", "learned", "projected_mixed") else 0,
            "excited_fraction_window_start_end": [round(exc0, 3), round(exc1, 3)],
            "V_max": float(V.max().item()),
        }
        log(f"{name}: {results[name]}")
        bd.close()

    head = "learned" if "learned" in results else ("mixed" if "mixed" in results else variants[0])
    r = results[head]
    for name in results:
        m64, m32 = results[name]["mean_matvecs_fp64"], results[name]["mean_matvecs_fp32"]
        results[name]["products_per_step"] = round(m64 + m32, 3)

    # roofline of the dominant FP64 pencil kernel (plain variant: every launch is FP64).  Dense
    # passes (dst_x, dst_y, dst_last) read and write the whole coupled field.  The matvec's z pass
    # (dst_last_sparse) reads only the z planes holding irregular nodes and writes only those holding
    # extrapolation-stencil nodes; the volume solve's z pass (dst_last_out) reads every plane and
    # writes the stencil planes.  The row-list x pass (dst_x_rows) reads and writes the rows holding
    # irregular nodes (forward) or stencil nodes (inverse); the masked y pass (dst_y_sparse) reads the
    # irregular rows and writes whole planes that hold any (forward), or reads whole stencil planes
    # and writes the stencil rows (inverse); each is priced per launch as the mean of its two forms.
    # The x passes of a step's box solves that carry the reaction (dst_x_fhn) are priced as the mean
    # of: forward Euler + source (V, q read, the pair written), source + correction (V, q and the
    # correction rows read, the pair written) and inverse + backward Euler (the pair, V and q read,
    # V, q written).  Without a stimulus current the volume solve's source is antisymmetric and its
    # forward passes run over one field: dst_x_fe1 (V, q read, one field written), dst_y1 (one field
    # read and written) and dst_last_anti (one field read, the stencil planes of both components
    # written).  When the potentials are not returned, the final solve needs only Phi_i - Phi_e:
    # dst_last_diff (the pair read, one field written), dst_y1 again for its inverse y pass, and
    # dst_x_be1 (one field, V and q read, V and q written).  Without a stimulus current as well, that
    # z pass (dst_last_comb) adds C psi's transform, taken through the masked row and plane passes,
    # to the volume solve's transform of kappa V1 as it loads: one field and the irregular planes of
    # the pair read, one field written.  dst_x_fhn is priced as the mean of the forms it still holds.
    ref = "plain" if "plain" in kt else head
    N = grid.n
    nc = co.ncomp
    field_bytes = nc * N ** 3 * 8
    irr = prob.table("irregular")
    stl = prob.table("st_lin")
    planes_in, planes_out = len(np.unique(irr // (N * N))), len(np.unique(stl // (N * N)))
    rows_in, rows_out = nc * len(np.unique(irr // N)), nc * len(np.unique(stl // N))
    algo_of = {"dst_x": 2.0 * field_bytes, "dst_y": 2.0 * field_bytes, "dst_last": 2.0 * field_bytes,
               "dst_last_sparse": float(nc * N * N * 8 * (planes_in + planes_out)),
               "dst_last_out": float(field_bytes + nc * N * N * 8 * planes_out),
               "dst_x_rows": float((rows_in + rows_out) * N * 8),
               "dst_y_sparse": float(((rows_in * N + planes_in * nc * N * N) + (planes_out * nc * N * N + rows_out * N))
                                     * 8 / 2),
               "dst_x_fe1": 1.5 * field_bytes, "dst_y1": float(field_bytes),
               "dst_last_anti": float(field_bytes / 2 + nc * N * N * 8 * planes_out),
               "dst_last_diff": 1.5 * field_bytes, "dst_x_be1": 2.5 * field_bytes,
               "dst_last_comb": float(field_bytes + nc * N * N * 8 * planes_in),
               "dst_x_fhn": float(np.mean(([2.0 * field_bytes + rows_in * N * 8]
                                           if kt[ref]["dst_last_comb"][1] == 0 else [])
                                          + ([2.0 * field_bytes] if kt[ref]["dst_x_fe1"][1] == 0 else [])
                                          + ([3.0 * field_bytes] if kt[ref]["dst_x_be1"][1] == 0 else [])
                                          or [0.0]))}
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
            "launches": launches,
            "z_planes_read_written_by_dst_last_sparse": [planes_in, planes_out],
            "rows_in_out": [rows_in, rows_out],
            "hbm_frac_by_class": {k: round(algo_of[k] / (kt[ref][k][0] * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)
                                  for k in priced},
            "traffic_by_class": {k: measured_traffic(k)[0] for k in priced},
            "algorithmic_bytes_per_launch_by_class": algo_of,
            "kernel_timing": f"HIP events on the solve stream over the {a.kernel_steps} steps after the timed window",
            "kernel_avg_us": {k: round(v[0], 2) for k, v in kt[ref].items()},
            "kernel_share_of_timed_kernels": {k: round(v / sum(tot.values()), 3) for k, v in tot.items()}}
    if "mixed" in kt:
        roof["kernel_avg_us_mixed_variant"] = {k: round(v[0], 2) for k, v in kt["mixed"].items()}
    out = {
        "metric": METRIC, "value": round(r["steps_per_s"], 3), "unit": "steps/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": round(r["ms_per_step"], 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head in ("plain", "projected", "richardson") else "f32+f64",
        "data": "synthetic (seeded thick-shell geometry, stimulus ball at steps 0 and 300)",
        "config": {"workload": f"FHN bidomain on a thick shell, {a.cells}^3 grid, {prob.M} interface nodes, "
                               f"dt=0.01, GMRES(50) tol 1e-8, {a.prefix} untimed steps (the learned variant's "
                               f"training data) + {a.warmup} warm-up, timed steps {t_win0 + 1}-{t_win0 + a.steps}",
                   "variant": head, "cells": a.cells,
                   "interface_nodes": prob.M, "crossings": prob.n_crossings, "parallelism": "single GPU"},
        "prefix_steps": a.prefix,
        "variants": {k: {kk: (float(f"{vv:.4g}") if isinstance(vv, float) else vv) for kk, vv in v.items()}
                     for k, v in results.items()},
        "speedup_vs_plain": {k: round(v["steps_per_s"] / results["plain"]["steps_per_s"], 3) for k, v in results.items()}
        if "plain" in results else None,
        "roofline": roof,
        "setup_s": round(setup_s, 2),
        "autotuned_tile_widths": {"f64": list(prob.tiles(K.KFBI_F64)), "f32": list(prob.tiles(K.KFBI_F32))},
    }
    prob.close()
    if not a.no_batch and not a.profile_run:
        log("batched 2D workload ...")
        out["batch"] = batch_run(torch, singles=False)
    if not a.no_examples and not a.profile_run:
        log("the paper's examples ...")
        out["paper_examples"] = paper_examples(torch)
    if not a.no_cpu_baseline and not a.profile_run:
        out["cpu_baseline"] = cpu_baseline(iface, grid, co, p, dt, V0, q0)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
