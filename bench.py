#!/usr/bin/env python3
"""Throughput of the BSGD hot path on one MI355X.

Workload: 2D fan beam 512x512 (0.5 mm), 720 views over 360 deg, 768 bins (1 mm),
SOD 500 mm, SDD 1000 mm, 8x8 image blocks, 16 angle subsets, importance sampling
by block column norms over 4 sub-detectors (BSGD-IM), node count 64 (Eq. 1:
one row block and all 64 column blocks per iteration). Synthetic seeded data:
24 random ellipses, Poisson noise at 1e5 incident photons, log transformed.

One step = one effective epoch (16 iterations): forward projection of the sampled
rays, residual rebuild, matched back projection fused with the block update.
Throughput = (forward + back projection ray-voxel updates) / s, where an update is
one nonzero a_ij applied; counts come from the exact per-(view, sub-detector,
block) nonzero table and the iteration's draws.

Prints one JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "c2_fan512_im"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def lipschitz_gpu(geom, n_vox, iters=20, seed=0):
    import torch
    v = torch.tensor(np.random.Generator(np.random.PCG64(seed)).uniform(size=n_vox), dtype=torch.float32,
                     device="cuda")
    lam = 0.0
    for _ in range(iters):
        w = geom.back_project(geom.forward_project(v))
        lam = float(torch.linalg.norm(w.double()))
        v = (w / lam).contiguous()
    return lam


def schedule_counts(geom, spec, rows, blocks, draws, nnz_tab, fp_rect, subdet_w):
    """Per-iteration exact update counts, z writes and selected voxels."""
    groups = geom.groups()
    S = spec.su * spec.sv
    per_it = []
    for it in range(rows.shape[0]):
        views = [v for i in rows[it] for v in groups[i]]
        U = 0
        zw = 0
        for a, v in enumerate(views):
            for b, j in enumerate(blocks[it]):
                s = int(draws[it, a, b])
                if s == -1:
                    continue
                if s == -2:
                    U += int(nnz_tab[v, :, j].sum())
                    u0, u1, v0, v1 = (int(t) for t in fp_rect[v, j])
                    zw += max(0, u1 - u0) * max(0, v1 - v0)
                else:
                    U += int(nnz_tab[v, s, j])
                    u0, u1, v0, v1 = (int(t) for t in fp_rect[v, j])
                    k0, k1 = subdet_w[s]
                    zw += max(0, min(u1, k1) - max(u0, k0)) * max(0, v1 - v0)
        per_it.append((U, zw, len(views)))
    return per_it


def profiled_traffic(workload_name, kernel_key):
    """HBM bytes per dispatch of a kernel from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel), or None when the kernel
    or launch sources changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
        src = b"".join(open(os.path.join(ROOT, "paper_1903_11874_amd", "csrc", n), "rb").read()
                       for n in ("bsgd_kernels.hip", "bsgd_device.h", "bsgd_kernels.h", "bsgd_capi.cpp"))
    except OSError:
        return None
    if hashlib.sha256(src).hexdigest() != t.get("source_sha256"):
        return None
    per = t.get("workloads", {}).get(workload_name, {})
    names = {"back_project_step": ["k_bp_step"], "forward_project": ["k_fp_pairs_lds", "k_fp_pairs"]}[kernel_key]
    for n in names:
        if n in per:
            return per[n]
    return None


def measure(geom, spec, solver, n_vox, warmup, steps, n_prof, workload_name):
    """Warm-up epochs, a timed region of `steps` epochs (captured HIP graphs, no
    events), then an event-timed eager region of `n_prof` epochs for per-kernel
    averages; exact update counts from the schedules; roofline of the dominant kernel."""
    import torch
    T = solver.epoch_iters
    args_warmup, args_steps = warmup, steps
    for _ in range(args_warmup):
        solver.step(T)
    r0 = solver.step(0, residual=True)
    torch.cuda.synchronize()

    # timed region: whole epochs, replayed as captured HIP graphs, no per-kernel events
    solver.set_profiling(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solver.step(T * args_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    rows, blocks, draws = solver.last_schedule()
    # second timed region of the same length with HIP events around every kernel
    # (eager launches on the solver's stream): per-kernel average durations
    base_times = solver.kernel_times()
    solver.set_profiling(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    solver.step(T * n_prof)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    times_p = solver.kernel_times()
    solver.set_profiling(False)
    times = {k: (times_p[k][0] - base_times[k][0], times_p[k][1] - base_times[k][1]) for k in times_p}
    prow, pblk, pdr = solver.last_schedule()
    r1 = solver.step(0, residual=True)

    nnz_tab = geom.table("nnz")
    fp_rect = geom.table("footprint")
    subdet_w = [((a * spec.nu) // spec.su, ((a + 1) * spec.nu) // spec.su) for a in range(spec.su)]
    per_it = schedule_counts(geom, spec, rows, blocks, draws, nnz_tab, fp_rect, subdet_w)
    U_fp = sum(p[0] for p in per_it)
    updates = 2 * U_fp
    value = updates / elapsed

    # roofline of the dominant kernel: algorithmic bytes per launch / mean launch time
    per_it_p = schedule_counts(geom, spec, prow, pblk, pdr, nnz_tab, fp_rect, subdet_w)
    n_it = len(per_it_p)
    vsel = n_vox * solver.blocks_per_iter // geom.info["n_blocks"]
    bytes_fp = sum(4 * u + 4 * zw for u, zw, _ in per_it_p) / n_it
    bytes_bp = sum(4 * u for u, _, _ in per_it_p) / n_it + vsel * (8 * solver.rows_per_iter + 16)
    avg_ms = {k: (ms / n if n else 0.0) for k, (ms, n) in times.items()}
    dominant = max(("forward_project", "back_project_step"), key=lambda k: times[k][0])
    alg_bytes = bytes_fp if dominant == "forward_project" else bytes_bp
    achieved = alg_bytes / (avg_ms[dominant] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(workload_name, dominant),
                "traffic_unit": "bytes per dispatch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms[dominant]}

    return {"elapsed": elapsed, "value": value, "updates": updates, "roofline": roofline,
            "kernels_avg_ms": avg_ms, "times": times, "r0": r0, "r1": r1, "n_prof": n_prof, "t2": t2, "t3": t3}


def cone_bench(steps, warmup, n_prof):
    """The 3D cone-beam workload with TV (256^3, 360 views of 384^2): same measurement."""
    import torch
    from bsgd_inputs.configs import workload
    from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise
    from paper_1903_11874_amd import Geometry, Solver
    wl = workload("c3_cone256_tv")
    spec = wl.geometry
    log("cone: geometry")
    geom = Geometry(spec)
    n_vox = spec.nx * spec.ny * spec.nz
    xt = torch.tensor(phantom_for(spec, wl.n_shapes, wl.phantom_seed), dtype=torch.float32, device="cuda")
    y = add_gaussian_noise(geom.forward_project(xt).double().cpu().numpy(), wl.noise_level, wl.noise_seed)
    yd = torch.tensor(y, dtype=torch.float32, device="cuda")
    del xt, y
    L = lipschitz_gpu(geom, n_vox, iters=6)
    mu = wl.solver.mu_scale / (2.0 * L)
    log(f"cone: L = {L:.4e}, mu = {mu:.4e}")
    x = torch.zeros(n_vox, dtype=torch.float32, device="cuda")
    solver = Solver(geom, yd, x, node_count=64, mu=mu, seed=wl.solver.seed, tv_lambda=wl.solver.tv_lambda,
                    tv_inner_iters=wl.solver.tv_inner_iters)
    m = measure(geom, spec, solver, n_vox, warmup, steps, n_prof, wl.name)
    T = solver.epoch_iters
    return {"workload": wl.description, "metric": "FP+BP ray-voxel updates/s", "value": m["value"],
            "unit": "updates/s", "steps": steps, "ms_per_step": m["elapsed"] / steps * 1e3,
            "rows_per_iter": solver.rows_per_iter, "blocks_per_iter": solver.blocks_per_iter,
            "iters_per_step": T, "step": "one effective epoch (TV prox once per epoch)",
            "roofline": m["roofline"], "kernels_avg_ms": m["kernels_avg_ms"],
            "kernel_launches": {k: n for k, (ms, n) in m["times"].items()},
            "residual_norm": {"before": m["r0"], "after": m["r1"]}, "updates_per_step": m["updates"] / steps}


def cpu_baseline(spec, x, budget_s=12.0):
    """The FP64 oracle's matrix-free FP + BP over every ray, repeated to a bounded time budget."""
    from oracle.cfast import Projector
    threads = max(1, min(16, os.cpu_count() or 1))
    P = Projector(spec)
    updates, elapsed, reps = 0, 0.0, 0
    while elapsed < budget_s and reps < 200:
        t0 = time.perf_counter()
        y = P.fp(x, threads=threads)
        P.bp(y, threads=threads)
        elapsed += time.perf_counter() - t0
        updates += 2 * P.last_nnz
        reps += 1
    return {"value": updates / elapsed, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} x (FP + BP over all {spec.n_views} views x {spec.nu} bins, full "
                      f"{spec.nx}x{spec.ny} image), FP64 matrix-free Siddon, {threads} threads: "
                      f"{updates:.3e} updates in {elapsed:.2f} s"}


def serving_bench(n_requests, rate, max_slots, tol, max_epochs, seed=4004):
    """Continuous-batching server vs the plain per-solve loop on a seeded Poisson stream
    of 2D fan-beam solves (sides 128..1024, views = bins = 1.5 side, 1% noise)."""
    import torch
    from bsgd_inputs.configs import SERVING_SIDES, fan_request_geometry
    from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise
    from paper_1903_11874_amd.serving import Request, Server, latency_stats
    rng = np.random.Generator(np.random.PCG64(seed))
    server = Server(max_slots=max_slots)
    mus = {}
    reqs = []
    truths = {}
    t = 0.0
    for rid in range(n_requests):
        t += rng.exponential(1.0 / rate)
        side = int(rng.choice(SERVING_SIDES))
        spec = fan_request_geometry(side)
        if spec not in server.geoms:
            log(f"serving: geometry side {side}")
        geom = server.geometry(spec)
        if spec not in mus:
            mus[spec] = 0.5 / (2.0 * lipschitz_gpu(geom, spec.nx * spec.ny, iters=15))
        x_true = torch.tensor(phantom_for(spec, 10, 5000 + rid), dtype=torch.float32, device="cuda")
        truths[rid] = x_true
        y = add_gaussian_noise(geom.forward_project(x_true).double().cpu().numpy(), 0.01, 6000 + rid)
        reqs.append(Request(rid=rid, geometry=spec, y=torch.tensor(y, dtype=torch.float32, device="cuda"),
                            arrival=t, mu=mus[spec], seed=rid, node_count=64, tol=tol, max_epochs=max_epochs,
                            check_every=5))
    torch.cuda.synchronize()
    log(f"serving: {n_requests} requests over {t:.2f} s, sides {sorted(set(r.geometry.nx for r in reqs))}")
    log("serving: batched run")
    served = server.run(reqs)
    log("serving: sequential run")
    seq = Server(max_slots=1).run_sequential(reqs)
    same = all(torch.equal(a.x, b.x) for a, b in zip(served, seq))
    st_b, st_s = latency_stats(served), latency_stats(seq)

    def snr(results):  # image SNR against each request's phantom, 20 log10(|x_true| / |x_true - x|)
        v = [float(20.0 * torch.log10(truths[r.rid].double().norm() / (truths[r.rid].double() - r.x.double()).norm()))
             for r in results]
        return {"mean_snr_db": float(np.mean(v)), "min_snr_db": float(np.min(v))}

    st_b.update(snr(served))
    st_s.update(snr(seq))
    return {"requests": n_requests, "rate_per_s": rate, "arrival_span_s": t, "max_slots": max_slots,
            "stop_rule": f"||A^T(y-Ax)||/||A^T y|| <= {tol} checked every 5 epochs, at most {max_epochs} epochs",
            "batched": st_b, "sequential": st_s,
            "solves_per_s_ratio": st_b["solves_per_s"] / st_s["solves_per_s"],
            "identical_results": bool(same),
            "max_active": max(e[1] for e in server.log) if server.log else 0,
            "ticks": len(server.log),
            "enqueue_s": sum(e[2] for e in server.log), "check_and_wait_s": sum(e[3] for e in server.log)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving", type=int, default=48,
                    help="requests of the continuous-batching serving measurement (0 = skip)")
    ap.add_argument("--serving-tol", type=float, default=1e-3)
    ap.add_argument("--serving-max-epochs", type=int, default=30)
    ap.add_argument("--cone-steps", type=int, default=3,
                    help="epochs of the 3D cone-beam (256^3, TV) measurement reported as 'secondary' (0 = skip)")
    ap.add_argument("--cone-only", action="store_true",
                    help="profiling aid: run only the cone-beam measurement and print its object")
    ap.add_argument("--tune", default="auto",
                    help="forward-projector launch shape: 'auto' (autotuner, before the timed region) "
                         "or 'V,S' (views per workgroup, lanes per ray)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters) and exit")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="epochs of the event-timed second region (0 = same as --steps)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the hot path has no multi-GPU mode)", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_probe:
        n = (1 << 30) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))
        return
    if args.cone_only:
        print(json.dumps(cone_bench(max(1, args.cone_steps), 1, max(1, args.cone_steps))), flush=True)
        return
    from bsgd_inputs.configs import workload
    from bsgd_inputs.phantoms import phantom_for, poisson_log_noise
    from paper_1903_11874_amd import Geometry, Solver

    wl = workload(WORKLOAD)
    spec = wl.geometry
    dev = torch.device("cuda:0")
    log("geometry")
    geom = Geometry(spec)
    n_vox = spec.nx * spec.ny * spec.nz
    x_true = phantom_for(spec, wl.n_shapes, wl.phantom_seed)
    xt = torch.tensor(x_true, dtype=torch.float32, device=dev)
    y_clean = geom.forward_project(xt).double().cpu().numpy()
    y = poisson_log_noise(y_clean, wl.noise_level, wl.noise_seed)
    yd = torch.tensor(y, dtype=torch.float32, device=dev)
    L = lipschitz_gpu(geom, n_vox)
    mu = wl.solver.mu_scale / (2.0 * L)
    log(f"L = {L:.4e}, mu = {mu:.4e}")

    if args.tune == "auto":
        from paper_1903_11874_amd.tuning import autotune
        tt = autotune(geom, yd, node_count=64, mu=mu, epochs=2, seed=wl.solver.seed)
        log("autotune: " + ", ".join(f"{k}: {v * 1e3:.3f} ms" for k, v in sorted(tt.items(), key=lambda kv: kv[1])[:4]))
    else:
        v_, s_ = (int(t) for t in args.tune.split(","))
        geom.set_tuning(fp_views_per_group=v_, fp_ray_split=s_)
    log(f"forward projector shape: {geom.fp_views_per_group} views per workgroup, {geom.fp_ray_split} lanes per ray")

    x = torch.zeros(n_vox, dtype=torch.float32, device=dev)
    solver = Solver(geom, yd, x, node_count=64, mu=mu, seed=wl.solver.seed)
    T = solver.epoch_iters
    log(f"alpha M = {solver.rows_per_iter}, gamma N = {solver.blocks_per_iter}, epoch = {T} iterations")

    m = measure(geom, spec, solver, n_vox, args.warmup, args.steps,
                args.profile_steps if args.profile_steps > 0 else args.steps, wl.name)
    elapsed, value, updates, roofline, avg_ms, times = (m["elapsed"], m["value"], m["updates"], m["roofline"],
                                                        m["kernels_avg_ms"], m["times"])
    r0, r1, n_prof, t2, t3 = m["r0"], m["r1"], m["n_prof"], m["t2"], m["t3"]

    out = {
        "metric": "FP+BP ray-voxel updates/s",
        "value": value,
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-ellipse phantom, Poisson noise)",
        "config": {"workload": "2D fan-beam BSGD-IM 512x512 @0.5 mm, 720 views/360 deg, 768 bins @1 mm, "
                               "SOD 500 SDD 1000, 8x8 blocks, 16 angle subsets, 4 sub-detectors, node count 64",
                   "rows_per_iter": solver.rows_per_iter, "blocks_per_iter": solver.blocks_per_iter,
                   "iters_per_step": T, "step": "one effective epoch",
                   "fp_views_per_group": geom.fp_views_per_group, "fp_ray_split": geom.fp_ray_split},
        "roofline": roofline,
        "kernels_avg_ms": avg_ms,
        "kernel_launches": {k: n for k, (ms, n) in times.items()},
        "kernel_timing": f"HIP events around every kernel in a second timed region of {n_prof} epochs "
                         f"(eager launches): {(t3 - t2) / n_prof * 1e3:.4f} ms per epoch; the first timed region "
                         "replays captured HIP graphs without events",
        "residual_norm": {"before": r0, "after": r1},
        "updates_per_step": updates / args.steps,
    }
    if args.cone_steps > 0:
        del solver, x, yd, geom
        torch.cuda.empty_cache()
        out["secondary"] = cone_bench(args.cone_steps, 1, args.cone_steps)
    if args.serving > 0:
        out["serving"] = serving_bench(args.serving, 20.0, 32, args.serving_tol, args.serving_max_epochs)
    if not args.no_cpu_baseline:
        log("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(spec, x_true)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
