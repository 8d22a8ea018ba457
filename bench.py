#!/usr/bin/env python3
"""Throughput of the BSGD hot path on one MI355X.

Headline workload: 3D cone beam with TV, 256^3 volume (0.5 mm voxels), 360 views over
360 deg onto a 384x384 detector (1 mm pixels), SOD 600 mm, SDD 1200 mm, 256 column
blocks (16 axial slabs x 4x4 tiles of 64x64x16), 24 angle subsets, TV weight 1e-3 with
20 inner iterations, node count 64 (Eq. 1: one row block and 64 column blocks per
iteration, 96 iterations per effective epoch). Synthetic seeded data: 32 random
ellipsoids, Gaussian noise at 1% of the maximum.

One step = one effective epoch: forward projection of the selected rays, residual
rebuild, matched back projection fused with the block update, and the TV prox.
Throughput = (forward + back projection ray-voxel updates) / s, where an update is one
nonzero a_ij applied; counts come from the exact per-(view, sub-detector, block)
nonzero table and the iteration's draws.

Also reported: the 2D fan-beam BSGD-IM workload (512^2) as `secondary`; the FP64 oracle
on the host cores (`cpu_baseline`); the serving mix (512 seeded Poisson requests of 2D
fan-beam solves, sides 128..1024) at the workload's 20 requests/s and at a saturating
rate, served with continuous batching against the plain per-solve loop.

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
# VALU issue of the chip: 256 CUs x 4 SIMDs, one wave64 instruction per SIMD every 4
# cycles (16 lanes per cycle) at 2.4 GHz
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
SIMDS = 256 * 4
CLOCK_HZ = 2.4e9


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


KERNEL_NAMES = {"back_project_step": ["k_bp_step"], "forward_project": ["k_fp_pairs_lds", "k_fp_pairs"]}


def profiled(workload_name, kernel_key):
    """The committed rocprofv3 counter runs of a kernel (profiles/traffic.json): HBM bytes
    per dispatch (FETCH_SIZE and WRITE_SIZE scaled by a plain copy kernel) and wave64
    VALU instructions per dispatch (SQ_INSTS_VALU); None when the kernel or launch
    sources changed since those counters were taken."""
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
    for n in KERNEL_NAMES[kernel_key]:
        if n in per:
            return per[n]
    return None


TRAFFIC_WORKLOADS = ("c3_cone256_tv", "c2_fan512_im")


def _kernel_base(name):
    """Kernel name without namespaces, template arguments and parameters."""
    n = name.replace("(anonymous namespace)::", "").split("(")[0].split("<")[0]
    return n.split("::")[-1].replace("void ", "").strip()


def _counters(db):
    """{kernel: {counter: mean value per dispatch}} from a rocprofv3 --pmc database."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select kernel_name, counter_name, count(distinct dispatch_id), sum(value) "
                     "from counters_collection group by kernel_name, counter_name").fetchall()
    out = {}
    for name, counter, n, total in rows:
        k = _kernel_base(name)
        d = out.setdefault(k, {})
        # template instances of one kernel are pooled
        acc = d.setdefault(counter, [0, 0.0])
        acc[0] += n
        acc[1] += total
    return {k: {cn: v[1] / v[0] for cn, v in d.items()} for k, d in out.items()}


def _kernel_times(db):
    """{kernel: (calls, mean us, min us, max us)} from a rocprofv3 --kernel-trace database."""
    import sqlite3
    c = sqlite3.connect(db)
    rows = c.execute("select name, end - start from kernels").fetchall()
    out = {}
    for name, dt in rows:
        out.setdefault(_kernel_base(name), []).append(dt / 1e3)
    return {k: (len(v), sum(v) / len(v), min(v), max(v)) for k, v in out.items()}


def write_traffic(d):
    """Write profiles/traffic.json from the rocprofv3 databases under d and print the
    per-kernel tables: d/copy_fetch, d/copy_write (FETCH_SIZE / WRITE_SIZE of the copy
    probe), and per workload w: d/w_trace (kernel trace), d/w_fetch, d/w_write, d/w_sq
    (SQ_INSTS_VALU and other SQ counters) and, when present, d/w_ta (TA/TD busy cycles
    summed over CUs, L2 hits and misses). HBM bytes per dispatch are the KiB counters
    scaled so that the 1 GiB copy reads and writes 1 GiB."""
    import glob
    import hashlib

    def db(sub):
        f = glob.glob(os.path.join(d, sub, "*_results.db"))
        if len(f) != 1:
            raise SystemExit(f"expected one rocprofv3 database under {os.path.join(d, sub)}, found {len(f)}")
        return f[0]

    copy_bytes = float(1 << 30)
    cf = _counters(db("copy_fetch"))["__amd_rocclr_copyBuffer"]["FETCH_SIZE"]
    cw = _counters(db("copy_write"))["__amd_rocclr_copyBuffer"]["WRITE_SIZE"]
    fetch_scale = copy_bytes / (cf * 1024.0)
    write_scale = copy_bytes / (cw * 1024.0)
    src = b"".join(open(os.path.join(ROOT, "paper_1903_11874_amd", "csrc", n), "rb").read()
                   for n in ("bsgd_kernels.hip", "bsgd_device.h", "bsgd_kernels.h", "bsgd_capi.cpp"))
    out = {"source_sha256": hashlib.sha256(src).hexdigest(), "fetch_scale": fetch_scale, "write_scale": write_scale,
           "calibration": f"plain 1 GiB device copy (__amd_rocclr_copyBuffer): FETCH_SIZE {cf:.1f} KiB, "
                          f"WRITE_SIZE {cw:.1f} KiB per dispatch",
           "workloads": {}}
    for w in TRAFFIC_WORKLOADS:
        fe, wr, sq = _counters(db(w + "_fetch")), _counters(db(w + "_write")), _counters(db(w + "_sq"))
        tt = _kernel_times(db(w + "_trace"))
        per = {}
        print(f"\n### {w}\n\n| kernel | calls | avg us | min us | max us |\n|---|---|---|---|---|")
        for k, (n, avg, mn, mx) in sorted(tt.items(), key=lambda kv: -kv[1][0] * kv[1][1]):
            print(f"| {k} | {n} | {avg:.2f} | {mn:.2f} | {mx:.2f} |")
        print("\n| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM MB (scaled) | VALU instr | SALU instr | LDS instr "
              "| waves | wait-any / wave cycles |\n|---|---|---|---|---|---|---|---|---|")
        for k in sorted(set(fe) & set(wr)):
            if not k.startswith("k_"):
                continue
            hbm = (fe[k]["FETCH_SIZE"] * fetch_scale + wr[k]["WRITE_SIZE"] * write_scale) * 1024.0
            q = sq.get(k, {})
            per[k] = {"hbm_bytes": hbm, "valu_insts": q.get("SQ_INSTS_VALU")}
            wait = q.get("SQ_WAIT_ANY", 0.0) / q["SQ_WAVE_CYCLES"] if q.get("SQ_WAVE_CYCLES") else float("nan")
            print(f"| {k} | {fe[k]['FETCH_SIZE']:.4g} | {wr[k]['WRITE_SIZE']:.4g} | {hbm / 1e6:.2f} "
                  f"| {q.get('SQ_INSTS_VALU', float('nan')):.3g} | {q.get('SQ_INSTS_SALU', float('nan')):.3g} "
                  f"| {q.get('SQ_INSTS_LDS', float('nan')):.3g} | {q.get('SQ_WAVES', float('nan')):.0f} | {wait:.2f} |")
        out["workloads"][w] = per
        ta_dir = glob.glob(os.path.join(d, w + "_ta", "*_results.db"))
        if ta_dir:
            ta = _counters(ta_dir[0])
            print("\n| kernel | TA busy per CU (us) | TD busy per CU (us) | L2 hit rate |\n|---|---|---|---|")
            for k in sorted(ta):
                if not k.startswith("k_"):
                    continue
                q = ta[k]
                hits, miss = q.get("TCC_HIT_sum", 0.0), q.get("TCC_MISS_sum", 0.0)
                rate = hits / (hits + miss) if hits + miss > 0 else float("nan")
                print(f"| {k} | {q.get('TA_TA_BUSY_sum', float('nan')) / SIMDS * 4 / CLOCK_HZ * 1e6:.1f} "
                      f"| {q.get('TD_TD_BUSY_sum', float('nan')) / SIMDS * 4 / CLOCK_HZ * 1e6:.1f} | {100 * rate:.1f}% |")
    path = os.path.join(ROOT, "profiles", "traffic.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(f"\nwrote {path}")


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
    prof = profiled(workload_name, dominant)
    updates_per_launch = sum(u for u, _, _ in per_it_p) / n_it
    valu = None
    if prof and prof.get("valu_insts"):
        v = prof["valu_insts"]
        issue_s = v * 4 / SIMDS / CLOCK_HZ
        valu = {"insts_per_dispatch": v, "lane_slots_per_update": v * 64 / updates_per_launch,
                "issue_us": issue_s * 1e6, "issue_frac": issue_s / (avg_ms[dominant] * 1e-3),
                "achieved_lane_ops_per_s": v * 64 / (avg_ms[dominant] * 1e-3), "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK,
                "source": "rocprofv3 SQ_INSTS_VALU (wave64 instructions per dispatch), profiles/traffic.json"}
    roofline = {"bound": "hbm", "kernel": dominant, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": prof.get("hbm_bytes") if prof else None,
                "traffic_unit": "bytes per dispatch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms[dominant],
                "updates_per_launch": updates_per_launch, "valu": valu}
    # the same figures for the other projector and, with TV, the prox (context)
    other = "back_project_step" if dominant == "forward_project" else "forward_project"
    ob = bytes_bp if other == "back_project_step" else bytes_fp
    oprof = profiled(workload_name, other)
    others = {other: {"achieved": ob / (avg_ms[other] * 1e-3) / 1e9, "frac": ob / (avg_ms[other] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                      "alg_bytes_per_launch": ob, "avg_launch_ms": avg_ms[other],
                      "traffic": oprof.get("hbm_bytes") if oprof else None,
                      "valu_lane_slots_per_update": (oprof["valu_insts"] * 64 / updates_per_launch
                                                     if oprof and oprof.get("valu_insts") else None)}}
    if times["tv_prox"][1]:
        K = solver.options.tv_inner_iters
        xt = 0 if geom.fp_staged else 8  # the copy of x stored y fastest, kept for the global walk
        tb = n_vox * (12 + 40 * K + 20 + xt)
        others["tv_prox"] = {"achieved": tb / (avg_ms["tv_prox"] * 1e-3) / 1e9,
                             "frac": tb / (avg_ms["tv_prox"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                             "alg_bytes_per_launch": tb, "avg_launch_ms": avg_ms["tv_prox"],
                             "alg_bytes_rule": f"per voxel: 12 (p = 0) + 40 x {K} fused FGP steps (p_k, p_k-1 and b "
                                               f"read, p_k+1 written) + 20 (final step) + {xt} (copy of x stored y "
                                               "fastest, refreshed after the prox)"}
    roofline["other_kernels"] = others

    return {"elapsed": elapsed, "steps": steps, "value": value, "updates": updates, "roofline": roofline,
            "kernels_avg_ms": avg_ms, "times": times, "r0": r0, "r1": r1, "n_prof": n_prof, "t2": t2, "t3": t3}


def cone_bench(steps, warmup, n_prof):
    """The 3D cone-beam workload with TV (256^3, 360 views of 384^2)."""
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
    m.update(workload=wl.description, spec=spec, rows_per_iter=solver.rows_per_iter,
             blocks_per_iter=solver.blocks_per_iter, iters_per_step=solver.epoch_iters, nnz=geom.info["nnz"],
             groups=geom.groups())
    return m


def fan_bench(steps, warmup, n_prof, tune="auto"):
    """The 2D fan-beam BSGD-IM workload (512^2, 720 views, 768 bins, 4 sub-detectors)."""
    import torch
    from bsgd_inputs.configs import workload
    from bsgd_inputs.phantoms import phantom_for, poisson_log_noise
    from paper_1903_11874_amd import Geometry, Solver
    wl = workload("c2_fan512_im")
    spec = wl.geometry
    log("fan: geometry")
    geom = Geometry(spec)
    n_vox = spec.nx * spec.ny * spec.nz
    x_true = phantom_for(spec, wl.n_shapes, wl.phantom_seed)
    xt = torch.tensor(x_true, dtype=torch.float32, device="cuda")
    y = poisson_log_noise(geom.forward_project(xt).double().cpu().numpy(), wl.noise_level, wl.noise_seed)
    yd = torch.tensor(y, dtype=torch.float32, device="cuda")
    L = lipschitz_gpu(geom, n_vox)
    mu = wl.solver.mu_scale / (2.0 * L)
    log(f"fan: L = {L:.4e}, mu = {mu:.4e}")
    if tune == "auto":
        from paper_1903_11874_amd.tuning import autotune
        tt = autotune(geom, yd, node_count=64, mu=mu, epochs=2, seed=wl.solver.seed)
        log("fan: autotune " + ", ".join(f"{k}: {v * 1e3:.3f} ms" for k, v in sorted(tt.items(), key=lambda kv: kv[1])[:4]))
    else:
        parts = [int(t) for t in tune.split(",")]
        geom.set_tuning(fp_views_per_group=parts[0], fp_ray_split=parts[1],
                        bp_waves=parts[2] if len(parts) > 2 else None)
    x = torch.zeros(n_vox, dtype=torch.float32, device="cuda")
    solver = Solver(geom, yd, x, node_count=64, mu=mu, seed=wl.solver.seed)
    m = measure(geom, spec, solver, n_vox, warmup, steps, n_prof, wl.name)
    m.update(workload=wl.description, spec=spec, rows_per_iter=solver.rows_per_iter,
             blocks_per_iter=solver.blocks_per_iter, iters_per_step=solver.epoch_iters, nnz=geom.info["nnz"],
             fp_views_per_group=geom.fp_views_per_group, fp_ray_split=geom.fp_ray_split, bp_waves=geom.bp_waves,
             x_true=x_true,
             groups=geom.groups())
    return m


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_rate(spec, rays, threads, budget_s):
    """FP64 oracle FP + BP over `rays` (all of the volume), repeated to a time budget."""
    import numpy as np
    from oracle.cfast import Projector
    P = Projector(spec, rays=rays)
    x = np.random.Generator(np.random.PCG64(7)).uniform(size=spec.nx * spec.ny * spec.nz)
    updates, elapsed, reps = 0, 0.0, 0
    while elapsed < budget_s and reps < 100:
        t0 = time.perf_counter()
        yv = P.fp(x, threads=threads)
        P.bp(yv, threads=threads)
        elapsed += time.perf_counter() - t0
        updates += 2 * P.last_nnz
        reps += 1
    return updates / elapsed, updates, elapsed, reps, P.last_nnz


def cpu_baseline_cone(spec, groups, nnz_total, budget_s=8.0):
    """The FP64 oracle's matrix-free FP + BP on the host cores, on a bounded sample of the
    cone workload: all cores on one row block (its views x every ray x all 256 blocks),
    one core on one view; extrapolated linearly to an effective epoch (FP + BP of every
    nonzero of A once)."""
    import numpy as np
    per_view = spec.nu * spec.nv
    views = groups[0]
    rays = np.concatenate([np.arange(v * per_view, (v + 1) * per_view) for v in views])
    nproc = os.cpu_count() or 1
    threads = max(1, min(16, nproc))  # the host share of one GPU
    rate, upd, el, reps, nnz_rb = _oracle_rate(spec, rays, threads, budget_s)
    rate1, upd1, el1, reps1, nnz_v = _oracle_rate(spec, rays[:per_view], 1, budget_s)
    return {"value": rate, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"row block 0 ({len(views)} views x {per_view} rays) through all {spec.n_blocks} blocks of the "
                      f"{spec.nx}^3 volume, FP + BP, FP64 matrix-free Siddon, {reps} repetitions: {upd:.3e} updates "
                      f"in {el:.2f} s on {threads} threads",
            "nproc": nproc, "cpu_model": _cpu_model(),
            "single_core": {"value": rate1, "unit": "updates/s", "cores": 1,
                            "sample": f"one view ({per_view} rays), FP + BP, {reps1} repetitions: {upd1:.3e} updates "
                                      f"in {el1:.2f} s"},
            "extrapolation": {"nnz_A": nnz_total, "updates_per_effective_epoch": 2 * nnz_total,
                              "seconds_per_effective_epoch": 2 * nnz_total / rate,
                              "seconds_per_effective_epoch_single_core": 2 * nnz_total / rate1,
                              "rule": "linear in the updates: an effective epoch applies every nonzero of A once in "
                                      "FP and once in BP; the sample's rate is taken for all row blocks"}}


def cpu_baseline_fan(spec, budget_s=6.0):
    """The FP64 oracle's FP + BP over every ray of the fan workload, all host cores."""
    nproc = os.cpu_count() or 1
    threads = max(1, min(16, nproc))
    rate, upd, el, reps, nnz = _oracle_rate(spec, None, threads, budget_s)
    return {"value": rate, "unit": "updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} x (FP + BP over all {spec.n_views} views x {spec.nu} bins, full {spec.nx}x{spec.ny} "
                      f"image), FP64 matrix-free Siddon, {threads} threads: {upd:.3e} updates in {el:.2f} s"}


def serving_requests(n_requests, seed=4004):
    """The seeded serving mix: sides from {128..1024}, views = bins = 1.5 side, 10
    random ellipses per phantom, 1% Gaussian noise; unit-rate Poisson gaps (scaled per
    run), step length half of 1 / (2 ||A||^2) per geometry."""
    import torch
    from bsgd_inputs.configs import SERVING_SIDES, fan_request_geometry
    from bsgd_inputs.phantoms import phantom_for, add_gaussian_noise
    from paper_1903_11874_amd.serving import Request
    from paper_1903_11874_amd import Geometry
    rng = np.random.Generator(np.random.PCG64(seed))
    geoms, mus, reqs, truths = {}, {}, [], {}
    t = 0.0
    for rid in range(n_requests):
        t += rng.exponential(1.0)
        side = int(rng.choice(SERVING_SIDES))
        spec = fan_request_geometry(side)
        if spec not in geoms:
            log(f"serving: geometry side {side}")
            geoms[spec] = Geometry(spec)
            mus[spec] = 0.5 / (2.0 * lipschitz_gpu(geoms[spec], spec.nx * spec.ny, iters=15))
        x_true = phantom_for(spec, 10, 5000 + rid)
        truths[rid] = torch.tensor(x_true, dtype=torch.float32, device="cuda")
        y = add_gaussian_noise(geoms[spec].forward_project(truths[rid]).double().cpu().numpy(), 0.01, 6000 + rid)
        reqs.append(Request(rid=rid, geometry=spec, y=torch.tensor(y, dtype=torch.float32, device="cuda"),
                            arrival=t, mu=mus[spec], seed=rid, node_count=64))
    torch.cuda.synchronize()
    return reqs, truths, sorted(geoms, key=lambda g: g.nx), mus


def serving_bench(reqs, truths, specs, mus, rate, max_slots, tol, max_epochs):
    """Continuous-batching server vs the plain per-solve loop on one Poisson stream."""
    import dataclasses
    import torch
    from paper_1903_11874_amd.serving import Server, latency_stats
    run_reqs = [dataclasses.replace(r, arrival=r.arrival / rate, tol=tol, max_epochs=max_epochs, check_every=5)
                for r in reqs]
    server = Server(max_slots=max_slots)
    server.prepare(specs, node_count=64, mu_of=lambda g: mus[g])
    log(f"serving at {rate:g}/s: batched run")
    served = server.run(run_reqs)
    log(f"serving at {rate:g}/s: sequential run")
    seq = server.run_sequential(run_reqs)
    same = all(torch.equal(a.x, b.x) for a, b in zip(served, seq))
    st_b, st_s = latency_stats(served), latency_stats(seq)

    def snr(results):  # image SNR against each request's phantom, 20 log10(|x_true| / |x_true - x|)
        v = [float(20.0 * torch.log10(truths[r.rid].double().norm() / (truths[r.rid].double() - r.x.double()).norm()))
             for r in results]
        return {"mean_snr_db": float(np.mean(v)), "min_snr_db": float(np.min(v))}

    st_b.update(snr(served))
    st_s.update(snr(seq))
    return {"requests": len(run_reqs), "rate_per_s": rate, "arrival_span_s": max(r.arrival for r in run_reqs),
            "max_slots": max_slots,
            "stop_rule": f"||A^T(y-Ax)||/||A^T y|| <= {tol} checked every 5 epochs, at most {max_epochs} epochs",
            "batched": st_b, "sequential": st_s,
            "solves_per_s_ratio": st_b["solves_per_s"] / st_s["solves_per_s"],
            "identical_results": bool(same),
            "max_active": max(e[1] for e in server.log) if server.log else 0, "ticks": len(server.log),
            "enqueue_s": sum(e[2] for e in server.log), "check_wait_s": sum(e[3] for e in server.log)}


def serving_mode(reqs, specs, mus, rate, max_slots, tol, max_epochs, mode):
    """One mode of the serving mix alone (for kernel traces of each mode): the server's
    continuous batching or the plain per-solve loop, with serving_bench's settings."""
    import dataclasses
    import torch
    from paper_1903_11874_amd.serving import Server, latency_stats
    run_reqs = [dataclasses.replace(r, arrival=r.arrival / rate, tol=tol, max_epochs=max_epochs, check_every=5)
                for r in reqs]
    server = Server(max_slots=max_slots)
    server.prepare(specs, node_count=64, mu_of=lambda g: mus[g])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = server.run(run_reqs) if mode == "batched" else server.run_sequential(run_reqs)
    torch.cuda.synchronize()
    st = latency_stats(res)
    st["wall_s"] = time.perf_counter() - t0
    if mode == "sequential":
        # the loop serves one request at a time, so admission to completion is its service time
        side = {r.rid: r.geometry.nx for r in run_reqs}
        by = {}
        for r in res:
            by[side[r.rid]] = by.get(side[r.rid], 0.0) + (r.finished - r.admitted)
        st["service_s_by_side"] = {str(k): v for k, v in sorted(by.items())}
    return st


def hbm_copy_rate(reps: int = 10):
    """Achievable HBM bandwidth: bytes read plus written per second of a plain 1 GiB device
    copy (torch's copy kernel), timed with HIP events after three untimed copies."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    gbps = 2.0 * 4 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbps


def _line_of(m):
    T = m["iters_per_step"]
    return {"workload": m["workload"], "metric": "FP+BP ray-voxel updates/s", "value": m["value"],
            "unit": "updates/s", "steps": m["steps"], "ms_per_step": m["elapsed"] / m["steps"] * 1e3,
            "rows_per_iter": m["rows_per_iter"], "blocks_per_iter": m["blocks_per_iter"], "iters_per_step": T,
            "roofline": m["roofline"], "kernels_avg_ms": m["kernels_avg_ms"],
            "kernel_launches": {k: n for k, (ms, n) in m["times"].items()},
            "residual_norm": {"before": m["r0"], "after": m["r1"]}, "updates_per_step": m["updates"] / m["steps"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving", type=int, default=512,
                    help="requests of the continuous-batching serving measurement (0 = skip)")
    ap.add_argument("--serving-rates", default="20,1000",
                    help="arrival rates (requests/s) of the serving runs: the workload's, then a saturating one")
    ap.add_argument("--serving-tol", type=float, default=1e-3)
    ap.add_argument("--serving-max-epochs", type=int, default=120)
    ap.add_argument("--serving-slots", type=int, default=48)
    ap.add_argument("--fan-steps", type=int, default=20,
                    help="epochs of the 2D fan-beam measurement reported as 'secondary' (0 = skip)")
    ap.add_argument("--cone-only", action="store_true",
                    help="profiling aid: run only the cone-beam measurement and print its line")
    ap.add_argument("--fan-only", action="store_true",
                    help="profiling aid: run only the fan-beam measurement and print its line")
    ap.add_argument("--tune", default="auto",
                    help="fan-beam launch shapes: 'auto' (autotuner, before the timed region) or 'V,S[,W]' "
                         "(views per forward-projection workgroup, lanes per ray, back-projection waves)")
    ap.add_argument("--serving-only", choices=("batched", "sequential"), default=None,
                    help="profiling aid: run only one mode of the serving mix at the last of --serving-rates "
                         "and print its statistics")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain 1 GiB device copy (calibrates HBM byte counters) and exit")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="epochs of the event-timed second region (0 = same as --steps)")
    ap.add_argument("--write-traffic", metavar="DIR", default=None,
                    help="write profiles/traffic.json from the rocprofv3 databases under DIR (no GPU use)")
    args = ap.parse_args()
    if args.write_traffic:
        write_traffic(args.write_traffic)
        return
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
    n_prof = args.profile_steps if args.profile_steps > 0 else args.steps
    if args.serving_only:
        reqs, truths, specs, mus = serving_requests(args.serving)
        rate = float(args.serving_rates.split(",")[-1])
        st = serving_mode(reqs, specs, mus, rate, args.serving_slots, args.serving_tol, args.serving_max_epochs,
                          args.serving_only)
        print(json.dumps({"serving_mode": args.serving_only, "requests": len(reqs), "rate_per_s": rate, **st}),
              flush=True)
        return
    if args.fan_only:
        f = fan_bench(args.steps, args.warmup, n_prof, args.tune)
        line = _line_of(f)
        line.update(fp_views_per_group=f["fp_views_per_group"], fp_ray_split=f["fp_ray_split"], bp_waves=f["bp_waves"])
        print(json.dumps(line), flush=True)
        return
    c = cone_bench(args.steps, args.warmup, n_prof)
    if args.cone_only:
        print(json.dumps(_line_of(c)), flush=True)
        return
    T = c["iters_per_step"]
    out = {
        "metric": "FP+BP ray-voxel updates/s",
        "value": c["value"],
        "unit": "updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": c["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded random-ellipsoid phantom, 1% Gaussian noise)",
        "config": {"workload": c["workload"], "rows_per_iter": c["rows_per_iter"],
                   "blocks_per_iter": c["blocks_per_iter"], "iters_per_step": T,
                   "step": "one effective epoch (TV prox once per epoch)"},
        "roofline": c["roofline"],
        "kernels_avg_ms": c["kernels_avg_ms"],
        "kernel_launches": {k: n for k, (ms, n) in c["times"].items()},
        "kernel_timing": f"HIP events around every kernel in a second timed region of {c['n_prof']} epochs "
                         f"(eager launches): {(c['t3'] - c['t2']) / c['n_prof'] * 1e3:.4f} ms per epoch; the first "
                         "timed region replays captured HIP graphs without events",
        "residual_norm": {"before": c["r0"], "after": c["r1"]},
        "updates_per_step": c["updates"] / args.steps,
    }
    cone_spec, cone_groups, cone_nnz = c["spec"], c["groups"], c["nnz"]
    del c
    torch.cuda.empty_cache()
    # context for the HBM fractions: what a plain device copy reaches on this GPU
    copy_gbps = hbm_copy_rate()
    out["roofline"]["copy_GBps"] = copy_gbps
    out["roofline"]["copy_note"] = ("achievable HBM bandwidth: a plain 1 GiB device copy, bytes read plus written "
                                    "per second (context; peak stays the published 8 TB/s)")
    if args.fan_steps > 0:
        f = fan_bench(args.fan_steps, args.warmup, args.fan_steps, args.tune)
        out["secondary"] = _line_of(f)
        out["secondary"]["fp_views_per_group"] = f["fp_views_per_group"]
        out["secondary"]["fp_ray_split"] = f["fp_ray_split"]
        out["secondary"]["bp_waves"] = f["bp_waves"]
        fan_spec = f["spec"]
        del f
        torch.cuda.empty_cache()
        if not args.no_cpu_baseline:
            log("cpu baseline: fan")
            out["secondary"]["cpu_baseline"] = cpu_baseline_fan(fan_spec)
    if args.serving > 0:
        reqs, truths, specs, mus = serving_requests(args.serving)
        out["serving"] = [serving_bench(reqs, truths, specs, mus, float(r), args.serving_slots, args.serving_tol,
                                        args.serving_max_epochs) for r in args.serving_rates.split(",")]
        del reqs, truths
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline: cone")
        out["cpu_baseline"] = cpu_baseline_cone(cone_spec, cone_groups, cone_nnz)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
