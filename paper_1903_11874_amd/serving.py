"""Continuous-batching reconstruction server on one GPU.

Requests (a scan geometry, its measured projections y and a stopping rule) arrive
over time. A request is admitted when a slot is free and the device has room for its
state (measured free HBM minus a reserve); waiting requests are admitted in arrival
order. The admitted solves share the GPU in ticks:

* each solve gets a quota of effective epochs per tick, (largest cost / its cost) **
  quota_power (at least one, at most max_quota), so with the default power 1 a small
  reconstruction is not paced by the largest one in the mix; a quota never passes the
  solve's next stopping check. A smaller power shares the GPU more evenly: it trades a
  longer median latency for a shorter tail;
* the epochs of a tick are issued round by round, each round one batched call
  (``bsgd_step_batch``: one launch per phase for all solves of the round, replayed as a
  captured HIP graph while the set recurs), the solves in admission order;
* a solve at a stopping check gets its statistic ||A^T (y - A x)|| / ||A^T y|| enqueued
  without waiting (``bsgd_normal_residual_async``) and its image copied aside; the
  host reads the values one tick later, while the GPU runs the next tick, so it never
  waits on the device between ticks. A finished solve returns the copy taken at its
  check and frees its slot.

Because a solve's arithmetic does not depend on the batch it runs in, and the checks
fall on the same epochs as in ``bsgd_solve``, every result equals the same request
solved alone by ``bsgd_solve`` (``run_sequential``, the plain per-solve loop).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional

import numpy as np

from .bsgd import Geometry, Solver, normal_residual, normal_residual_async, solve, step_batch


@dataclass
class Request:
    rid: int
    geometry: object            # a GeometrySpec
    y: object                   # float32 device tensor [n_views * nv * nu]
    arrival: float              # seconds after the stream starts
    mu: float
    seed: int = 0
    node_count: int = 64
    tol: float = 1e-3
    max_epochs: int = 50
    check_every: int = 5


@dataclass
class Result:
    rid: int
    x: object
    epochs: int
    iterations: int
    arrival: float
    admitted: float
    finished: float
    rel_normal_residual: float

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def epoch_cost(geom: Geometry, node_count: int) -> float:
    """Relative cost of one effective epoch: forward and back projection of every
    nonzero of A once, plus the launches of its iterations."""
    info = geom.info
    blocks = min(node_count, info["n_blocks"])
    rows = max(1, node_count // blocks)
    iters = max(1, round(info["n_row_blocks"] * info["n_blocks"] / (rows * blocks)))
    return 2.0 * info["nnz"] / 4e11 + iters * 3 * 8e-6


def state_bytes(geom: Geometry, node_count: int) -> int:
    """Device bytes one solve of this geometry holds: x, z, g_hat (M c), g, the selected
    rows' residual records (four floats per ray in 2D, one in 3D), the stopping
    statistic's scratch (n_rays + c), the image copy taken at a check, schedule and work
    records of one epoch."""
    info = geom.info
    g = geom.spec
    c = info["n_voxels"]
    per_view = g.nu * g.nv
    blocks = min(node_count, info["n_blocks"])
    rows = max(1, node_count // blocks)
    maxv = info["max_group_views"] * rows
    iters = max(1, round(info["n_row_blocks"] * info["n_blocks"] / (rows * blocks)))
    rec = 4 if not g.is_3d else 1
    floats = (c + info["z_floats"] + g.n_row_blocks * c + c + rec * maxv * per_view + info["n_rays"] + c + c)
    records = max(iters, 64) * maxv * blocks * (80 + 1) + max(iters, 64) * 4 * (maxv + 2 * rows + blocks + 4)
    return int(4 * floats + records + (1 << 20))


class _Active:
    def __init__(self, req: Request, geom: Geometry, stream, admitted: float, order: int):
        import torch
        self.req = req
        self.geom = geom
        g = req.geometry
        self.x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=req.y.device)
        self.solver = Solver(geom, req.y, self.x, stream=stream, node_count=req.node_count, mu=req.mu,
                             seed=req.seed)
        self.epochs = 0
        self.admitted = admitted
        self.order = order
        self.cost = epoch_cost(geom, req.node_count)
        self.checked = None  # epochs of the check in flight

    def to_next_check(self) -> int:
        r = self.req
        nxt = min(r.max_epochs, (self.epochs // r.check_every + 1) * r.check_every)
        return max(1, nxt - self.epochs)

    def due(self) -> bool:
        return self.epochs % self.req.check_every == 0 or self.epochs >= self.req.max_epochs


class Server:
    def __init__(self, max_slots: int = 32, hbm_reserve: float = 0.1, stream=None,
                 clock: Callable[[], float] = time.perf_counter, max_quota: int = 16, allocator="torch",
                 quota_power: float = 1.0):
        import torch
        self.max_slots = max_slots
        self.hbm_reserve = hbm_reserve
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.clock = clock
        self.max_quota = max_quota
        self.quota_power = quota_power
        self.allocator = allocator
        self.geoms: Dict[object, Geometry] = {}
        self.log: List[tuple] = []

    def geometry(self, spec) -> Geometry:
        if spec not in self.geoms:
            self.geoms[spec] = Geometry(spec, stream=self.stream, allocator=self.allocator)
        return self.geoms[spec]

    def prepare(self, specs, node_count: int, mu_of: Callable[[object], float], tune: bool = True) -> Dict:
        """Create the geometries of the classes a stream will use and tune each one's
        forward-projection launch shape (the autotuner, on zero data), before serving."""
        import torch
        from .tuning import autotune
        shapes = {}
        for spec in specs:
            geom = self.geometry(spec)
            if tune:
                y0 = torch.zeros(geom.info["n_rays"], dtype=torch.float32, device="cuda")
                timings = autotune(geom, y0, node_count=node_count, mu=mu_of(spec), epochs=1, stream=self.stream)
                shapes[spec] = (min(timings, key=timings.get), min(timings.values()))
        return shapes

    def _fits(self, geom: Geometry, node_count: int) -> bool:
        import torch
        free, total = torch.cuda.mem_get_info()
        return free - state_bytes(geom, node_count) > self.hbm_reserve * total

    def run(self, requests: List[Request]) -> List[Result]:
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        active: List[_Active] = []
        results: List[Result] = []
        retired: List[tuple] = []        # (event, active) closed once the event has passed
        inflight: Optional[tuple] = None  # (event, pinned values, [(active, epochs, image copy)])
        counter = 0
        t0 = self.clock()
        while pending or active or inflight:
            now = self.clock() - t0
            while pending and pending[0].arrival <= now and len(active) < self.max_slots:
                geom = self.geometry(pending[0].geometry)
                if active and not self._fits(geom, pending[0].node_count):
                    break
                req = pending.pop(0)
                active.append(_Active(req, geom, self.stream, self.clock() - t0, counter))
                counter += 1
            t_tick = self.clock()
            # quotas: the largest epoch cost of the mix gets one epoch per tick; none for a
            # solve whose check in flight is its last
            stepping = [a for a in active if not (a.checked is not None and a.epochs >= a.req.max_epochs)]
            if stepping:
                cmax = max(a.cost for a in stepping)
                quota = {id(a): min(self.max_quota, max(1, int((cmax / a.cost) ** self.quota_power)),
                                    a.to_next_check())
                         for a in stepping}
                for e in range(max(quota.values())):
                    groups: Dict[tuple, List[_Active]] = {}
                    for a in stepping:
                        if quota[id(a)] > e:
                            groups.setdefault((a.solver.epoch_iters, a.req.geometry.is_3d), []).append(a)
                    for (T, _), grp in groups.items():
                        step_batch([a.solver for a in grp], T, stream=self.stream)
                        for a in grp:
                            a.epochs += 1
            t_enq = self.clock()
            # the previous tick's checks (queued ahead of this tick's epochs)
            finished = set()
            if inflight is not None:
                ev, vals, copies = inflight
                ev.synchronize()
                num, ref = vals[0::2].numpy(), vals[1::2].numpy()
                for (a, ep, xc), nn, rr in zip(copies, num, ref):
                    a.checked = None
                    ratio = math.sqrt(nn) / max(math.sqrt(rr), 1e-300)
                    if ratio <= a.req.tol or ep >= a.req.max_epochs:
                        results.append(Result(a.req.rid, xc, ep, ep * a.solver.epoch_iters, a.req.arrival,
                                              a.admitted, self.clock() - t0, ratio))
                        finished.add(id(a))
                inflight = None
            t_wait = self.clock()
            if finished:
                marker = torch.cuda.Event()
                marker.record(self.stream)
                retired += [(marker, a) for a in active if id(a) in finished]
                active = [a for a in active if id(a) not in finished]
            # this tick's checks: statistic enqueued without waiting, image copied aside
            checks = [a for a in active if a.due() and a.checked is None]
            if checks:
                vals = torch.zeros(2 * len(checks), dtype=torch.float64, pin_memory=True)
                normal_residual_async([a.solver for a in checks], vals, stream=self.stream)
                with torch.cuda.stream(self.stream):
                    copies = [(a, a.epochs, a.x.clone()) for a in checks]
                for a in checks:
                    a.checked = a.epochs
                ev = torch.cuda.Event()
                ev.record(self.stream)
                inflight = (ev, vals, copies)
            # close retired solves whose last launches have completed
            keep = []
            for ev_r, a in retired:
                if ev_r.query():
                    a.solver.close()
                else:
                    keep.append((ev_r, a))
            retired = keep
            # (tick end, active solves, seconds enqueueing, seconds waiting on the previous checks)
            self.log.append((self.clock() - t0, len(active), t_enq - t_tick, t_wait - t_enq))
            if not active and inflight is None and pending:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.005))
        self.stream.synchronize()
        for _, a in retired:
            a.solver.close()
        return sorted(results, key=lambda r: r.rid)

    def run_sequential(self, requests: List[Request]) -> List[Result]:
        """Baseline: the plain per-solve loop, bsgd_solve for one request at a time in
        arrival order with the same stopping rule. The final statistic of each result
        is recomputed after the timed loop (bsgd_solve does not return it)."""
        import torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        epoch_iters: Dict[object, int] = {}
        for req in pending:
            if req.geometry not in epoch_iters:
                geom = self.geometry(req.geometry)
                g = req.geometry
                probe = Solver(geom, req.y, torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32,
                                                       device=req.y.device),
                               stream=self.stream, node_count=req.node_count, mu=req.mu)
                epoch_iters[req.geometry] = probe.epoch_iters
                probe.close()
        self.stream.synchronize()
        raw = []
        t0 = self.clock()
        for req in pending:
            wait = req.arrival - (self.clock() - t0)
            if wait > 0:
                time.sleep(wait)
            geom = self.geometry(req.geometry)
            g = req.geometry
            admitted = self.clock() - t0
            x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=req.y.device)
            iters, _ = solve(geom, req.y, x, stream=self.stream, node_count=req.node_count, mu=req.mu,
                             seed=req.seed, tol=req.tol, max_effective_epochs=req.max_epochs,
                             check_every=req.check_every)
            raw.append((req, x, iters, admitted, self.clock() - t0))
        results = []
        for req, x, iters, admitted, finished in raw:
            s = Solver(self.geometry(req.geometry), req.y, x, stream=self.stream, node_count=req.node_count,
                       mu=req.mu)
            ratio = float(normal_residual([s], True, self.stream)[0])
            s.close()
            results.append(Result(req.rid, x, iters // epoch_iters[req.geometry], iters, req.arrival, admitted,
                                  finished, ratio))
        return sorted(results, key=lambda r: r.rid)


def latency_stats(results: List[Result]) -> dict:
    lat = np.array([r.latency for r in results])
    span = max(r.finished for r in results) - min(r.arrival for r in results)
    return {"solves": len(results), "solves_per_s": len(results) / span if span > 0 else float("inf"),
            "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_epochs": float(np.mean([r.epochs for r in results])),
            "max_rel_normal_residual": float(max(r.rel_normal_residual for r in results))}
