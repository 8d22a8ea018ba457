"""Continuous-batching reconstruction server on one GPU.

Requests (a scan geometry, its measured projections y and a stopping rule) arrive
over time. A request is admitted when a slot is free and the device has room for
its state (measured free HBM minus a reserve). Every tick advances all admitted
solves by one effective epoch with one launch per phase (``bsgd_step_batch``), so
small and large reconstructions share the GPU. A solve stops when its relative
normal-equation residual ||A^T (y - A x)|| / ||A^T y|| falls to the requested
tolerance (checked every ``check_every`` epochs, the rule of ``bsgd_solve``) or at
its epoch cap; the checks of a tick are computed for all due solves with one
synchronisation (``bsgd_normal_residual``). Finished solves free their slot at once
and waiting requests are admitted in arrival order.

Because a solve's arithmetic does not depend on the batch it runs in, the result of
every request equals the same request solved alone by ``bsgd_solve``
(``run_sequential``, the plain per-solve loop).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from .bsgd import Geometry, Solver, normal_residual, solve, step_batch


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


class _Active:
    def __init__(self, req: Request, geom: Geometry, stream, admitted: float):
        import torch
        self.req = req
        self.geom = geom
        g = req.geometry
        self.x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=req.y.device)
        self.solver = Solver(geom, req.y, self.x, stream=stream, node_count=req.node_count, mu=req.mu,
                             seed=req.seed)
        self.epochs = 0
        self.admitted = admitted
        self.ratio = math.inf

    def due(self) -> bool:
        return self.epochs % self.req.check_every == 0 or self.epochs >= self.req.max_epochs

    def done(self) -> bool:
        return self.ratio <= self.req.tol or self.epochs >= self.req.max_epochs


def state_bytes(geom: Geometry, node_count: int) -> int:
    """Device bytes one solve of this geometry holds (x, z, g_hat, g, the residual of
    the selected rows, schedule and work records), used for admission."""
    info = geom.info
    g = geom.spec
    c = info["n_voxels"]
    per_view = g.nu * g.nv
    blocks = min(node_count, info["n_blocks"])
    rows = max(1, node_count // blocks)
    maxv = info["max_group_views"] * rows
    records = 2 * info["n_row_blocks"] * maxv * blocks * 96
    return int(4 * (c + info["z_floats"] + g.n_row_blocks * c + c + maxv * per_view) + records + (4 << 20))


class Server:
    def __init__(self, max_slots: int = 32, hbm_reserve: float = 0.1, stream=None,
                 clock: Callable[[], float] = time.perf_counter):
        import torch
        self.max_slots = max_slots
        self.hbm_reserve = hbm_reserve
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.clock = clock
        self.geoms: Dict[object, Geometry] = {}
        self.log: List[tuple] = []

    def geometry(self, spec) -> Geometry:
        if spec not in self.geoms:
            self.geoms[spec] = Geometry(spec, stream=self.stream)
        return self.geoms[spec]

    def _fits(self, geom: Geometry, node_count: int) -> bool:
        import torch
        free, total = torch.cuda.mem_get_info()
        return free - state_bytes(geom, node_count) > self.hbm_reserve * total

    def run(self, requests: List[Request]) -> List[Result]:
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        active: List[_Active] = []
        results: List[Result] = []
        t0 = self.clock()
        while pending or active:
            now = self.clock() - t0
            while (pending and pending[0].arrival <= now and len(active) < self.max_slots):
                geom = self.geometry(pending[0].geometry)
                if active and not self._fits(geom, pending[0].node_count):
                    break
                req = pending.pop(0)
                active.append(_Active(req, geom, self.stream, self.clock() - t0))
            if not active:
                wait = pending[0].arrival - (self.clock() - t0)
                if wait > 0:
                    time.sleep(min(wait, 0.01))
                continue
            # one tick: one effective epoch of every active solve, grouped by epoch
            # length and dimension, one launch per phase per group
            groups: Dict[tuple, List[_Active]] = {}
            for a in active:
                key = (a.solver.epoch_iters, a.req.geometry.is_3d)
                groups.setdefault(key, []).append(a)
            t_tick = self.clock()
            for (T, _), grp in groups.items():
                step_batch([a.solver for a in grp], T, stream=self.stream)
                for a in grp:
                    a.epochs += 1
            t_enq = self.clock()
            due = [a for a in active if a.due()]
            if due:
                for a, r in zip(due, normal_residual([a.solver for a in due], True, self.stream)):
                    a.ratio = float(r)
            # (tick end, active solves, seconds enqueueing the epoch, seconds in the checks)
            self.log.append((self.clock() - t0, len(active), t_enq - t_tick, self.clock() - t_enq))
            still: List[_Active] = []
            for a in active:
                if a.due() and a.done():
                    results.append(Result(a.req.rid, a.x, a.epochs, a.solver.iterations, a.req.arrival,
                                          a.admitted, self.clock() - t0, a.ratio))
                    a.solver.close()
                else:
                    still.append(a)
            active = still
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
