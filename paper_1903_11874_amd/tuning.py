"""Launch-shape autotuner: times one effective epoch of a throwaway solver for each
candidate forward-projection workgroup shape (views per workgroup) and keeps the
fastest on the geometry. The shape never changes results, only speed."""
from __future__ import annotations

import time
from typing import Dict, Sequence

from .bsgd import Geometry, Solver

CANDIDATES = (1, 2, 3, 4, 6, 8, 12)


def autotune(geom: Geometry, y, node_count: int, mu: float, candidates: Sequence[int] = CANDIDATES,
             epochs: int = 2, seed: int = 0, stream=None) -> Dict[int, float]:
    """Return {views per workgroup: seconds per epoch}; the best is set on geom."""
    import torch
    g = geom.spec
    timings: Dict[int, float] = {}
    for c in candidates:
        geom.fp_views_per_group = c
        x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=y.device)
        s = Solver(geom, y, x, stream=stream, node_count=node_count, mu=mu, seed=seed, eager=True)
        T = s.epoch_iters
        s.step(T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(T * epochs)
        torch.cuda.synchronize()
        timings[c] = (time.perf_counter() - t0) / epochs
        s.close()
    geom.fp_views_per_group = min(timings, key=timings.get)
    return timings
