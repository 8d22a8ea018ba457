"""Launch-shape autotuner: times one effective epoch of a throwaway solver for each
candidate forward-projection shape (views per workgroup, lanes per 2D ray) and keeps
the fastest on the geometry. Views per workgroup never changes results; the ray
split changes them only through FP32 rounding (fixed-order partial sums)."""
from __future__ import annotations

import time
from typing import Dict, Sequence, Tuple

from .bsgd import Geometry, Solver

VIEWS = (1, 2, 3, 4, 6, 8, 12, 16)
SPLITS = (1, 2, 4)


def autotune(geom: Geometry, y, node_count: int, mu: float, views: Sequence[int] = VIEWS,
             splits: Sequence[int] = SPLITS, epochs: int = 2, seed: int = 0,
             stream=None) -> Dict[Tuple[int, int], float]:
    """Return {(views per workgroup, ray split): seconds per epoch}; the best is set on geom."""
    import torch
    g = geom.spec
    if g.is_3d:
        splits = (1,)
    timings: Dict[Tuple[int, int], float] = {}
    for c in views:
        for sp in splits:
            geom.set_tuning(fp_views_per_group=c, fp_ray_split=sp)
            x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=y.device)
            s = Solver(geom, y, x, stream=stream, node_count=node_count, mu=mu, seed=seed, eager=True)
            T = s.epoch_iters
            s.step(T)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s.step(T * epochs)
            torch.cuda.synchronize()
            timings[(c, sp)] = (time.perf_counter() - t0) / epochs
            s.close()
    best = min(timings, key=timings.get)
    geom.set_tuning(fp_views_per_group=best[0], fp_ray_split=best[1])
    return timings
