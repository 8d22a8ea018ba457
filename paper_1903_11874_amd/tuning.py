"""Launch-shape autotuner: times one effective epoch of a throwaway solver for each
candidate shape and keeps the fastest on the geometry.

* Forward projector: where it stages blocks in LDS the shape is (views per workgroup,
  lanes per 2D ray); where it walks global memory (blocks too large for LDS) it is the
  number of waves per (view, block) pair.
* 2D back projector: the waves of a workgroup, each gathering a share of the views into
  the tile's voxels (searched after the forward shape is fixed).

Views per workgroup and waves per pair never change results; the ray split and the back
projector's waves change them only through FP32 rounding (fixed-order partial sums)."""
from __future__ import annotations

import time
from typing import Dict, Sequence, Tuple

from .bsgd import Geometry, Solver

VIEWS = (1, 2, 3, 4, 6, 8, 12, 16)
SPLITS = (1, 2, 4)
WAVES = (8, 16, 24, 32, 48, 64)
BP_WAVES = (2, 4, 8)


def _epoch_seconds(geom: Geometry, y, node_count: int, mu: float, epochs: int, seed: int, stream) -> float:
    import torch
    g = geom.spec
    x = torch.zeros(g.nx * g.ny * g.nz, dtype=torch.float32, device=y.device)
    s = Solver(geom, y, x, stream=stream, node_count=node_count, mu=mu, seed=seed, eager=True)
    try:
        T = s.epoch_iters
        s.step(T)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(T * epochs)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / epochs
    finally:
        s.close()


def autotune(geom: Geometry, y, node_count: int, mu: float, views: Sequence[int] = VIEWS,
             splits: Sequence[int] = SPLITS, waves: Sequence[int] = WAVES, bp_waves: Sequence[int] = BP_WAVES,
             epochs: int = 2, seed: int = 0, stream=None) -> Dict[Tuple, float]:
    """Return {shape: seconds per epoch} and set the fastest shapes on geom. Forward
    shapes are (views per workgroup, ray split) when the forward projector stages blocks
    in LDS, (waves per pair,) when it walks global memory; 2D back-projection shapes are
    ("bp_waves", waves), timed with the chosen forward shape."""
    timings: Dict[Tuple, float] = {}
    if not geom.fp_staged:
        for w in waves:
            geom.set_tuning(fp_waves_per_pair=w)
            timings[(w,)] = _epoch_seconds(geom, y, node_count, mu, epochs, seed, stream)
        best = min(timings, key=timings.get)
        geom.set_tuning(fp_waves_per_pair=best[0])
    else:
        if geom.spec.is_3d:
            splits = (1,)
        for c in views:
            for sp in splits:
                geom.set_tuning(fp_views_per_group=c, fp_ray_split=sp)
                timings[(c, sp)] = _epoch_seconds(geom, y, node_count, mu, epochs, seed, stream)
        best = min(timings, key=timings.get)
        geom.set_tuning(fp_views_per_group=best[0], fp_ray_split=best[1])
    if not geom.spec.is_3d and bp_waves:
        for w in bp_waves:
            geom.set_tuning(bp_waves=w)
            timings[("bp_waves", w)] = _epoch_seconds(geom, y, node_count, mu, epochs, seed, stream)
        best_bp = min((k for k in timings if k[0] == "bp_waves"), key=timings.get)
        geom.set_tuning(bp_waves=best_bp[1])
    return timings
