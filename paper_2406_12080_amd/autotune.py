"""Autotuner of the blend stage: picks the (tile edge, splats staged per
batch) with the fastest step for a given batch of views.  Every candidate
gives bit-identical images, so the choice only moves time."""
from __future__ import annotations

import time

# tile_w, tile_h, batch: every combination the library supports
CANDIDATES = ((8, 8, 64), (8, 8, 128), (16, 8, 128), (16, 8, 256), (16, 16, 256), (16, 16, 512), (32, 16, 512))


def autotune(r, views, step=None, reps: int = 1, candidates=CANDIDATES, log=None) -> dict:
    """Time `step` (default: a batched render of `views` on renderer `r`)
    once to warm up and `reps` times per candidate, keep the fastest as the
    renderer's tuning and return it."""
    import torch
    if step is None:
        def step():
            r.render(views)
    best = None
    for tw, th, b in candidates:
        r.set_tuning(tw, th, b)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        if log:
            log(f"autotune tile {tw}x{th} batch {b}: {dt * 1e3:.2f} ms")
        if best is None or dt < best[0]:
            best = (dt, tw, th, b)
    r.set_tuning(best[1], best[2], best[3])
    return dict(tile_w=best[1], tile_h=best[2], batch=best[3])
