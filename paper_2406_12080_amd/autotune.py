"""Autotuner of the blend stage: picks the (tile edge, splats staged per
batch, work distribution) with the fastest step for a given batch of views.
Every candidate gives bit-identical images, so the choice only moves time."""
from __future__ import annotations

import time

# tile_w, tile_h, batch: every combination the library supports
SHAPES = ((8, 8, 64), (8, 8, 128), (16, 8, 128), (16, 8, 256), (16, 16, 256), (16, 16, 512), (32, 16, 512))
# each with one workgroup per tile (0) and with a persistent grid over a
# device-side tile queue (1)
CANDIDATES = tuple((tw, th, b, p) for tw, th, b in SHAPES for p in (0, 1))


def autotune(r, views, step=None, reps: int = 1, candidates=CANDIDATES, log=None) -> dict:
    """Time `step` (default: a batched render of `views` on renderer `r`)
    once to warm up and `reps` times per candidate, keep the fastest as the
    renderer's tuning and return it."""
    import torch
    if step is None:
        def step():
            r.render(views)
    best = None
    times = {}
    for tw, th, b, p in candidates:
        r.set_tuning(tw, th, b, p)
        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        times[f"{tw}x{th}x{b}{'p' if p else ''}"] = round(dt * 1e3, 3)
        if log:
            log(f"autotune tile {tw}x{th} batch {b} {'persistent' if p else 'grid'}: {dt * 1e3:.2f} ms")
        if best is None or dt < best[0]:
            best = (dt, tw, th, b, p)
    r.set_tuning(best[1], best[2], best[3], best[4])
    return dict(tile_w=best[1], tile_h=best[2], batch=best[3], persistent=best[4], ms=times)


def autotune_step(r, views, params, seed: int = 1234, reps: int = 1, log=None) -> dict:
    """Tune on the differentiable step: one batched render of `views` and one
    backward with a seeded N(0, 1) cotangent into zeroed gradient buffers
    shaped like `params` (the dict of bound parameter tensors).  This is the
    choice the benchmark times."""
    import torch
    dev = params["mean"].device
    gen = torch.Generator(device=dev).manual_seed(seed)
    dL = [torch.randn((v.height, v.width, 3), device=dev, generator=gen) for v in views]
    imgs = [torch.empty((v.height, v.width, 3), device=dev) for v in views]
    grads = {k: torch.zeros_like(t) for k, t in params.items()}

    def step():
        r.render(views, out=imgs)
        r.backward(dL, grads)

    step()  # sizes the workspaces
    torch.cuda.synchronize()
    return autotune(r, views, step, reps, log=log)
