#!/usr/bin/env python3
"""Throughput of the hierarchical-Gaussian cut + splatting path on one MI355X.

One step = the whole path for one batch of views: the per-view cut and
interpolation weights, preprocess (interpolation, EWA projection, SH
colour), visibility compaction and depth sort, pair duplication, (tile,
depth) sort, tile ranges, alpha blending, and the backward (blend backward
plus preprocess backward to every interior node's parameters).  The batch
is rendered in one call (one graph launch); the same views rendered one call
per view are reported as the plain comparison.

Prints one JSON line (see the "metric" field); progress goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "views/s and Gaussian-pixel blends/s at 1080p tau=6px, batched vs plain; fwd+bwd"

WORKLOADS = {
    # 30M leaves along a 3 km corridor, 32 views of 1920x1080 at tau = 6 px
    "corridor30m_32x1080p_tau6": dict(config=5, headline=True),
    # 8M leaves along a 1 km corridor, 64 views of 1920x1080 at tau = 6 px
    "corridor8m_64x1080p_tau6": dict(config=3, headline=True),
    # 1M leaves in a 100x100x20 m box with a dense core, one 1920x1080 view at tau = 6 px
    "box1m_1x1080p_tau6": dict(config=2, tau=6.0),
    # 2M leaves, 8 views of 1280x720 at tau = 6 px
    "box2m_8x720p_tau6": dict(config=4),
}
DEFAULT = "corridor30m_32x1080p_tau6"

# Algorithmic FP32 work of the blend kernels, in the units of the scope
# table's measurement row: per evaluated (pixel, splat) pair about 16
# lane-operations (the quadratic form, the two clamps and compares, the
# colour and transmittance FMAs) plus one transcendental (exp2), and 4 more
# (log2, exp2, two FMAs) when the splat is interpolated (t > 0); the
# backward about three times the forward's work per contributing pair.
F_PAIR, F_PAIR_T = 17, 4
BWD_FACTOR = 3
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector peak (256 CU, 2.4 GHz, packed)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # without packed FP32 (one FMA per lane and clock)
PEAK_HBM_GBS = 8000.0

def log(*a):
    print(*a, file=sys.stderr, flush=True)


def build_workload(name: str, leaves: int | None = None):
    from paper_2406_12080_amd import synth
    w = WORKLOADS[name]
    cfg = w["config"]
    t0 = time.time()
    h = synth.make_scene(cfg, n_leaves=leaves, progress=lambda m: log(f"[bench] scene: {m} ({time.time() - t0:.1f}s)"))
    if cfg in (3, 5):
        views = synth.make_views(cfg, headline=True)
    else:
        views = synth.make_views(cfg, tau=w.get("tau"))
    log(f"[bench] scene {name}: {h.info} views={len(views)} ({time.time() - t0:.1f}s)")
    return h, views


def autotune(r, views, P):
    """The package's autotuner on the fwd+bwd step (images are bit-identical
    across choices)."""
    from paper_2406_12080_amd.autotune import autotune_step
    return autotune_step(r, views, P, log=lambda m: log(f"[bench] {m}"))


def cpu_baseline(h, view, row_stride: int = 1):
    """The FP64 oracle on the host cores for one view of the batch: its cut,
    then forward compositing and backward over every `row_stride`-th pixel
    row (1: the whole image, the default).  With a stride above 1 the time of
    the sampled rows is scaled to the full image (an upper estimate: the
    oracle's per-view set-up is scaled with it)."""
    import numpy as np
    from oracle import oracle as O
    t0 = time.perf_counter()
    H = O.Hier(h)
    t_prep = time.perf_counter() - t0
    t0 = time.perf_counter()
    ids, t = O.cut(H, view)
    t_cut = time.perf_counter() - t0
    rows = np.arange(0, view.height, row_stride)
    pix = (rows[:, None] * view.width + np.arange(view.width)[None, :]).reshape(-1)
    frac = pix.size / float(view.width * view.height)
    t0 = time.perf_counter()
    o = O.render(H, view, ids, t, pix=pix if row_stride > 1 else None, alternatives=False)
    t_render = time.perf_counter() - t0
    blends = int(o["nblend"].sum())
    del o
    rng = np.random.default_rng(0)
    dL = np.zeros((view.height * view.width, 3))
    dL[pix] = rng.normal(size=(pix.size, 3))
    t0 = time.perf_counter()
    O.backward(H, view, ids, t, dL, pix=pix if row_stride > 1 else None)
    t_bwd = time.perf_counter() - t0
    t_view = t_cut + (t_render + t_bwd) / frac
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    what = ("the whole image" if row_stride == 1 else
            f"every {row_stride}th pixel row ({frac:.4f} of the pixels), scaled to the full image")
    return dict(value=1.0 / t_view, unit="views/s", cores=cores, kind="oracle",
                sample=(f"1 view of the batch ({view.width}x{view.height}, tau={view.tau:g}): cut ({len(ids)} nodes, "
                        f"{t_cut:.2f}s), forward ({t_render:.2f}s) and backward ({t_bwd:.2f}s) over {what}; FP64 "
                        f"widening of the hierarchy ({t_prep:.1f}s) not counted"),
                seconds=dict(cut=t_cut, render=t_render, backward=t_bwd, full_view_estimate=t_view),
                blends_per_s_forward=blends / t_render, cpu_model=cpu_model()), H


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


# Learning rates per parameter group for the timed optimisation steps (the
# magnitudes 3D Gaussian Splatting uses; the timing does not depend on them).
ADAM_LR = dict(mean=1.6e-4, scale=5e-3, rot=1e-3, opacity=5e-2, sh=2.5e-3)


def optimize_steps(r, h, P, grads, imgs, dL, workload: str, steps: int) -> dict:
    """Time `steps` steps of the hierarchy optimisation: per step a new batch
    of eyes with tau log-uniform over the workload's range (config 5: 32
    views of 1920x1080, tau in [3, 15] px), render, and the backward with a
    fixed synthetic cotangent with the Adam step on the interior nodes fused
    into its gradient gather (hgs_backward_adam_step).  The same steps with
    the backward into gradient arrays followed by the separate Adam step are
    timed beside it.  Cameras are drawn before the timed region."""
    import torch
    from paper_2406_12080_amd import synth
    cfg = WORKLOADS[workload]["config"]
    if cfg not in (3, 5):
        raise SystemExit("--optimize needs a corridor workload (configs 3 and 5)")
    warm = 2
    batches = [synth.make_views(cfg, seed=1000 * cfg + s) for s in range(warm + steps)]
    same = all((v.width, v.height) == (o.shape[1], o.shape[0]) for v, o in zip(batches[0], imgs))
    out = imgs if same else [torch.empty((v.height, v.width, 3), device=imgs[0].device) for v in batches[0]]
    cot = dL if same else [torch.randn(o.shape, device=o.device) for o in out]
    M, V = r.adam_moments(P)  # one row per interior node
    for g in grads.values():
        g.zero_()
    n_step = 0

    def one(views, fused=True):
        nonlocal n_step
        n_step += 1
        r.render(views, out=out)
        if fused:
            r.backward_adam_step(cot, P, M, V, ADAM_LR, n_step)
        else:
            r.backward(cot, grads)
            r.adam_step(P, grads, M, V, ADAM_LR, n_step)

    def timed(fused, n):
        for s in range(warm):
            one(batches[s], fused)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(warm, warm + n):
            one(batches[s], fused)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n

    dt = timed(True, steps)
    n_sep = min(steps, 20)
    dt_sep = timed(False, n_sep)
    taus = [v.tau for b in batches[warm:] for v in b]
    nv = len(batches[0])
    log(f"[bench] optimisation: {steps} steps, {dt * 1e3:.2f} ms/step (backward and Adam separate: "
        f"{dt_sep * 1e3:.2f} ms/step over {n_sep} steps)")
    # the Adam step alone (HBM-bound): per interior node and parameter the
    # parameter, gradient and both moments are read and written once
    n_adam = 10
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for s in range(n_adam):
        r.adam_step(P, grads, M, V, ADAM_LR, n_step + 1 + s)
    ev[1].record()
    torch.cuda.synchronize()
    ms_adam = ev[0].elapsed_time(ev[1]) / n_adam
    per_node = sum(t.numel() for t in P.values()) // h.n_nodes
    adam_bytes = (h.n_nodes - h.n_leaves) * per_node * 4 * 8
    gbs = adam_bytes / (ms_adam * 1e-3) / 1e9
    log(f"[bench] Adam step alone: {ms_adam:.3f} ms, {gbs:.0f} GB/s")
    return dict(steps=steps, warmup=warm, ms_per_step=round(dt * 1e3, 3), views_per_s=round(nv / dt, 3),
                views_per_step=nv, tau_min=round(min(taus), 3), tau_max=round(max(taus), 3),
                step="new eyes and tau per step; render + backward with Adam on the interior nodes fused into "
                     "the gradient gather",
                ms_per_step_separate=round(dt_sep * 1e3, 3),
                adam=dict(ms=round(ms_adam, 4), bytes=int(adam_bytes), gb_per_s=round(gbs, 1),
                          frac_hbm=round(gbs / 8000.0, 4), launches_per_step=len(P),
                          bytes_per_node=per_node * 32))


# FP64 operations of one granularity evaluation (per interior node and view,
# compares counted like arithmetic): per axis the extent, its running
# maximum, the two-sided clamp of the eye to the box, the difference and its
# square (6 x 3), the sum of squares (2), sqrt, f L and the division (3), and
# the running maximum over the views (1)
F_GRAN = 24


def compaction(r, h, workload: str, n_views: int) -> dict:
    """Time the GPU marking of the hierarchy compaction (Sec. 5.2) for
    `n_views` training views of the workload (eyes drawn as for its batches),
    tau from 3 px doubling up to half the image's larger side."""
    from paper_2406_12080_amd import synth
    cfg = WORKLOADS[workload]["config"]
    views = []
    s = 0
    while len(views) < n_views:
        views += synth.make_views(cfg, seed=50000 + s, headline=True)
        s += 1
    views = views[:n_views]
    tau_max = 0.5 * max(max(v.width, v.height) for v in views)
    keep = r.compact_mark(views, 3.0, tau_max)  # warm-up (allocates its buffer)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        keep = r.compact_mark(views, 3.0, tau_max)  # synchronises
    dt = (time.perf_counter() - t0) / reps
    kept = int(keep.sum().item())
    levels = 0
    t = 3.0
    while t <= tau_max:
        levels += 1
        t *= 2.0
    evals = (h.n_nodes - h.n_leaves) * n_views
    tflops = evals * F_GRAN / dt / 1e12
    log(f"[bench] compaction marking: {n_views} views, {dt * 1e3:.2f} ms, kept {kept} of {h.n_nodes}")
    return dict(views=n_views, tau_min=3.0, tau_max=tau_max, levels=levels, ms=round(dt * 1e3, 3),
                nodes=h.n_nodes, kept=kept, node_view_evals_per_s=round(evals / dt, 1),
                roofline=dict(bound="alu", achieved=round(tflops, 3), peak=78.6, unit="TFLOP/s (FP64)",
                              frac=round(tflops / 78.6, 4), flops_per_eval=F_GRAN))


# scale and opacity are stored activated (metres, |o|), so their steps are
# smaller than the 3DGS rates for the pre-activation values
CONVERGE_LR = dict(mean=1e-3, scale=5e-4, rot=1e-3, opacity=5e-3, sh=2.5e-3)


def converge(r, h, views, steps: int) -> dict:
    """Convergence of the hierarchy optimisation (Sec. 5.1) on the
    workload's views, posed as the differentiation workload is: the targets
    are the images of the hierarchy as generated; the interior nodes' means,
    log-scales and SH coefficients are then perturbed by N(0, 0.05), and
    `steps` steps of render, L1 loss, backward and Adam on the interior nodes
    (leaves frozen) pull the images back.  Returns the loss along the way.
    Binds a fresh copy of the hierarchy's parameters."""
    import torch
    from paper_2406_12080_amd import hgs
    P = hgs.params_to_device(h)
    r.bind(*[P[k] for k in hgs.PARAM_FIELDS])
    dev = P["mean"].device
    imgs, _ = r.render(views)
    tgt = [o.clone() for o in imgs]
    interior = torch.from_numpy(h.child_count > 0).to(dev)
    gen = torch.Generator(device="cpu").manual_seed(4)

    def noise(t):
        return torch.randn(t.shape, generator=gen).to(dev) * 0.05

    with torch.no_grad():
        P["mean"] += noise(P["mean"]) * interior[:, None]
        P["scale"] *= torch.exp(noise(P["scale"]) * interior[:, None])
        P["sh"] += noise(P["sh"]) * interior[:, None]
    M, V = r.adam_moments(P)
    n_val = sum(t.numel() for t in tgt)
    losses = []
    t0 = time.perf_counter()
    for s in range(steps + 1):
        imgs, _ = r.render(views, out=imgs)
        with torch.no_grad():
            diffs = [i - t for i, t in zip(imgs, tgt)]
            losses.append(sum(float(d.abs().sum()) for d in diffs) / n_val)
            dL = [torch.sign(d) / n_val for d in diffs]
        if s == steps:
            break
        r.backward_adam_step(dL, P, M, V, CONVERGE_LR, s + 1)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(steps, 1)
    marks = sorted({0, steps} | {steps * k // 10 for k in range(1, 10)})
    log(f"[bench] convergence: L1 {losses[0]:.6f} -> {losses[-1]:.6f} in {steps} steps ({dt * 1e3:.2f} ms/step)")
    return dict(steps=steps, ms_per_step=round(dt * 1e3, 3), lr=CONVERGE_LR, perturbation=0.05,
                l1_unperturbed=0.0, l1={str(k): round(losses[k], 7) for k in marks},
                reduction=round(losses[-1] / max(losses[0], 1e-30), 4))


def kernel_source_sha() -> str:
    p = os.path.join(ROOT, "paper_2406_12080_amd", "csrc", "k_blend.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 --pmc
    summary, if it was taken on the current kernel source."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("source_sha") != kernel_source_sha():
        return None
    return d.get("bytes_per_launch")


def _omp_threads(n: int) -> None:
    """Sets the OpenMP thread count of this (host) thread's later parallel
    regions, such as the oracle's."""
    import ctypes
    try:
        ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))
    except OSError:
        pass


def cpu_one_core(H, view, row_stride: int) -> dict:
    """The oracle on one host core (the OpenMP regions of this thread set to
    one thread): the cut and the forward and backward of every
    `row_stride`-th pixel row of one view, scaled to the whole view, with
    its blended-pair count (blends/s of the forward).  H: the oracle's FP64
    copy of the hierarchy."""
    import numpy as np
    from oracle import oracle as O
    v = view
    _omp_threads(1)
    try:
        t0 = time.perf_counter()
        ids, t = O.cut(H, v)
        t_cut = time.perf_counter() - t0
        rows = np.arange(0, v.height, row_stride)
        pix = (rows[:, None] * v.width + np.arange(v.width)[None, :]).reshape(-1)
        frac = pix.size / float(v.width * v.height)
        t0 = time.perf_counter()
        o = O.render(H, v, ids, t, pix=pix, alternatives=False)
        t_render = time.perf_counter() - t0
        blends = int(o["nblend"].sum())
        dL = np.zeros((v.height * v.width, 3))
        dL[pix] = np.random.default_rng(0).normal(size=(pix.size, 3))
        t0 = time.perf_counter()
        O.backward(H, v, ids, t, dL, pix=pix)
        t_bwd = time.perf_counter() - t0
    finally:
        _omp_threads(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))
    t_view = t_cut + (t_render + t_bwd) / frac
    return dict(value=1.0 / t_view, unit="views/s", cores=1, kind="oracle",
                sample=(f"1 view ({v.width}x{v.height}, tau={v.tau:g}): cut ({len(ids)} nodes) and forward + "
                        f"backward over every {row_stride}th pixel row ({frac:.4f} of the pixels), scaled to the "
                        f"whole view"),
                blends_per_s_forward=blends / t_render,
                seconds=dict(cut=t_cut, render=t_render, backward=t_bwd, full_view_estimate=t_view))


def forward_leg(name: str, steps: int, taus=(6.0,), plain: bool = True) -> dict:
    """Forward throughput of another workload: its scene and views, the
    autotuned forward, batched (one call for every view) and, with `plain`,
    one call per view; per tau when several are given (single-view
    workloads: plain only)."""
    import torch
    from paper_2406_12080_amd import hgs
    from paper_2406_12080_amd.autotune import autotune
    h, views = build_workload(name)
    r = hgs.Renderer(0)
    r.upload(h)
    P = hgs.params_to_device(h)
    r.bind(*[P[k] for k in hgs.PARAM_FIELDS])
    out = dict(workload=name, leaves=h.n_leaves, nodes=h.n_nodes, views=len(views), per_tau={})
    for tau in taus:
        vs = [v.replace(tau=tau) for v in views]
        imgs = [torch.empty((v.height, v.width, 3), device="cuda") for v in vs]
        r.render(vs, out=imgs)
        tuning = autotune(r, vs, step=lambda: r.render(vs, out=imgs), log=lambda m: log(f"[bench] {name} {m}"))
        res = dict(tuning={k: tuning[k] for k in ("tile_w", "tile_h", "batch", "persistent")})
        r.render(vs, out=imgs)
        torch.cuda.synchronize()
        if len(vs) > 1:
            t0 = time.perf_counter()
            for _ in range(steps):
                _, st = r.render(vs, out=imgs)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            res.update(ms_batched=round(dt * 1e3, 3), views_per_s_batched=round(len(vs) / dt, 3),
                       blends_per_s_batched=round(st["blended"] / dt, 1), blended=st["blended"], cut=st["cut"],
                       pairs=st["pairs"])
        if plain:
            for k, v in enumerate(vs):
                r.render([v], out=[imgs[k]])
            torch.cuda.synchronize()
            reps = max(1, steps // 4) if len(vs) > 1 else steps
            blended = 0
            t0 = time.perf_counter()
            for _ in range(reps):
                blended = 0
                for k, v in enumerate(vs):
                    _, st1 = r.render([v], out=[imgs[k]])
                    blended += st1["blended"]
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / reps
            res.update(ms_plain=round(dt * 1e3, 3), views_per_s_plain=round(len(vs) / dt, 3),
                       blends_per_s_plain=round(blended / dt, 1))
        log(f"[bench] {name} tau {tau:g}: {res}")
        out["per_tau"][f"{tau:g}"] = res
        del imgs
    r.close()
    del P
    torch.cuda.empty_cache()
    return out


def stream_leg(r, h, frames: int = 120, step_m: float = 0.5, cache_nodes: int = 8_000_000,
               cleanup_every: int = 100, max_age: int = 50) -> dict:
    """Out-of-core rendering (Sec. 6.3) along a camera path down the
    corridor: one 1920x1080 view per frame at tau = 6 px, the eye moving
    `step_m` metres a frame; the parameters stay in pinned host memory and a
    device cache of `cache_nodes` records takes what each frame's cut needs
    (cleanup every `cleanup_every` frames of records older than `max_age`).
    Reports per frame the cut size (#Render), the records transferred
    (#Trans) and the time, against the same path rendered in core."""
    import torch
    from paper_2406_12080_amd import synth
    path = [synth.look_dir((100.0 + step_m * f, 0.0, 1.7), 0.0, 0.0, 1920, 1080, 6.0) for f in range(frames)]
    img = [torch.empty((1080, 1920, 3), device="cuda")]
    r.unbind()
    r.render([path[0]], out=img)  # in core, the same path
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cut = []
    for v in path:
        _, st = r.render([v], out=img)
        cut.append(st["cut"])
    torch.cuda.synchronize()
    t_core = (time.perf_counter() - t0) / frames
    r.stream_begin(min(cache_nodes, h.n_nodes))
    trans, ms = [], []
    try:
        for f, v in enumerate(path, start=1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r.render([v], out=img)  # synchronises at its end
            ms.append((time.perf_counter() - t0) * 1e3)
            trans.append(r.stream_info()["requested"])
            if f % cleanup_every == 0:
                r.stream_cleanup(max_age)
        info = r.stream_info()
    finally:
        r.stream_end()
    res = dict(frames=frames, step_m=step_m, cache_nodes=min(cache_nodes, h.n_nodes), cleanup_every=cleanup_every,
               max_age=max_age, render_per_frame_mean=round(float(sum(cut)) / frames, 1),
               trans_per_frame_mean=round(float(sum(trans[1:])) / max(frames - 1, 1), 1),
               trans_first_frame=trans[0], trans_max=max(trans[1:]) if frames > 1 else trans[0],
               ms_per_frame_stream=round(sum(ms[1:]) / max(frames - 1, 1), 3), ms_first_frame=round(ms[0], 3),
               ms_per_frame_in_core=round(t_core * 1e3, 3), resident_end=info["resident"],
               transferred_total=info["transferred_total"], host_bytes_per_node=236)
    log(f"[bench] stream leg: {res}")
    return res


def build_leg(workload: str) -> dict:
    """Hierarchy generation on the GPU (hgs_build) over the workload's leaves,
    already in device memory: the octree, the merges, the orientation
    matching and the boxes.  Timed on the second of two builds."""
    import torch
    from paper_2406_12080_amd import hgs, synth
    cfg = synth.CONFIGS[WORKLOADS[workload]["config"]]
    t0 = time.time()
    lv = synth.make_leaves(cfg["leaves"], cfg["layout"], WORKLOADS[workload]["config"])
    log(f"[bench] build leg: {cfg['leaves']} leaves drawn ({time.time() - t0:.1f}s)")
    dl = {("mean" if k == "pos" else k): torch.from_numpy(v).cuda() for k, v in lv.items()}
    del lv
    r = hgs.Renderer(0)
    times = []
    for _ in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n_nodes = r.build(dl)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    r.close()
    del dl
    torch.cuda.empty_cache()
    log(f"[bench] build leg: {n_nodes} nodes in {times[-1] * 1e3:.1f} ms")
    return dict(leaves=cfg["leaves"], nodes=n_nodes, ms=round(times[-1] * 1e3, 2),
                nodes_per_s=round(n_nodes / times[-1], 1), first_ms=round(times[0] * 1e3, 2))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default=DEFAULT, choices=sorted(WORKLOADS))
    ap.add_argument("--leaves", type=int, default=None, help="override the leaf count (smaller runs)")
    ap.add_argument("--tile", default=None, help="WxHxB[p], skips the autotuner (e.g. 16x16x256, 8x8x64p)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-row-stride", type=int, default=1)
    ap.add_argument("--cpu-one-core-stride", type=int, default=24,
                    help="pixel-row stride of the one-core oracle sample (0: skip it)")
    ap.add_argument("--optimize", type=int, default=100, metavar="K",
                    help="also time K steps of the hierarchy optimisation (corridor workloads): every step new "
                         "eyes and tau log-uniform over the workload's range, render, backward and an Adam step "
                         "on the interior nodes (reported under 'optimize'; `value` stays the fwd+bwd step); "
                         "0 skips it")
    ap.add_argument("--other-workloads", type=int, default=1,
                    help="1: also the forward legs of the 1M-leaf single view (tau 3, 6, 15) and of the 8M-leaf "
                         "corridor's 64 views (batched vs plain); 0: skip them")
    ap.add_argument("--stream", type=int, default=120, metavar="F",
                    help="also render F frames of a camera path out of core (corridor workloads; 0: skip)")
    ap.add_argument("--build", type=int, default=1,
                    help="1: also time the GPU hierarchy generation over the workload's leaves (0: skip)")
    ap.add_argument("--compact", type=int, default=0, metavar="V",
                    help="also time the GPU marking of the hierarchy compaction over V training views "
                         "(reported under 'compaction')")
    ap.add_argument("--converge", type=int, default=0, metavar="K",
                    help="also K steps of the hierarchy optimisation against targets rendered before the interior "
                         "nodes are perturbed (L1 loss reported under 'convergence')")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a known-size transfer that calibrates "
                         "rocprofv3 FETCH_SIZE / WRITE_SIZE readings)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only; --gpus {args.gpus} is not supported "
              "(views would shard across GPUs with no communication in the forward and one reduction of "
              "interior-node gradients per step, which is not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_12080_amd import hgs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy of {args.copy_calibration_mib} MiB done")
        del src, dst
    t_host = time.time()
    h, views = build_workload(args.workload, args.leaves)
    host_build_s = time.time() - t_host  # the NumPy generation of the input scene, for comparison
    nv = len(views)
    dev = torch.device("cuda", 0)
    r = hgs.Renderer(0)
    t0 = time.time()
    r.upload(h)
    P = hgs.params_to_device(h, dev)
    r.bind(*[P[k] for k in hgs.PARAM_FIELDS])
    grads = {k: torch.zeros_like(P[k]) for k in hgs.PARAM_FIELDS}
    gen = torch.Generator(device=dev).manual_seed(1234)
    dL = [torch.randn((v.height, v.width, 3), device=dev, generator=gen) for v in views]
    imgs = [torch.empty((v.height, v.width, 3), device=dev) for v in views]
    log(f"[bench] upload + buffers {time.time() - t0:.1f}s")

    def step_batched():
        r.render(views, out=imgs)
        r.backward(dL, grads)

    def step_plain():
        for k, v in enumerate(views):
            r.render([v], out=[imgs[k]])
            r.backward([dL[k]], grads)

    def fwd_batched():
        r.render(views, out=imgs)

    step_batched()  # sizes the workspaces
    torch.cuda.synchronize()
    if args.tile:
        spec = args.tile.rstrip("p")
        tw, th, b = (int(x) for x in spec.split("x"))
        pers = 1 if args.tile.endswith("p") else 0
        r.set_tuning(tw, th, b, pers)
        tuning = dict(tile_w=tw, tile_h=th, batch=b, persistent=pers)
    else:
        tuning = autotune(r, views, P)
    log(f"[bench] tuning {tuning}")

    # timed region: graphs as shipped, no events inside
    r.set_profiling(False)
    for _ in range(max(args.warmup, 1)):
        step_batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step_batched()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    ctr = r.counters()
    log(f"[bench] batched fwd+bwd {t_batched * 1e3:.2f} ms/step, counters {ctr}")

    # kernel times from a separate profiled pass (events around the blend,
    # its backward and the preprocess backward; the blend then runs right
    # after the forward graph and the backward without a graph)
    r.set_profiling(True)
    n_prof = max(3, min(args.steps, 5))
    for _ in range(n_prof):
        step_batched()
    torch.cuda.synchronize()
    k_ms = {k: r.kernel_time(k) for k in (hgs.K_BLEND, hgs.K_BLEND_BWD, hgs.K_PREPROCESS_BWD)}
    r.set_profiling(False)

    # forward only, batched
    fwd_batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_batched()
    torch.cuda.synchronize()
    t_fwd = (time.perf_counter() - t0) / args.steps

    # stage times of one view rendered on its own (HIP events between stages)
    _, st1 = r.render([views[0]], out=[imgs[0]], timed=True)
    stage_names = ("cut", "preprocess", "visible_and_depth_sort", "duplicate", "tile_sort", "ranges", "blend",
                   "total")
    stages_plain = {n: round(float(x), 4) for n, x in zip(stage_names, st1["ms"])}
    log(f"[bench] stages of one view rendered alone (ms): {stages_plain}")

    t_plain = t_plain_fwd = None
    if not args.no_plain:
        step_plain()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 2))
        t0 = time.perf_counter()
        for _ in range(reps):
            step_plain()
        torch.cuda.synchronize()
        t_plain = (time.perf_counter() - t0) / reps
        log(f"[bench] plain fwd+bwd {t_plain * 1e3:.2f} ms/step")
        t0 = time.perf_counter()
        for _ in range(reps):
            for k, v in enumerate(views):
                r.render([v], out=[imgs[k]])
        torch.cuda.synchronize()
        t_plain_fwd = (time.perf_counter() - t0) / reps

    opt = None
    if args.optimize > 0 and WORKLOADS[args.workload]["config"] in (3, 5):
        opt = optimize_steps(r, h, P, grads, imgs, dL, args.workload, args.optimize)
    cmp = None
    if args.compact > 0:
        cmp = compaction(r, h, args.workload, args.compact)
    conv = None
    if args.converge > 0:
        conv = converge(r, h, views, args.converge)
    stream = None
    if args.stream > 0 and WORKLOADS[args.workload]["config"] in (3, 5):
        stream = stream_leg(r, h, frames=args.stream)

    # roofline of the dominant kernel (the longer of blend and blend backward)
    ms_blend, n_blend = k_ms[hgs.K_BLEND]
    ms_bwd, n_bwd = k_ms[hgs.K_BLEND_BWD]
    tfrac = ctr["evaluated_t"] / max(ctr["evaluated"], 1)
    per_pair = F_PAIR + F_PAIR_T * tfrac
    flops_fwd = per_pair * ctr["evaluated"]
    flops_bwd = BWD_FACTOR * per_pair * ctr["bwd_contrib"]
    if ms_bwd >= ms_blend:
        kname, avg_ms, flops = "k_blend_bwd", ms_bwd / max(n_bwd, 1), flops_bwd
    else:
        kname, avg_ms, flops = "k_blend", ms_blend / max(n_blend, 1), flops_fwd
    achieved = flops / (avg_ms * 1e-3) / 1e12
    traffic = load_traffic(args.workload, kname)
    roofline = dict(bound="alu", achieved=round(achieved, 3), peak=PEAK_FP32_TFLOPS, unit="TFLOP/s",
                    frac=round(achieved / PEAK_FP32_TFLOPS, 4),
                    frac_nonpacked=round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4), traffic=traffic, kernel=kname,
                    avg_launch_ms=round(avg_ms, 4), flops_per_launch=int(flops),
                    flops_unit=(f"{F_PAIR} + {F_PAIR_T} t-share per evaluated pair (forward); {BWD_FACTOR} x that "
                                f"per contributing pair (backward)"),
                    evaluated_per_contributing=round(ctr["bwd_evaluated"] / max(ctr["bwd_contrib"], 1), 3),
                    other_kernels_avg_ms={"k_blend": round(ms_blend / max(n_blend, 1), 4),
                                          "k_blend_bwd": round(ms_bwd / max(n_bwd, 1), 4),
                                          "k_preprocess_bwd+k_grad_gather": round(k_ms[hgs.K_PREPROCESS_BWD][0] /
                                                                    max(k_ms[hgs.K_PREPROCESS_BWD][1], 1), 4)})

    cpu = None
    if not args.no_cpu_baseline:
        log("[bench] CPU oracle baseline ...")
        cpu, H = cpu_baseline(h, views[0], args.cpu_row_stride)
        if args.cpu_one_core_stride > 0:
            cpu["one_core"] = cpu_one_core(H, views[0], args.cpu_one_core_stride)
        del H
        log(f"[bench] cpu {cpu}")

    v0 = views[0]
    out = {
        "metric": METRIC,
        "value": round(nv / t_batched, 3),
        "unit": "views/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_batched * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "leaves": h.n_leaves, "nodes": h.n_nodes, "views": nv,
                   "width": v0.width, "height": v0.height, "tau": v0.tau, "mode": "batched fwd+bwd",
                   "tuning": {k: tuning[k] for k in ("tile_w", "tile_h", "batch", "persistent")}},
        "blends_per_s": round(ctr["blended"] / t_batched, 1),
        "views_per_s_plain": round(nv / t_plain, 3) if t_plain else None,
        "views_per_s_fwd_batched": round(nv / t_fwd, 3),
        "views_per_s_fwd_plain": round(nv / t_plain_fwd, 3) if t_plain_fwd else None,
        "blends_per_s_fwd_batched": round(ctr["blended"] / t_fwd, 1),
        "ms_per_step_plain": round(t_plain * 1e3, 3) if t_plain else None,
        "stages_ms_one_view": stages_plain,
        "counters_per_step": ctr,
        "autotune_ms": tuning.get("ms"),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if opt is not None:
        out["optimize"] = opt
    if cmp is not None:
        out["compaction"] = cmp
    if conv is not None:
        out["convergence"] = conv
    if stream is not None:
        out["stream"] = stream
    r.close()
    del P, grads, imgs, dL
    torch.cuda.empty_cache()
    if args.build and args.leaves is None:
        out["build"] = build_leg(args.workload)
        out["build"]["host_numpy_s"] = round(host_build_s, 1)
    if args.other_workloads and args.leaves is None:
        legs = {}
        legs["box1m_1x1080p"] = forward_leg("box1m_1x1080p_tau6", args.steps, taus=(3.0, 6.0, 15.0))
        legs["corridor8m_64x1080p_tau6"] = forward_leg("corridor8m_64x1080p_tau6", max(args.steps // 2, 3))
        out["forward_legs"] = legs
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
