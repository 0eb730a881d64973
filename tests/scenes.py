"""Small hand-built hierarchies for closed-form and invariant tests.

Input construction only (no cut, projection or compositing arithmetic)."""
from __future__ import annotations

import numpy as np

from paper_2406_12080_amd.synth import Hierarchy, View, quat_to_mat


def hierarchy(parent, mean, scale, rot, opacity, sh) -> Hierarchy:
    """Build a Hierarchy from per-node arrays in BFS order (parent[0] = -1,
    parent index < child index, siblings contiguous).  Boxes: leaf = mean +-
    3 sqrt(diag Sigma) rounded outward to FP32; interior = union of its
    children's boxes."""
    parent = np.asarray(parent, np.int32)
    N = parent.shape[0]
    child_count = np.bincount(parent[1:], minlength=N).astype(np.int32)
    child_begin = np.zeros(N, np.int32)
    for i in range(N - 1, 0, -1):
        child_begin[parent[i]] = i
    mean = np.asarray(mean, np.float32).reshape(N, 3)
    scale = np.asarray(scale, np.float32).reshape(N, 3)
    rot = np.asarray(rot, np.float64).reshape(N, 4)
    rot = (rot / np.linalg.norm(rot, axis=1, keepdims=True)).astype(np.float32)
    Rm = quat_to_mat(rot.astype(np.float64))
    cov = np.einsum("nij,nj,nkj->nik", Rm, scale.astype(np.float64) ** 2, Rm)
    ext = 3.0 * np.sqrt(np.einsum("nii->ni", cov))
    bmin = (mean.astype(np.float64) - ext)
    bmax = (mean.astype(np.float64) + ext)
    bmin32 = bmin.astype(np.float32)
    bmin32[bmin32.astype(np.float64) > bmin] = np.nextafter(bmin32[bmin32.astype(np.float64) > bmin], -np.inf)
    bmax32 = bmax.astype(np.float32)
    bmax32[bmax32.astype(np.float64) < bmax] = np.nextafter(bmax32[bmax32.astype(np.float64) < bmax], np.inf)
    for i in range(N - 1, -1, -1):
        if child_count[i] > 0:
            c = slice(child_begin[i], child_begin[i] + child_count[i])
            bmin32[i] = bmin32[c].min(0)
            bmax32[i] = bmax32[c].max(0)
    return Hierarchy(parent=parent, child_begin=child_begin, child_count=child_count,
                     bmin=np.ascontiguousarray(bmin32.T), bmax=np.ascontiguousarray(bmax32.T),
                     mean=np.ascontiguousarray(mean.T), scale=np.ascontiguousarray(scale.T),
                     rot=np.ascontiguousarray(rot.T), opacity=np.asarray(opacity, np.float32).reshape(N),
                     sh=np.ascontiguousarray(np.asarray(sh, np.float32).reshape(N, 48).T))


def axis_view(width, height, f, tau=1.0, eye=(0.0, 0.0, 0.0)) -> View:
    """Camera at ``eye`` whose right/down/forward axes are world x/y/z."""
    return View(R=np.eye(3, dtype=np.float32), eye=np.asarray(eye, np.float32), fx=float(f), fy=float(f),
                cx=width / 2.0, cy=height / 2.0, width=width, height=height, z_near=0.2, tau=float(tau))


def random_params(rng, N, center, spread, log_scale=-2.0):
    mean = np.asarray(center, np.float64) + spread * rng.normal(size=(N, 3))
    scale = np.exp(rng.normal(log_scale, 0.3, (N, 3)))
    rot = rng.normal(size=(N, 4))
    op = rng.uniform(0.2, 0.9, N)
    sh = rng.normal(0.0, 0.3, (N, 48))
    return mean, scale, rot, op, sh
