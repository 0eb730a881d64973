"""The differentiation workload's own gradient check, on the oracle: FP64
central differences on 64 parameters of the 2M-leaf scene (8 views of
1280x720, tau = 6 px), L1 loss against targets the oracle renders from the
hierarchy with interior means, log-scales and SH perturbed by N(0, 0.05).
48 parameters are drawn among those with a nonzero oracle gradient, 16
uniformly over the interior nodes the views reach (zeros included).  CPU
only.

A parameter of node i moves the splats of the cut entries of i (weight
1 - t) and of its children's entries with t > 0 (weight t), and nothing else.
Both sides take the loss over a window of at most 48 x 48 pixels per view,
centred on one of those splats and inside the union of their footprint
boxes (at theta and theta +- h), composited from the cut entries whose
footprint box meets the window: the rest of the image and the rest of the
cut do not change that loss.  The loss is the plain sum of |C - C*| over the
windows (the workload's mean differs by a constant factor).  A step that
changes a decision (the signature of contributing sets, order and clamps)
or the sign of a pixel's L1 residual is rejected and counted.
"""
from __future__ import annotations

import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_12080_amd import synth

WIN = 48


@pytest.fixture(scope="module")
def box2m():
    h = synth.make_scene(4)
    views = synth.make_views(4)
    H, Hp = O.Hier(h), O.Hier(synth.perturb_interior(h, seed=2024))
    per_view = []
    for v in views:
        ids, t = O.cut(H, v)
        pr, prp = O.project(H, v, ids, t), O.project(Hp, v, ids, t)
        per_view.append(dict(v=v, ids=ids, t=t, par=H.parent[ids], rect=_rects(pr), rect_p=_rects(prp),
                             uv=np.stack([pr["u"], pr["v"]], 1)))
    return dict(h=h, H=H, Hp=Hp, views=per_view)


def _rects(pr):
    r = np.stack([pr["x0"], pr["x1"], pr["y0"], pr["y1"]], 1).astype(np.int64)
    r[pr["valid"] == 0] = (0, -1, 0, -1)
    return r


def _meets(rects, R):
    return (rects[:, 0] <= R[1]) & (rects[:, 1] >= R[0]) & (rects[:, 2] <= R[3]) & (rects[:, 3] >= R[2]) & \
        (rects[:, 1] >= rects[:, 0])


def _mini(H, ids):
    """The nodes that cut entries `ids` read (the entries' nodes and their
    parents) as a small hierarchy, numbered in ascending order of the full
    hierarchy's ids (so ties in depth still break by node id), with the full
    hierarchy's child counts (K of each parent).  Returns (hierarchy, the
    entries' new ids, new id of every old id in a dict)."""
    par = H.parent[ids]
    keep = np.unique(np.concatenate([ids, par[par >= 0]]))
    remap = np.full(keep.max() + 1, -1, np.int64)
    remap[keep] = np.arange(keep.size)
    m = O.Hier.__new__(O.Hier)
    p = H.parent[keep]
    m.parent = np.where(p >= 0, remap[np.clip(p, 0, None)], -1).astype(np.int32)
    m.child_count = H.child_count[keep].copy()
    m.child_begin = np.zeros(keep.size, np.int32)
    m.bmin, m.bmax = H.bmin[:, keep].copy(), H.bmax[:, keep].copy()
    for fld in O.Hier.FIELDS:
        a = getattr(H, fld)
        setattr(m, fld, np.ascontiguousarray(a[..., keep]))
    m.n = keep.size
    return m, remap[ids].astype(np.int32), remap


def _entries(pv, node):
    return np.nonzero((pv["ids"] == node) | ((pv["par"] == node) & (pv["t"] > 0)))[0]


def _view_terms(f, pv, slot, node, rng):
    """(fd numerator parts, oracle gradient, rejected) of one view for the
    parameter (slot, node): L(theta + h), L(theta - h) and dL/dtheta over
    the sampled pixels; None when the parameter reaches no pixel here."""
    H, v = f["H"], pv["v"]
    E = _entries(pv, node)
    if E.size == 0:
        return None
    arr = H.param_flat(slot)
    th = arr[node]
    hstep = 1e-6 * max(1.0, abs(th))
    boxes = [pv["rect"][E]]
    for x in (th + hstep, th - hstep):
        arr[node] = x
        boxes.append(_rects(O.project(H, v, pv["ids"][E], pv["t"][E])))
    arr[node] = th
    b = np.concatenate(boxes)
    b = b[b[:, 1] >= b[:, 0]]
    if b.size == 0:
        return None
    U = (b[:, 0].min(), b[:, 1].max(), b[:, 2].min(), b[:, 3].max())
    # a window inside U centred on one of the splats' centres
    k = E[rng.integers(E.size)]
    cx, cy = int(np.clip(pv["uv"][k, 0], U[0], U[1])), int(np.clip(pv["uv"][k, 1], U[2], U[3]))
    x0 = int(np.clip(cx - WIN // 2, U[0], max(U[0], U[1] - WIN + 1)))
    y0 = int(np.clip(cy - WIN // 2, U[2], max(U[2], U[3] - WIN + 1)))
    R = (x0, min(U[1], x0 + WIN - 1), y0, min(U[3], y0 + WIN - 1))
    xs, ys = np.arange(R[0], R[1] + 1), np.arange(R[2], R[3] + 1)
    pix = (ys[:, None] * v.width + xs[None, :]).ravel()
    sub = np.nonzero(_meets(pv["rect"], R))[0]
    sub_p = np.nonzero(_meets(pv["rect_p"], R))[0]
    Mp, ids_p, _ = _mini(f["Hp"], pv["ids"][sub_p])
    tgt = O.render(Mp, v, ids_p, pv["t"][sub_p], pix=pix, alternatives=False)["rgb"]
    tgt = tgt.astype(np.float32).astype(np.float64)  # targets are stored in FP32
    M, ids, remap = _mini(H, pv["ids"][sub])
    t = pv["t"][sub]
    marr, mnode = M.param_flat(slot), int(remap[node])
    base = O.render(M, v, ids, t, pix=pix, alternatives=False)["rgb"]
    sig0 = O.signature(M, v, ids, t, pix)
    out = []
    for x in (th + hstep, th - hstep):
        marr[mnode] = x
        c = O.render(M, v, ids, t, pix=pix, alternatives=False)["rgb"]
        same = O.signature(M, v, ids, t, pix) == sig0 and np.array_equal(np.sign(c - tgt), np.sign(base - tgt))
        out.append((np.abs(c - tgt).sum(), same))
    marr[mnode] = th
    cot = np.zeros((v.height * v.width, 3))
    cot[pix] = np.sign(base - tgt)
    g = O.backward(M, v, ids, t, cot, pix=pix)["grad"][slot, mnode]
    return out[0][0], out[1][0], g, hstep, not (out[0][1] and out[1][1])


def _check(f, slot, node, rng):
    Lp = Lm = g = 0.0
    hstep, reached, rejected = None, False, False
    for pv in f["views"]:
        r = _view_terms(f, pv, slot, node, rng)
        if r is None:
            continue
        reached = True
        lp, lm, gv, hstep, rej = r
        Lp, Lm, g = Lp + lp, Lm + lm, g + gv
        rejected |= rej
    if not reached:
        return None
    return (Lp - Lm) / (2 * hstep), g, rejected


def test_central_differences_on_the_2m_leaf_scene(box2m):
    f = box2m
    h = f["h"]
    rng = np.random.default_rng(64)
    interior = np.nonzero(h.child_count > 0)[0]
    reached = np.zeros(h.n_nodes, bool)
    for pv in f["views"]:
        reached[pv["ids"][pv["rect"][:, 1] >= pv["rect"][:, 0]]] = True
        p = pv["par"][(pv["t"] > 0) & (pv["rect"][:, 1] >= pv["rect"][:, 0])]
        reached[p[p >= 0]] = True
    inner_reached = interior[reached[interior]]
    assert inner_reached.size > 10000
    nonzero, uniform, rejected, tries = [], [], 0, 0
    while len(nonzero) < 48 or len(uniform) < 16:
        tries += 1
        assert tries < 400, (len(nonzero), len(uniform), rejected)
        slot, node = int(rng.integers(O.NPARAM)), int(rng.choice(inner_reached))
        r = _check(f, slot, node, rng)
        if r is None:
            continue
        fd, g, rej = r
        if rej:
            rejected += 1
            continue
        if len(uniform) < 16:
            uniform.append((slot, node, fd, g))
        elif g != 0.0 and len(nonzero) < 48:
            nonzero.append((slot, node, fd, g))
    picks = nonzero + uniform
    scale = math.sqrt(np.mean([g * g for *_, g in picks]))
    for slot, node, fd, g in picks:
        assert abs(fd - g) <= 1e-4 * max(abs(g), 1e-3 * scale), (slot, node, fd, g)
    assert sum(abs(g) > 0 for *_, g in uniform) >= 8
    print(f"64 parameters checked ({rejected} steps rejected for a changed decision), rms gradient {scale:.3e}")
