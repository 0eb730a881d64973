"""Shared parity checks of the GPU path against the oracle (test-side only)."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O

PIX_TOL = 2e-4   # max abs per pixel channel
GRAD_REL = 1e-3  # relative L2 per parameter group


def safe_tau(h, v, rel=1e-9):
    """Nudge tau (in FP32 steps) until no interior node's granularity lies
    within a relative `rel` of it, so that the selection never hinges on the
    last bit of an FP64 evaluation.  Returns the (possibly) new view."""
    H = h if isinstance(h, O.Hier) else O.Hier(h)
    inner = H.child_count > 0
    for _ in range(64):
        eps = O.granularity(H, v)[inner]
        tau = float(np.float32(v.tau))
        if tau == 0.0 or not np.any(np.abs(eps / tau - 1.0) < rel):
            return v
        v = v.replace(tau=float(np.nextafter(np.float32(tau), np.float32(np.inf))))
    raise AssertionError("could not move tau away from every granularity")


def check_pixels(gpu_rgb, gpu_T, o, tol=PIX_TOL):
    """Two-branch acceptance: a pixel passes when it is within `tol` of the
    oracle's nominal value or of one of its single-flip alternatives (a
    decision within a relative 1e-4 of the 1/255 skip or the 1e-4 stop
    threshold, inverted).  gpu_rgb [m, 3], gpu_T [m] at o['pix']."""
    nom = np.abs(gpu_rgb - o["rgb"]).max(-1)
    nomT = np.abs(gpu_T - o["T"])
    ok = (nom <= tol) & (nomT <= tol)
    alt_used = np.zeros_like(ok)
    for k in range(O.MAX_ALT):
        has = o["nalt"] > k
        ea = np.abs(gpu_rgb - o["alt_rgb"][:, k]).max(-1)
        eT = np.abs(gpu_T - o["alt_T"][:, k])
        hit = has & (ea <= tol) & (eT <= tol) & ~ok
        alt_used |= hit
        ok |= hit
    bad = np.nonzero(~ok)[0]
    return dict(ok=bool(ok.all()), n_bad=int(bad.size), bad=bad[:10], max_nominal=float(nom.max(initial=0.0)),
                n_alt=int(alt_used.sum()), n_ambiguous=int((o["nalt"] > 0).sum()), m=int(ok.size))


def ambiguous(o):
    """Pixels where the oracle's result or gradient has more than one
    correct value: a skip or stop decision within the guard band of its
    threshold, or a blended splat whose opacity term sits on the 0.99 clamp
    (the value is continuous there, its derivative is not).  The gradient
    tests give these pixels no cotangent."""
    return (o["nalt"] > 0) | (o["nclamp"] > 0)


NEAR_DEPTH = 1.0  # metres: 5 x the near plane


def near_nodes(h, v, ids, t, depth=NEAR_DEPTH):
    """Nodes (and their parents) whose splat in this view lies closer than
    `depth`.  Their splats cover most of the image from a centre far off
    screen, and the mean and covariance parts of their geometric gradient
    cancel almost entirely: the hardest case for FP32 accumulation.  Used to
    report how many such nodes a gradient check covers."""
    pr = O.project(h, v, ids, t)
    sel = (pr["valid"] > 0) & (pr["depth"] < depth)
    n = h.n_nodes if hasattr(h, "n_nodes") else h.n
    m = np.zeros(n, bool)
    m[ids[sel]] = True
    par = np.asarray(h.parent)[ids[sel]]
    m[par[par >= 0]] = True
    return m


# Rounding of an FP32 composite, per unit of the oracle's rounding budget
# (oracle.backward_budget weighs every term by its pixel's contributor count
# + 16): the transmittance in front of a splat carries about one rounding
# per contributor from the forward product and one and a half from each
# backward division, and a term's own chain (G, alpha, the products) a
# handful; four units of 2^-24 per weight unit cover both.
BUDGET_U = 4.0 * 2.0 ** -24


def check_grads(gpu: dict, og: np.ndarray, leaf_mask, rel=GRAD_REL, budget=None):
    """Per parameter group: relative L2 error (`rel`, to be <= GRAD_REL) and
    the per-element bound over every node (`n_bad` elements violate it):
        |diff| <= GRAD_REL * max(|g|, 1e-3 rms(group)) + BUDGET_U * B,
    B = the oracle's rounding budget of the element (oracle.backward_budget,
    same layout as og), which only matters where the element is a sum of
    terms that cancel far below their own size; None: no budget term."""
    out = {}
    for name, (a, b) in O.SLOTS.items():
        ref = og[a:b].copy()
        ref[:, leaf_mask] = 0.0
        # GPU gradients are node-major ([N][k]), the oracle's component-major
        g = np.asarray(gpu[name], np.float64).reshape(-1, b - a).T
        nrm = np.linalg.norm(ref)
        err = np.linalg.norm(g - ref)
        rms = nrm / np.sqrt(ref.size)
        bound = rel * np.maximum(np.abs(ref), 1e-3 * rms) + 1e-30
        plain = np.abs(g - ref) <= bound
        if budget is not None:
            bb = BUDGET_U * budget[a:b].copy()
            bb[:, leaf_mask] = 0.0
            bound = bound + bb
        elem = np.abs(g - ref) <= bound
        ratio = np.abs(g - ref) / bound
        # n_budget: elements within the bound only thanks to the budget term
        out[name] = dict(rel=float(err / max(nrm, 1e-30)), n_bad=int((~elem).sum()), norm=float(nrm),
                         worst=float(ratio.max(initial=0.0) * rel), n_budget=int((elem & ~plain).sum()))
        if not elem.all():  # where the worst elements are: (component, column, oracle, GPU)
            top = np.argsort(ratio, axis=None)[::-1][:4]
            out[name]["at"] = [(int(c), int(j), float(ref[c, j]), float(g[c, j]))
                               for c, j in zip(*np.unravel_index(top, ratio.shape))]
    return out


def assert_grads(res, ctx=""):
    """Every group within GRAD_REL (relative L2) and every element within
    its per-element bound."""
    for name, r in res.items():
        assert r["rel"] <= GRAD_REL, (ctx, name, r)
        assert r["n_bad"] == 0, (ctx, name, r)
