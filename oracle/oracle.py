"""ctypes wrapper of the FP64 C oracle in ``hgs_oracle.c``.

Test infrastructure only: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  Every array handed to
the C code is widened from the stored FP32 values to FP64 here; the oracle then
computes in FP64 throughout.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hgs_oracle.c")
SRC_BUILD = os.path.join(HERE, "build_oracle.c")
LIB = os.path.join(HERE, "_build", "liboracle.so")

NPARAM = 59
NSPLAT = 20
MAX_ALT = 4
ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4

# parameter slots of the gradient array
SLOTS = dict(mean=(0, 3), scale=(3, 6), rot=(6, 10), opacity=(10, 11), sh=(11, 59))


def build() -> str:
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    tmp = LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                           "-shared", "-o", tmp, SRC, SRC_BUILD, "-lm"])
    os.replace(tmp, LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        P = ctypes.POINTER
        d, i32, i64 = ctypes.c_double, ctypes.c_int32, ctypes.c_int64
        L.or_granularity_all.argtypes = [P(_OHier), P(_OView), P(d)]
        L.or_cut.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64]
        L.or_cut.restype = i64
        L.or_project.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64, P(d)]
        L.or_render.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64, P(i64), i64, P(d), P(d), P(i32),
                                P(i32), P(d), P(d), P(i32)]
        L.or_render.restype = i64
        L.or_signature.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64]
        L.or_signature.restype = ctypes.c_uint64
        L.or_signature_pix.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64, P(i64), i64]
        L.or_signature_pix.restype = ctypes.c_uint64
        L.or_backward.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64, P(i64), i64, P(d), P(d), P(d), P(d)]
        L.or_backward_budget.argtypes = [P(_OHier), P(_OView), P(i32), P(d), i64, P(i64), i64, P(d), P(d)]
        L.or_sh_basis.argtypes = [P(d), P(d)]
        L.ob_count.argtypes = [P(_OLeaves)]
        L.ob_count.restype = i64
        L.ob_build.argtypes = [P(_OLeaves), i64, P(i32), P(i32), P(i32), P(i32), P(d), P(d), P(d), P(d), P(d),
                               P(ctypes.c_float), P(ctypes.c_float)]
        L.ob_surface.argtypes = [P(d)]
        L.ob_surface.restype = d
        L.ob_eigen.argtypes = [P(d), P(d), P(d)]
        L.ob_match.argtypes = [P(d), P(d), P(d), P(d), P(d)]
        _lib = L
    return _lib


class _OLeaves(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("pos", ctypes.POINTER(ctypes.c_double)),
                ("scale", ctypes.POINTER(ctypes.c_double)),
                ("rot", ctypes.POINTER(ctypes.c_double)),
                ("opacity", ctypes.POINTER(ctypes.c_double)),
                ("sh", ctypes.POINTER(ctypes.c_double))]


class _OHier(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64),
                ("parent", ctypes.POINTER(ctypes.c_int32)),
                ("child_begin", ctypes.POINTER(ctypes.c_int32)),
                ("child_count", ctypes.POINTER(ctypes.c_int32)),
                ("bmin", ctypes.POINTER(ctypes.c_double)),
                ("bmax", ctypes.POINTER(ctypes.c_double)),
                ("mean", ctypes.POINTER(ctypes.c_double)),
                ("scale", ctypes.POINTER(ctypes.c_double)),
                ("rot", ctypes.POINTER(ctypes.c_double)),
                ("opacity", ctypes.POINTER(ctypes.c_double)),
                ("sh", ctypes.POINTER(ctypes.c_double))]


class _OView(ctypes.Structure):
    _fields_ = [("R", ctypes.c_double * 9), ("eye", ctypes.c_double * 3),
                ("fx", ctypes.c_double), ("fy", ctypes.c_double), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("z_near", ctypes.c_double), ("tau", ctypes.c_double)]


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class Hier:
    """FP64 copy of a hierarchy (values widened from the FP32 storage)."""

    FIELDS = ("mean", "scale", "rot", "opacity", "sh")

    def __init__(self, h):
        a = h.arrays() if hasattr(h, "arrays") else dict(h)
        self.parent = np.ascontiguousarray(a["parent"], np.int32)
        self.child_begin = np.ascontiguousarray(a["child_begin"], np.int32)
        self.child_count = np.ascontiguousarray(a["child_count"], np.int32)
        self.bmin = np.ascontiguousarray(a["bmin"], np.float64)
        self.bmax = np.ascontiguousarray(a["bmax"], np.float64)
        for f in self.FIELDS:
            setattr(self, f, np.ascontiguousarray(a[f], np.float64))
        self.n = self.parent.shape[0]

    def struct(self):
        s = _OHier()
        s.n = self.n
        s.parent = _p(self.parent, ctypes.c_int32)
        s.child_begin = _p(self.child_begin, ctypes.c_int32)
        s.child_count = _p(self.child_count, ctypes.c_int32)
        s.bmin = _p(self.bmin, ctypes.c_double)
        s.bmax = _p(self.bmax, ctypes.c_double)
        for f in self.FIELDS:
            setattr(s, f, _p(getattr(self, f), ctypes.c_double))
        return s

    def copy(self):
        c = Hier.__new__(Hier)
        for k in ("parent", "child_begin", "child_count", "bmin", "bmax") + self.FIELDS:
            setattr(c, k, getattr(self, k).copy())
        c.n = self.n
        return c

    def param_flat(self, slot: int) -> np.ndarray:
        """View of gradient slot ``slot`` (0..58) in the parameter arrays."""
        if slot < 3:
            return self.mean[slot]
        if slot < 6:
            return self.scale[slot - 3]
        if slot < 10:
            return self.rot[slot - 6]
        if slot == 10:
            return self.opacity
        return self.sh[slot - 11]


def view_struct(v) -> _OView:
    s = _OView()
    R = np.asarray(v.R, np.float32).astype(np.float64).reshape(9)
    for k in range(9):
        s.R[k] = R[k]
    e = np.asarray(v.eye, np.float32).astype(np.float64)
    for k in range(3):
        s.eye[k] = e[k]
    f32 = lambda x: float(np.float32(x))  # noqa: E731  (the values the GPU sees)
    s.fx, s.fy, s.cx, s.cy = f32(v.fx), f32(v.fy), f32(v.cx), f32(v.cy)
    s.width, s.height = int(v.width), int(v.height)
    s.z_near, s.tau = f32(v.z_near), f32(v.tau)
    return s


def _H(h):
    return h if isinstance(h, Hier) else Hier(h)


def granularity(h, v) -> np.ndarray:
    H = _H(h)
    out = np.empty(H.n, np.float64)
    hs, vs = H.struct(), view_struct(v)
    lib().or_granularity_all(ctypes.byref(hs), ctypes.byref(vs), _p(out, ctypes.c_double))
    return out


def cut(h, v):
    """(ids int32 ascending, t float64) of the cut for view v."""
    H = _H(h)
    hs, vs = H.struct(), view_struct(v)
    ids = np.empty(max(H.n, 1), np.int32)
    t = np.empty(max(H.n, 1), np.float64)
    c = lib().or_cut(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32), _p(t, ctypes.c_double), H.n)
    return ids[:c].copy(), t[:c].copy()


SPLAT_COLS = ("valid", "u", "v", "depth", "ca", "cb", "cc", "kappa", "A_n", "A_p", "t", "K",
              "r", "g", "b", "x0", "x1", "y0", "y1", "depth32")


def project(h, v, ids, t) -> dict:
    H = _H(h)
    ids = np.ascontiguousarray(ids, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    out = np.zeros((ids.shape[0], NSPLAT), np.float64)
    hs, vs = H.struct(), view_struct(v)
    lib().or_project(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32), _p(t, ctypes.c_double),
                     ids.shape[0], _p(out, ctypes.c_double))
    return {k: out[:, i] for i, k in enumerate(SPLAT_COLS)}


def render(h, v, ids=None, t=None, pix=None, alternatives=True) -> dict:
    """Render view v (all pixels, or the linear pixel indices ``pix``).
    Besides the image: per pixel the number of blended splats, the results
    with one near-threshold decision inverted (``nalt``, ``alt_rgb``,
    ``alt_T``), and ``nclamp``, the number of blended splats whose unclamped
    opacity term lies within a relative 1e-4 of the 0.99 clamp (where the
    gradient has two correct values)."""
    H = _H(h)
    if ids is None:
        ids, t = cut(H, v)
    ids = np.ascontiguousarray(ids, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    if pix is None:
        pix = np.arange(v.width * v.height, dtype=np.int64)
    pix = np.ascontiguousarray(pix, np.int64)
    m = pix.shape[0]
    rgb = np.zeros((m, 3))
    T = np.zeros(m)
    nb = np.zeros(m, np.int32)
    nalt = np.zeros(m, np.int32)
    alt_rgb = np.zeros((m, MAX_ALT, 3))
    alt_T = np.zeros((m, MAX_ALT))
    nclamp = np.zeros(m, np.int32)
    hs, vs = H.struct(), view_struct(v)
    P = ctypes.POINTER
    total = lib().or_render(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32), _p(t, ctypes.c_double),
                            ids.shape[0], _p(pix, ctypes.c_int64), m, _p(rgb, ctypes.c_double),
                            _p(T, ctypes.c_double), _p(nb, ctypes.c_int32),
                            _p(nalt, ctypes.c_int32) if alternatives else P(ctypes.c_int32)(),
                            _p(alt_rgb, ctypes.c_double) if alternatives else P(ctypes.c_double)(),
                            _p(alt_T, ctypes.c_double) if alternatives else P(ctypes.c_double)(),
                            _p(nclamp, ctypes.c_int32))
    return dict(rgb=rgb, T=T, nblend=nb, nalt=nalt, alt_rgb=alt_rgb, alt_T=alt_T, nclamp=nclamp,
                blended=int(total), pix=pix, ids=ids, t=t)


def render_image(h, v, ids=None, t=None):
    r = render(h, v, ids, t, alternatives=False)
    return r["rgb"].reshape(v.height, v.width, 3), r["T"].reshape(v.height, v.width)


def signature(h, v, ids, t, pix=None) -> int:
    """Hash of the decisions (contributing sets and order, clamp states,
    colour clamps) of every pixel, or of the linear pixel indices ``pix``."""
    H = _H(h)
    hs, vs = H.struct(), view_struct(v)
    ids = np.ascontiguousarray(ids, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    if pix is None:
        return int(lib().or_signature(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32),
                                      _p(t, ctypes.c_double), ids.shape[0]))
    pix = np.ascontiguousarray(pix, np.int64)
    return int(lib().or_signature_pix(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32),
                                      _p(t, ctypes.c_double), ids.shape[0], _p(pix, ctypes.c_int64), pix.shape[0]))


def backward(h, v, ids, t, dL_drgb, pix=None) -> dict:
    """Vector-Jacobian product of the rendered image with dL_drgb[H, W, 3]
    (restricted to the linear pixel indices ``pix`` when given; the cotangent
    is zero elsewhere).  Returns grad[59, n] (no leaf masking), dt per cut
    node and the per-node screen-space adjoints [count, 11]."""
    H = _H(h)
    ids = np.ascontiguousarray(ids, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    g = np.ascontiguousarray(dL_drgb, np.float64).reshape(-1, 3)
    assert g.shape[0] == v.width * v.height
    if pix is None:
        pix = np.arange(v.width * v.height, dtype=np.int64)
    pix = np.ascontiguousarray(pix, np.int64)
    gp = np.ascontiguousarray(g[pix])
    grad = np.zeros((NPARAM, H.n))
    dt = np.zeros(ids.shape[0])
    scr = np.zeros((ids.shape[0], 11))
    hs, vs = H.struct(), view_struct(v)
    lib().or_backward(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32), _p(t, ctypes.c_double),
                      ids.shape[0], _p(pix, ctypes.c_int64), pix.shape[0], _p(gp, ctypes.c_double),
                      _p(grad, ctypes.c_double), _p(dt, ctypes.c_double), _p(scr, ctypes.c_double))
    return dict(grad=grad, dt=dt, screen=scr)


def backward_budget(h, v, ids, t, dL_drgb, pix=None) -> np.ndarray:
    """Rounding budget of the gradient of ``backward`` (same arguments):
    per parameter element [59, n], the sum over its (pixel, splat) terms of
    (contributors of the pixel + 16) times the term's magnitude with every
    factor of the chain in absolute value.  A result composited in FP32 is
    expected within a few 2^-24 of this of the exact gradient."""
    H = _H(h)
    ids = np.ascontiguousarray(ids, np.int32)
    t = np.ascontiguousarray(t, np.float64)
    g = np.ascontiguousarray(dL_drgb, np.float64).reshape(-1, 3)
    assert g.shape[0] == v.width * v.height
    if pix is None:
        pix = np.arange(v.width * v.height, dtype=np.int64)
    pix = np.ascontiguousarray(pix, np.int64)
    gp = np.ascontiguousarray(g[pix])
    out = np.zeros((NPARAM, H.n))
    hs, vs = H.struct(), view_struct(v)
    lib().or_backward_budget(ctypes.byref(hs), ctypes.byref(vs), _p(ids, ctypes.c_int32), _p(t, ctypes.c_double),
                             ids.shape[0], _p(pix, ctypes.c_int64), pix.shape[0], _p(gp, ctypes.c_double),
                             _p(out, ctypes.c_double))
    return out


def sh_basis(d) -> np.ndarray:
    d = np.ascontiguousarray(d, np.float64)
    Y = np.zeros(16)
    lib().or_sh_basis(_p(d, ctypes.c_double), _p(Y, ctypes.c_double))
    return Y


def adam_step(params: dict, grads: dict, m: dict, v: dict, interior: np.ndarray, lr, step: int,
              beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-15) -> None:
    """One optimiser step of the hierarchy optimisation (Sec. 5.1: the
    generated hierarchy is optimised with its leaves unchanged; the paper
    does not name the optimiser of this stage, and this is Adam as in 3D
    Gaussian Splatting), in FP64, in place on dicts of arrays in the
    parameter layouts (first axis = node).  ``interior``: boolean mask of the
    nodes that move.  Gradients of the interior nodes are zeroed afterwards;
    leaf rows of every array are left alone."""
    c1 = 1.0 - beta1 ** step
    c2 = 1.0 - beta2 ** step
    for name in params:
        g = np.asarray(grads[name], np.float64)[interior]
        mm = beta1 * np.asarray(m[name], np.float64)[interior] + (1.0 - beta1) * g
        vv = beta2 * np.asarray(v[name], np.float64)[interior] + (1.0 - beta2) * g * g
        rate = lr[name] if isinstance(lr, dict) else lr
        m[name][interior] = mm
        v[name][interior] = vv
        params[name][interior] = np.asarray(params[name], np.float64)[interior] - \
            rate * (mm / c1) / (np.sqrt(vv / c2) + eps)
        grads[name][interior] = 0.0


def compact_keep(h, views, tau_min: float = 3.0, tau_max: float | None = None) -> np.ndarray:
    """Keep flags of the hierarchy compaction, Sec. 5.2 "Compacting the
    Hierarchy", taken step by step: the leaves start out marked; for tau =
    tau_min, 2 tau_min, ... while tau <= tau_max (default: half the largest
    image side), the union of the views' cuts (Sec. 4.2) is formed, its
    bottom-most nodes (those with no descendant in the union) are found, every
    node between one of them and the already marked nodes below it is
    removed, and they are marked.  The taus are the FP32 arguments widened to
    FP64, doubled exactly."""
    H = _H(h)
    n = H.n
    parent = np.asarray(h.parent, np.int64)
    cb = np.asarray(h.child_begin, np.int64)
    cc = np.asarray(h.child_count, np.int64)
    views = list(views)
    if tau_max is None:
        tau_max = 0.5 * max(max(v.width, v.height) for v in views)
    marked = cc == 0
    removed = np.zeros(n, bool)
    tau = float(np.float32(tau_min))
    top = float(np.float32(tau_max))
    while tau <= top:
        union = np.zeros(n, bool)
        for v in views:
            ids, _ = cut(H, v.replace(tau=tau))
            union[ids] = True
        # nodes with a descendant in the union: every proper ancestor of a
        # union node (a walk stops where an earlier one already passed)
        has_desc = np.zeros(n, bool)
        for m in np.nonzero(union)[0]:
            p = parent[m]
            while p >= 0 and not has_desc[p]:
                has_desc[p] = True
                p = parent[p]
        bottom = union & ~has_desc
        for b in np.nonzero(bottom)[0]:
            stack = list(range(cb[b], cb[b] + cc[b]))
            while stack:
                c = stack.pop()
                if marked[c]:
                    continue
                removed[c] = True
                stack.extend(range(cb[c], cb[c] + cc[c]))
        assert not (removed & bottom).any()
        marked |= bottom
        tau *= 2.0
    return ~removed


# ---------------------------------------------------------------------------
# hierarchy generation (Sec. 4.1; orientation matching of Sec. 4.2)
# ---------------------------------------------------------------------------
def build_hierarchy(leaves: dict) -> dict:
    """The hierarchy over the leaves, by the plain FP64 definition in
    ``build_oracle.c``.  ``leaves``: FP32 arrays pos [n, 3], scale [n, 3],
    rot [n, 4] (w, x, y, z), opacity [n], sh [n, 48] (widened here).
    Returns component-major arrays in the storage layout of a hierarchy
    (parent, child_begin, child_count, leaf_src int32 [N]; mean, scale [3, N],
    rot [4, N], opacity [N], sh [48, N] as FP32 rounded to the nearest;
    bmin, bmax [3, N] FP32 rounded outward) and the FP64 values before that
    rounding under ``*64`` keys."""
    n = int(np.asarray(leaves["pos"]).shape[0])
    cm = {k: np.ascontiguousarray(np.asarray(leaves[k], np.float32).astype(np.float64).reshape(n, -1).T)
          for k in ("pos", "scale", "rot", "sh")}
    op = np.ascontiguousarray(np.asarray(leaves["opacity"], np.float32).astype(np.float64))
    s = _OLeaves()
    s.n = n
    for k in ("pos", "scale", "rot", "sh"):
        setattr(s, k, _p(cm[k], ctypes.c_double))
    s.opacity = _p(op, ctypes.c_double)
    L = lib()
    N = int(L.ob_count(ctypes.byref(s)))
    out = dict(parent=np.zeros(N, np.int32), child_begin=np.zeros(N, np.int32), child_count=np.zeros(N, np.int32),
               leaf_src=np.zeros(N, np.int32))
    f64 = dict(mean=np.zeros((3, N)), scale=np.zeros((3, N)), rot=np.zeros((4, N)), opacity=np.zeros(N),
               sh=np.zeros((48, N)))
    bmin = np.zeros((3, N), np.float32)
    bmax = np.zeros((3, N), np.float32)
    L.ob_build(ctypes.byref(s), N, _p(out["parent"], ctypes.c_int32), _p(out["child_begin"], ctypes.c_int32),
               _p(out["child_count"], ctypes.c_int32), _p(out["leaf_src"], ctypes.c_int32),
               _p(f64["mean"], ctypes.c_double), _p(f64["scale"], ctypes.c_double), _p(f64["rot"], ctypes.c_double),
               _p(f64["opacity"], ctypes.c_double), _p(f64["sh"], ctypes.c_double), _p(bmin, ctypes.c_float),
               _p(bmax, ctypes.c_float))
    for k, a in f64.items():
        out[k] = a.astype(np.float32)
        out[k + "64"] = a
    out["bmin"], out["bmax"] = bmin, bmax
    return out


def ellipsoid_surface(s) -> float:
    s = np.ascontiguousarray(s, np.float64)
    return float(lib().ob_surface(_p(s, ctypes.c_double)))


def eigen_sym3(A):
    A = np.ascontiguousarray(A, np.float64).reshape(9)
    lam, V = np.zeros(3), np.zeros(9)
    lib().ob_eigen(_p(A, ctypes.c_double), _p(lam, ctypes.c_double), _p(V, ctypes.c_double))
    return lam, V.reshape(3, 3)


def match_axes(Rp, V, s):
    """The oracle's orientation matching of one node: axes V (columns) with
    scales s against the parent frame Rp; returns (R, s')."""
    Rp = np.ascontiguousarray(Rp, np.float64).reshape(9)
    V = np.ascontiguousarray(V, np.float64).reshape(9)
    s = np.ascontiguousarray(s, np.float64)
    R, so = np.zeros(9), np.zeros(3)
    lib().ob_match(_p(Rp, ctypes.c_double), _p(V, ctypes.c_double), _p(s, ctypes.c_double), _p(R, ctypes.c_double),
                   _p(so, ctypes.c_double))
    return R.reshape(3, 3), so
