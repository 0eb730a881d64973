"""Independent NumPy brute-force renderer for tiny inputs.

A second, deliberately different implementation of the forward definition
(per-node cut predicate instead of a descent, complex-step Jacobian of the
pixel map instead of the closed-form EWA Jacobian, SH from scipy's complex
spherical harmonics, every (pixel, splat) pair evaluated).  It shares no code
with ``oracle/hgs_oracle.c`` and is used only to pin it.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sps

ALPHA_MIN = 1.0 / 255.0
T_MIN = 1e-4
ALPHA_MAX = 0.99
DILATION = 0.3


def real_sh(d: np.ndarray) -> np.ndarray:
    """Real orthonormal SH up to degree 3 at unit vectors d[M, 3] -> [M, 16],
    index l*l + l + m, from complex Y_l^m: for m > 0, sqrt(2) (-1)^m Re Y_l^m;
    for m < 0, sqrt(2) (-1)^m Im Y_l^|m|; for m = 0, Y_l^0."""
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    polar = np.arccos(np.clip(z, -1, 1))
    azim = np.arctan2(y, x)
    out = np.zeros((d.shape[0], 16))
    for l in range(4):
        for m in range(-l, l + 1):
            Y = sps.sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                val = np.sqrt(2) * (-1) ** m * Y.real
            elif m < 0:
                val = np.sqrt(2) * (-1) ** m * Y.imag
            else:
                val = Y.real
            out[:, l * l + l + m] = val
    return out


def _rot(q):
    q = q / np.linalg.norm(q)
    w, x, y, z = q
    # rotation of a vector v by q: v' = q v q*, assembled column by column
    def rotate(v):
        qv = np.array([0.0, *v])
        def mul(a, b):
            return np.array([a[0] * b[0] - a[1:] @ b[1:],
                             *(a[0] * b[1:] + b[0] * a[1:] + np.cross(a[1:], b[1:]))])
        r = mul(mul(q, qv), np.array([w, -x, -y, -z]))
        return r[1:]
    return np.stack([rotate(e) for e in np.eye(3)], 1)


def granularity(h, v) -> np.ndarray:
    bmin = h.bmin.astype(np.float64)
    bmax = h.bmax.astype(np.float64)
    e = np.asarray(v.eye, np.float32).astype(np.float64)[:, None]
    L = (bmax - bmin).max(0)
    d = np.linalg.norm(e - np.clip(e, bmin, bmax), axis=0)
    f = max(float(np.float32(v.fx)), float(np.float32(v.fy)))
    with np.errstate(divide="ignore"):
        return np.where(d > 0, f * L / np.where(d > 0, d, 1.0), np.inf)


def cut(h, v):
    eps = granularity(h, v)
    tau = float(np.float32(v.tau))
    leaf = h.child_count == 0
    F = leaf | (eps <= tau)
    par = h.parent
    root = par < 0
    Fp = np.where(root, False, F[np.maximum(par, 0)])
    ids = np.nonzero(F & (root | ~Fp))[0]
    t = np.zeros(ids.shape[0])
    for k, i in enumerate(ids):
        p = par[i]
        if p < 0:
            continue
        en, ep = eps[i], eps[p]
        if np.isinf(ep) or not ep > en:
            continue
        t[k] = min(1.0, max(0.0, (tau - en) / (ep - en)))
    return ids, t


def splats(h, v, ids, t):
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)  # noqa: E731
    R = f32(v.R).reshape(3, 3)
    eye = f32(v.eye)
    fx, fy, cx, cy = (float(np.float32(a)) for a in (v.fx, v.fy, v.cx, v.cy))
    out = []
    for i, tt in zip(ids, t):
        p = h.parent[i]
        q_ = p if p >= 0 else i
        tt = tt if p >= 0 else 0.0
        lerp = lambda a: (1 - tt) * f32(a[:, i]) + tt * f32(a[:, q_])  # noqa: E731
        mu = f32(h.mean[:, i]) + tt * (f32(h.mean[:, q_]) - f32(h.mean[:, i]))
        s = lerp(h.scale)
        q = lerp(h.rot)
        sh = lerp(h.sh).reshape(16, 3)
        Rq = _rot(q)
        Sig3 = Rq @ np.diag(s * s) @ Rq.T

        def pix_map(X):
            c = R @ (X - eye)
            return np.array([fx * c[0] / c[2] + cx, fy * c[1] / c[2] + cy])

        cpos = R @ (mu - eye)
        if not cpos[2] > float(np.float32(v.z_near)):
            continue
        # complex-step Jacobian of the world -> pixel map at mu
        J = np.zeros((2, 3))
        for k in range(3):
            X = mu.astype(complex)
            X[k] += 1e-30j
            J[:, k] = pix_map(X).imag / 1e-30
        S2 = J @ Sig3 @ J.T
        S2d = S2 + DILATION * np.eye(2)
        det, detd = np.linalg.det(S2), np.linalg.det(S2d)
        if not detd > 0:
            continue
        kappa = np.sqrt(det / detd) if det > 0 else 0.0
        Y = real_sh(((mu - eye) / np.linalg.norm(mu - eye))[None])[0]
        rgb = np.maximum(0.0, Y @ sh + 0.5)
        o_n = abs(float(h.opacity[i]))
        o_p = abs(float(h.opacity[p])) if p >= 0 else 0.0
        K = int(h.child_count[p]) if p >= 0 else 1
        out.append(dict(node=int(i), t=tt, mean2=pix_map(mu), inv=np.linalg.inv(S2d), kappa=kappa,
                        o_n=o_n, o_p=o_p, K=K, rgb=rgb, depth=np.float32(cpos[2])))
    return out


def alpha_at(s, x, y):
    dvec = np.array([x, y]) - s["mean2"]
    G = np.exp(-0.5 * dvec @ s["inv"] @ dvec)
    an = min(ALPHA_MAX, s["kappa"] * s["o_n"] * G)
    if s["t"] > 0:
        ap = min(ALPHA_MAX, s["kappa"] * s["o_p"] * G)
        return (1 - s["t"]) * an + s["t"] * (1 - (1 - ap) ** (1.0 / s["K"]))
    return an


def render(h, v, ids=None, t=None):
    if ids is None:
        ids, t = cut(h, v)
    sp = splats(h, v, ids, t)
    sp.sort(key=lambda s: (s["depth"], s["node"]))
    img = np.zeros((v.height, v.width, 3))
    Tf = np.ones((v.height, v.width))
    nb = np.zeros((v.height, v.width), np.int64)
    for py in range(v.height):
        for px in range(v.width):
            T = 1.0
            C = np.zeros(3)
            for s in sp:
                a = alpha_at(s, px + 0.5, py + 0.5)
                if a < ALPHA_MIN:
                    continue
                if T * (1 - a) < T_MIN:
                    break
                C += s["rgb"] * a * T
                T *= 1 - a
                nb[py, px] += 1
            img[py, px] = C
            Tf[py, px] = T
    return img, Tf, nb
