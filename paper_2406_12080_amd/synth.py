"""Seeded synthetic scenes, hierarchies and cameras.

This module only *makes inputs*.  It holds none of the hot path's arithmetic
(no granularity, no cut, no interpolation, no projection, no compositing): the
FP64 oracle under ``oracle/`` and the HIP library both consume what it writes,
and neither is imported here.

What it builds, and where the paper describes it:

* leaf Gaussians with the distributions of the synthetic street-like
  workloads (position layouts, log-normal scales, uniform rotations,
  sigmoid opacities, degree-3 SH);
* a tree over the leaves.  The paper builds a binary median-split BVH
  (Sec. 4.1, "Hierarchy Generation"); the workloads here ask for an octree
  whose cells split into their non-empty spatial octants, so that is what is
  built (Morton order, one level at a time);
* interior Gaussians merged bottom-up with the KL-minimising moment match of
  Eq. (merge) and the unnormalised weights o_i * S_i (surface of the 3D
  ellipsoid standing in for sqrt|Sigma'_i|, Sec. 4.1); SH merged with the same
  weights; the interior "falloff" sum(w'_i)/S_p stored as opacity (may be >1);
* orientation matching (Sec. 4.2, last paragraph before Fig. simple-hier):
  top-down, each child's axes are re-assigned among the 24 proper signed axis
  permutations to minimise the rotation relative to its parent, then the
  quaternion sign is fixed so that q_child . q_parent >= 0;
* per-node axis-aligned boxes: a leaf's box is mean +- 3*sqrt(diag Sigma)
  (the 3x stored-size extent of Sec. 4.1), an interior node's box is the union
  of its leaves' boxes.  Boxes are rounded outward to FP32.

Storage convention (shared by everything that reads a hierarchy): nodes in
BFS order, root = 0, parent index < child index, each node's children
contiguous; structure-of-arrays FP32 with the component index major
(``mean[3, N]``, ``scale[3, N]``, ``rot[4, N]`` as w,x,y,z, ``opacity[N]``,
``sh[48, N]`` with row ``3*k + c`` = SH coefficient k of colour channel c).
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

SH_COEFFS = 16
MORTON_BITS = 21  # per axis, 63-bit codes


# ----------------------------------------------------------------------------
# containers
# ----------------------------------------------------------------------------
@dataclass
class Hierarchy:
    parent: np.ndarray        # int32[N], root = -1
    child_begin: np.ndarray   # int32[N]
    child_count: np.ndarray   # int32[N], 0 <=> leaf
    bmin: np.ndarray          # float32[3, N]
    bmax: np.ndarray          # float32[3, N]
    mean: np.ndarray          # float32[3, N]
    scale: np.ndarray         # float32[3, N] (activated, metres)
    rot: np.ndarray           # float32[4, N] (w, x, y, z), unit
    opacity: np.ndarray       # float32[N]   (leaf: opacity, interior: falloff)
    sh: np.ndarray            # float32[48, N]
    info: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.parent.shape[0])

    @property
    def n_leaves(self) -> int:
        return int(np.count_nonzero(self.child_count == 0))

    def arrays(self):
        return dict(parent=self.parent, child_begin=self.child_begin,
                    child_count=self.child_count, bmin=self.bmin, bmax=self.bmax,
                    mean=self.mean, scale=self.scale, rot=self.rot,
                    opacity=self.opacity, sh=self.sh)

    def save(self, path: str) -> None:
        np.savez(path, **self.arrays())

    @staticmethod
    def load(path: str) -> "Hierarchy":
        z = np.load(path, allow_pickle=False)
        return Hierarchy(**{k: z[k] for k in z.files})


@dataclass
class View:
    """Pinhole camera.  ``R`` rows are the camera's right, down and forward
    axes in world coordinates (world->camera rotation); pixel (i, j) samples
    the image-plane point (i + 1/2, j + 1/2)."""
    R: np.ndarray       # float32[3, 3]
    eye: np.ndarray     # float32[3]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float
    tau: float

    def replace(self, **kw) -> "View":
        d = dict(R=self.R, eye=self.eye, fx=self.fx, fy=self.fy, cx=self.cx,
                 cy=self.cy, width=self.width, height=self.height,
                 z_near=self.z_near, tau=self.tau)
        d.update(kw)
        return View(**d)


# ----------------------------------------------------------------------------
# rotations
# ----------------------------------------------------------------------------
def quat_to_mat(q: np.ndarray) -> np.ndarray:
    """q: [M, 4] (w, x, y, z), unit -> [M, 3, 3]; columns are the axes."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3), dtype=np.float64)
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def mat_to_quat(R: np.ndarray) -> np.ndarray:
    """Shepperd's method, vectorised; [M,3,3] proper rotations -> [M,4] unit."""
    m00, m11, m22 = R[:, 0, 0], R[:, 1, 1], R[:, 2, 2]
    tr = m00 + m11 + m22
    q = np.empty((R.shape[0], 4), dtype=np.float64)
    which = np.argmax(np.stack([tr, m00, m11, m22], 1), axis=1)
    # case 0: trace largest
    s = which == 0
    r = np.sqrt(np.maximum(1.0 + tr[s], 1e-300)) * 2
    q[s, 0] = 0.25 * r
    q[s, 1] = (R[s, 2, 1] - R[s, 1, 2]) / r
    q[s, 2] = (R[s, 0, 2] - R[s, 2, 0]) / r
    q[s, 3] = (R[s, 1, 0] - R[s, 0, 1]) / r
    s = which == 1
    r = np.sqrt(np.maximum(1.0 + m00[s] - m11[s] - m22[s], 1e-300)) * 2
    q[s, 0] = (R[s, 2, 1] - R[s, 1, 2]) / r
    q[s, 1] = 0.25 * r
    q[s, 2] = (R[s, 0, 1] + R[s, 1, 0]) / r
    q[s, 3] = (R[s, 0, 2] + R[s, 2, 0]) / r
    s = which == 2
    r = np.sqrt(np.maximum(1.0 + m11[s] - m00[s] - m22[s], 1e-300)) * 2
    q[s, 0] = (R[s, 0, 2] - R[s, 2, 0]) / r
    q[s, 1] = (R[s, 0, 1] + R[s, 1, 0]) / r
    q[s, 2] = 0.25 * r
    q[s, 3] = (R[s, 1, 2] + R[s, 2, 1]) / r
    s = which == 3
    r = np.sqrt(np.maximum(1.0 + m22[s] - m00[s] - m11[s], 1e-300)) * 2
    q[s, 0] = (R[s, 1, 0] - R[s, 0, 1]) / r
    q[s, 1] = (R[s, 0, 2] + R[s, 2, 0]) / r
    q[s, 2] = (R[s, 1, 2] + R[s, 2, 1]) / r
    q[s, 3] = 0.25 * r
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


def _signed_perms() -> np.ndarray:
    """The 24 signed permutation matrices with determinant +1."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            P = np.zeros((3, 3))
            for col, row in enumerate(perm):
                P[row, col] = signs[col]
            if np.linalg.det(P) > 0:
                out.append(P)
    P = np.stack(out)
    assert P.shape[0] == 24
    return P


_PERMS = _signed_perms()


def _ellipsoid_surface(s: np.ndarray) -> np.ndarray:
    """Thomsen's approximation of the surface of an ellipsoid with semi-axes
    s[:, 0..2] (relative error below about 1.1%)."""
    p = 1.6075
    a, b, c = (s[:, 0] ** p, s[:, 1] ** p, s[:, 2] ** p)
    return 4.0 * math.pi * ((a * b + a * c + b * c) / 3.0) ** (1.0 / p)


def _cov_from(scale: np.ndarray, R: np.ndarray) -> np.ndarray:
    M = R * scale[:, None, :]
    return M @ np.swapaxes(M, 1, 2)


# ----------------------------------------------------------------------------
# leaves
# ----------------------------------------------------------------------------
_CHUNK = 1 << 20


def _workers() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _par(fn, n: int, chunk: int = _CHUNK) -> None:
    """Run fn(start, stop) over [0, n) in chunks on a thread pool (numpy
    releases the GIL inside its kernels); fn writes disjoint slices."""
    spans = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
    if len(spans) <= 1:
        for a, b in spans:
            fn(a, b)
        return
    with ThreadPoolExecutor(_workers()) as ex:
        list(ex.map(lambda ab: fn(*ab), spans))


def make_leaves(n: int, layout: str, seed: int) -> dict:
    """Leaf Gaussians (FP32), drawn in chunks of 2^20 leaves from PCG64
    streams spawned per attribute and per chunk (deterministic in seed and n)."""
    ss = np.random.SeedSequence(seed)
    s_pos, s_scale, s_rot, s_op, s_sh = ss.spawn(5)
    nch = max(1, (n + _CHUNK - 1) // _CHUNK)
    seeds = {k: v.spawn(nch) for k, v in dict(pos=s_pos, scale=s_scale, rot=s_rot, op=s_op, sh=s_sh).items()}
    pos = np.empty((n, 3), np.float32)
    scale = np.empty((n, 3), np.float32)
    rot = np.empty((n, 4), np.float32)
    op = np.empty(n, np.float32)
    sh = np.empty((n, 3 * SH_COEFFS), np.float32)
    if layout.startswith("corridor"):
        length = float(layout.split(":")[1]) if ":" in layout else 1000.0
    elif layout not in ("cube", "box_core"):
        raise ValueError(layout)
    n_core = n // 5 if layout == "box_core" else 0

    def fill(a, b):
        c = a // _CHUNK
        m = b - a
        g = lambda k: np.random.Generator(np.random.PCG64(seeds[k][c]))  # noqa: E731
        rp = g("pos")
        u = rp.random((m, 3))
        if layout == "cube":
            P = -1.0 + 2.0 * u
        elif layout == "box_core":
            core = (np.arange(a, b) >= n - n_core)[:, None]
            big = np.array([-50.0, -50.0, 0.0]) + np.array([100.0, 100.0, 20.0]) * u
            small = np.array([-10.0, -10.0, 0.0]) + np.array([20.0, 20.0, 5.0]) * u
            P = np.where(core, small, big)
        else:
            cap = 1.0 - math.exp(-20.0 / 3.0)
            P = np.stack([u[:, 0] * length, -20.0 + 40.0 * u[:, 1], -3.0 * np.log1p(-u[:, 2] * cap)], 1)
        pos[a:b] = P
        scale[a:b] = np.exp(g("scale").normal(-4.0, 0.5, (m, 3)))
        q = g("rot").normal(0.0, 1.0, (m, 4))
        rot[a:b] = q / np.linalg.norm(q, axis=1, keepdims=True)
        op[a:b] = 1.0 / (1.0 + np.exp(-g("op").normal(0.0, 1.0, m)))
        sh[a:b] = g("sh").standard_normal((m, 3 * SH_COEFFS), dtype=np.float32) * np.float32(0.3)

    _par(fill, n)
    return dict(pos=pos, scale=scale, rot=rot, opacity=op, sh=sh)


# ----------------------------------------------------------------------------
# octree topology (BFS order)
# ----------------------------------------------------------------------------
def _morton(pos: np.ndarray) -> np.ndarray:
    lo = pos.min(0)
    ext = float((pos.max(0) - lo).max()) or 1.0
    g = np.floor((pos - lo) / ext * ((1 << MORTON_BITS) - 1) + 0.5).astype(np.uint64)

    def spread(v):
        v = v & np.uint64(0x1FFFFF)
        v = (v | (v << np.uint64(32))) & np.uint64(0x1F00000000FFFF)
        v = (v | (v << np.uint64(16))) & np.uint64(0x1F0000FF0000FF)
        v = (v | (v << np.uint64(8))) & np.uint64(0x100F00F00F00F00F)
        v = (v | (v << np.uint64(4))) & np.uint64(0x10C30C30C30C30C3)
        v = (v | (v << np.uint64(2))) & np.uint64(0x1249249249249249)
        return v

    return spread(g[:, 0]) | (spread(g[:, 1]) << np.uint64(1)) | (spread(g[:, 2]) << np.uint64(2))


def build_topology(codes: np.ndarray, collapse_chains: bool = False):
    """BFS node arrays from per-level leaf ranges."""
    if collapse_chains:
        levels_lo, levels_hi = _octree_levels_collapsed(codes)
    else:
        levels_lo, levels_hi = _octree_levels_plain(codes)
    sizes = [x.shape[0] for x in levels_lo]
    first = np.concatenate([[0], np.cumsum(sizes)])
    N = int(first[-1])
    parent = np.full(N, -1, np.int32)
    child_begin = np.zeros(N, np.int32)
    child_count = np.zeros(N, np.int32)
    for L in range(len(levels_lo) - 1):
        plo, phi = levels_lo[L], levels_hi[L]
        clo = levels_lo[L + 1]
        inner = np.nonzero(phi - plo >= 2)[0]
        owner = np.searchsorted(plo[inner], clo, side="right") - 1
        pid = first[L] + inner[owner]
        parent[first[L + 1]:first[L + 2]] = pid
        cnt = np.bincount(owner, minlength=inner.shape[0])
        beg = first[L + 1] + np.concatenate([[0], np.cumsum(cnt)[:-1]])
        child_begin[first[L] + inner] = beg
        child_count[first[L] + inner] = cnt
    lo_all = np.concatenate(levels_lo)
    hi_all = np.concatenate(levels_hi)
    return parent, child_begin, child_count, lo_all, hi_all, first


def _split_starts(codes, plo, phi, d):
    """First leaf of every non-empty child cell (Morton level d) of the
    multi-leaf ranges [plo, phi); past the last Morton level, groups of at most
    8 consecutive leaves."""
    if d <= MORTON_BITS:
        shift = np.uint64(3 * (MORTON_BITS - d))
        lens = phi - plo - 1
        tot = int(lens.sum())
        if tot == 0:
            return plo.copy()
        base = np.repeat(plo + 1 - np.concatenate([[0], np.cumsum(lens)[:-1]]), lens)
        idx = np.arange(tot, dtype=np.int64) + base
        diff = (codes[idx] >> shift) != (codes[idx - 1] >> shift)
        return np.sort(np.concatenate([plo, idx[diff]]))
    st = []
    for a, b in zip(plo.tolist(), phi.tolist()):
        m = b - a
        k = min(8, m)
        st.append(a + (np.arange(k, dtype=np.int64) * m) // k)
    return np.concatenate(st)


def _octree_levels_plain(codes):
    """Octree keeping single-child chains: every Morton level of a multi-leaf
    cell is a node."""
    n = codes.shape[0]
    levels_lo = [np.array([0], np.int64)]
    levels_hi = [np.array([n], np.int64)]
    d = 0
    while True:
        lo, hi = levels_lo[-1], levels_hi[-1]
        inner = (hi - lo) >= 2
        if not inner.any():
            break
        plo, phi = lo[inner], hi[inner]
        starts = _split_starts(codes, plo, phi, d + 1)
        owner = np.searchsorted(plo, starts, side="right") - 1
        nxt = np.empty_like(starts)
        nxt[:-1] = starts[1:]
        nxt[-1] = n
        levels_lo.append(starts)
        levels_hi.append(np.minimum(nxt, phi[owner]))
        d += 1
    return levels_lo, levels_hi


def _octree_levels_collapsed(codes):
    """Octree without single-child chains: a multi-leaf cell descends Morton
    levels until its leaves fall into at least two octants; each node is thus
    split at its own depth."""
    n = codes.shape[0]
    levels_lo = [np.array([0], np.int64)]
    levels_hi = [np.array([n], np.int64)]
    levels_d = [np.array([0], np.int64)]
    while True:
        lo, hi, dd = levels_lo[-1], levels_hi[-1], levels_d[-1]
        inner = (hi - lo) >= 2
        if not inner.any():
            break
        plo, phi, pd = lo[inner], hi[inner], dd[inner].copy()
        # split depth of each parent = first level at which its first and
        # last codes differ (past MORTON_BITS: coincident grouping)
        a = codes[plo]
        b = codes[phi - 1]
        x = a ^ b
        bl = np.zeros(x.shape[0], np.int64)
        nz = x != 0
        bl[nz] = np.floor(np.log2(x[nz].astype(np.float64))).astype(np.int64) + 1
        # float log2 can be off by one near powers of two: fix exactly
        hi_bit = np.left_shift(np.uint64(1), np.maximum(bl - 1, 0).astype(np.uint64))
        too_big = nz & (hi_bit > x)
        bl[too_big] -= 1
        hi_bit = np.left_shift(np.uint64(1), bl.astype(np.uint64))
        too_small = nz & (hi_bit <= x)
        bl[too_small] += 1
        split_d = np.where(nz, MORTON_BITS - (bl - 1) // 3, MORTON_BITS + 1)
        starts_all = []
        for dval in np.unique(split_d):
            sel = split_d == dval
            starts_all.append(_split_starts(codes, plo[sel], phi[sel], int(dval)))
        starts = np.sort(np.concatenate(starts_all))
        owner = np.searchsorted(plo, starts, side="right") - 1
        nxt = np.empty_like(starts)
        nxt[:-1] = starts[1:]
        nxt[-1] = n
        levels_lo.append(starts)
        levels_hi.append(np.minimum(nxt, phi[owner]))
        levels_d.append(split_d[owner])
    return levels_lo, levels_hi


# ----------------------------------------------------------------------------
# merges, orientation matching, boxes
# ----------------------------------------------------------------------------
def _cov6(scale, R):
    """Symmetric covariance R diag(s^2) R^T as [6, M] (xx xy xz yy yz zz)."""
    s2 = scale * scale
    out = np.empty((6, scale.shape[0]))
    for k, (i, j) in enumerate(((0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2))):
        out[k] = (R[:, i, :] * R[:, j, :] * s2).sum(1)
    return out


def _full(c6):
    """[6, M] -> [M, 3, 3]."""
    M = np.empty((c6.shape[1], 3, 3))
    M[:, 0, 0], M[:, 0, 1], M[:, 0, 2] = c6[0], c6[1], c6[2]
    M[:, 1, 0], M[:, 1, 1], M[:, 1, 2] = c6[1], c6[3], c6[4]
    M[:, 2, 0], M[:, 2, 1], M[:, 2, 2] = c6[2], c6[4], c6[5]
    return M


def _perm_trace_index():
    """trace(C P) for the 24 proper signed permutations as sums of 3 signed
    entries of C: (flat index [24, 3], sign [24, 3])."""
    idx = np.zeros((24, 3), np.int64)
    sg = np.zeros((24, 3))
    for p in range(24):
        P = _PERMS[p]
        for col in range(3):
            row = int(np.nonzero(P[:, col])[0][0])
            # (C P)_{col,col} = sum_j C[col, j] P[j, col] = C[col, row] * P[row, col]
            idx[p, col] = 3 * col + row
            sg[p, col] = P[row, col]
    return idx, sg


_PT_IDX, _PT_SG = _perm_trace_index()


def build_hierarchy(leaves: dict, collapse_chains: bool = False, progress=None) -> Hierarchy:
    say = progress or (lambda msg: None)
    pos = np.asarray(leaves["pos"], np.float64)
    n = pos.shape[0]
    codes = _morton(pos)
    order = np.argsort(codes, kind="stable")
    codes = codes[order]

    parent, child_begin, child_count, lo_all, hi_all, first = build_topology(codes, collapse_chains)
    N = parent.shape[0]
    say(f"topology: {N} nodes in {len(first) - 1} levels")
    is_leaf = child_count == 0
    leaf_nodes = np.nonzero(is_leaf)[0]
    assert np.all(hi_all[leaf_nodes] - lo_all[leaf_nodes] == 1)
    src = order[lo_all[leaf_nodes]]  # original leaf index of each leaf node

    # component-major working arrays (segment sums run along contiguous rows)
    mean = np.zeros((3, N))
    cov = np.zeros((6, N))
    sh = np.zeros((3 * SH_COEFFS, N), np.float32)
    op = np.zeros(N)
    surf = np.zeros(N)
    scale = np.zeros((3, N))
    Rm = np.zeros((N, 3, 3))

    def leaf_fill(a, b):
        nd, sr = leaf_nodes[a:b], src[a:b]
        mean[:, nd] = pos[sr].T
        q = np.asarray(leaves["rot"][sr], np.float64)
        s_ = np.asarray(leaves["scale"][sr], np.float64)
        R = quat_to_mat(q)
        cov[:, nd] = _cov6(s_, R)
        sh[:, nd] = leaves["sh"][sr].T
        op[nd] = leaves["opacity"][sr]
        scale[:, nd] = s_.T
        Rm[nd] = R
        surf[nd] = _ellipsoid_surface(s_)

    _par(leaf_fill, leaf_nodes.shape[0])

    nlev = len(first) - 1
    # bottom-up merge, one level at a time (children live on the next level),
    # each level in chunks of parents whose children are contiguous
    for lv in range(nlev - 2, -1, -1):
        ids = np.arange(first[lv], first[lv + 1])
        inner = ids[child_count[ids] > 0]
        if inner.shape[0] == 0:
            continue

        def merge(a, b, inner=inner):
            nd = inner[a:b]
            cb = child_begin[nd].astype(np.int64)
            cc = child_count[nd].astype(np.int64)
            c0, c1 = int(cb[0]), int(cb[-1] + cc[-1])
            seg = cb - c0
            ch = slice(c0, c1)
            wp = op[ch] * surf[ch]                       # unnormalised weights o_i S_i
            wsum = np.add.reduceat(wp, seg)
            wn = wp / np.repeat(wsum, cc)
            mu = np.add.reduceat(wn * mean[:, ch], seg, axis=1)
            dmu = mean[:, ch] - np.repeat(mu, cc, axis=1)
            outer = np.stack([dmu[0] * dmu[0], dmu[0] * dmu[1], dmu[0] * dmu[2],
                              dmu[1] * dmu[1], dmu[1] * dmu[2], dmu[2] * dmu[2]], 0)
            cv = np.add.reduceat(wn * (cov[:, ch] + outer), seg, axis=1)
            shm = np.add.reduceat(wn.astype(np.float32) * sh[:, ch], seg, axis=1)
            lam, V = np.linalg.eigh(_full(cv))
            lam = np.maximum(lam, 1e-20)
            V[np.linalg.det(V) < 0, :, 2] *= -1.0
            s_ = np.sqrt(lam)
            sp = _ellipsoid_surface(s_)
            mean[:, nd] = mu
            cov[:, nd] = cv
            sh[:, nd] = shm
            scale[:, nd] = s_.T
            Rm[nd] = V
            surf[nd] = sp
            op[nd] = wsum / sp                           # falloff, may exceed 1

        _par(merge, inner.shape[0], chunk=1 << 18)
        say(f"merged level {lv} ({inner.shape[0]} interior nodes)")

    # top-down orientation matching
    for lv in range(1, nlev):
        lo, hi = int(first[lv]), int(first[lv + 1])

        def match(a, b, lo=lo):
            ids = np.arange(lo + a, lo + b)
            C = (np.swapaxes(Rm[parent[ids]], 1, 2) @ Rm[ids]).reshape(-1, 9)  # R_p^T R_c
            tr = (C[:, _PT_IDX] * _PT_SG).sum(2)
            P = _PERMS[np.argmax(tr, axis=1)]
            Rm[ids] = Rm[ids] @ P
            # new axis k takes the scale of old axis pi(k): s' = |P|^T s
            scale[:, ids] = np.einsum("njk,jn->kn", np.abs(P), scale[:, ids])

        _par(match, hi - lo, chunk=1 << 18)

    say("orientation matching done")
    q = np.empty((N, 4))

    def quats(a, b):
        q[a:b] = mat_to_quat(Rm[a:b])

    _par(quats, N)
    for lv in range(1, nlev):
        ids = np.arange(first[lv], first[lv + 1])
        dots = np.einsum("ni,ni->n", q[ids], q[parent[ids]])
        q[ids[dots < 0]] *= -1.0
    del Rm

    # boxes: leaf = mean +- 3 sqrt(diag cov) from the stored FP32 scale and
    # rotation, rounded outward to FP32; interior = union of its children
    bmin = np.zeros((N, 3), np.float32)
    bmax = np.zeros((N, 3), np.float32)
    scale32 = scale.astype(np.float32)   # [3, N]
    q32 = q.astype(np.float32)

    def leaf_box(a, b):
        nd = leaf_nodes[a:b]
        qq = q32[nd].astype(np.float64)
        qq /= np.linalg.norm(qq, axis=1, keepdims=True)
        R = quat_to_mat(qq)
        s32 = scale32[:, nd].T.astype(np.float64)
        ext = 3.0 * np.sqrt(np.einsum("nij,nj->ni", R ** 2, s32 ** 2))
        m = mean[:, nd].T
        bmin[nd] = _round_down32(m - ext)
        bmax[nd] = _round_up32(m + ext)

    _par(leaf_box, leaf_nodes.shape[0])
    for lv in range(nlev - 2, -1, -1):
        ids = np.arange(first[lv], first[lv + 1])
        inner = ids[child_count[ids] > 0]
        if inner.shape[0] == 0:
            continue
        cb = child_begin[inner].astype(np.int64)
        cc = child_count[inner].astype(np.int64)
        c0, c1 = int(cb[0]), int(cb[-1] + cc[-1])
        seg = cb - c0
        bmin[inner] = np.minimum.reduceat(bmin[c0:c1], seg, axis=0)
        bmax[inner] = np.maximum.reduceat(bmax[c0:c1], seg, axis=0)

    f32 = np.float32
    h = Hierarchy(parent=parent, child_begin=np.where(child_count > 0, child_begin, 0).astype(np.int32),
                  child_count=child_count,
                  bmin=np.ascontiguousarray(bmin.T),
                  bmax=np.ascontiguousarray(bmax.T),
                  mean=mean.astype(f32),
                  scale=scale32,
                  rot=np.ascontiguousarray(q32.T),
                  opacity=op.astype(f32),
                  sh=sh)
    h.info = dict(n_nodes=int(N), n_leaves=int(n), n_interior=int(N - n), levels=int(nlev),
                  single_child=int(np.count_nonzero(child_count == 1)),
                  max_children=int(child_count.max()))
    return h


def _round_down32(x):
    y = x.astype(np.float32)
    bad = y.astype(np.float64) > x
    y[bad] = np.nextafter(y[bad], np.float32(-np.inf))
    return y


def _round_up32(x):
    y = x.astype(np.float32)
    bad = y.astype(np.float64) < x
    y[bad] = np.nextafter(y[bad], np.float32(np.inf))
    return y


# ----------------------------------------------------------------------------
# cameras
# ----------------------------------------------------------------------------
def look_at(eye, target, up, width, height, tau, vfov_deg=60.0, z_near=0.2) -> View:
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    r = np.cross(f, np.asarray(up, np.float64))
    r /= np.linalg.norm(r)
    d = np.cross(f, r)
    R = np.stack([r, d, f], 0).astype(np.float32)
    foc = (height / 2.0) / math.tan(math.radians(vfov_deg) / 2.0)
    return View(R=R, eye=eye.astype(np.float32), fx=float(np.float32(foc)), fy=float(np.float32(foc)),
                cx=width / 2.0, cy=height / 2.0, width=int(width), height=int(height),
                z_near=z_near, tau=float(tau))


def look_dir(eye, yaw_deg, pitch_deg, width, height, tau, vfov_deg=60.0) -> View:
    y, p = math.radians(yaw_deg), math.radians(pitch_deg)
    fwd = np.array([math.cos(p) * math.cos(y), math.cos(p) * math.sin(y), math.sin(p)])
    return look_at(eye, np.asarray(eye, np.float64) + fwd, (0, 0, 1), width, height, tau, vfov_deg)


# ----------------------------------------------------------------------------
# the five workloads
# ----------------------------------------------------------------------------
CONFIGS = {
    1: dict(leaves=4096, layout="cube"),
    2: dict(leaves=1_000_000, layout="box_core"),
    3: dict(leaves=8_000_000, layout="corridor:1000"),
    4: dict(leaves=2_000_000, layout="box_core"),
    5: dict(leaves=30_000_000, layout="corridor:3000"),
}


def make_scene(config: int, seed: int | None = None, n_leaves: int | None = None,
               collapse_chains: bool = False, progress=None) -> Hierarchy:
    c = CONFIGS[config]
    n = n_leaves if n_leaves is not None else c["leaves"]
    seed = config if seed is None else seed
    leaves = make_leaves(n, c["layout"], seed)
    if progress:
        progress(f"{n} leaves drawn")
    return build_hierarchy(leaves, collapse_chains=collapse_chains, progress=progress)


def make_views(config: int, seed: int | None = None, headline: bool = False,
               n_views: int | None = None, tau: float | None = None,
               corridor: float | None = None) -> list[View]:
    """Cameras of each workload.  Config 3: 64 views of uneven resolution,
    tau log-uniform in [2, 15] px; config 5: 32 views of 1920x1080 (the batch
    of one optimisation step; ``seed`` draws another step's eyes), tau
    log-uniform in [3, 15] px.  ``headline`` switches configs 3 and 5 to
    every view at 1920x1080 and tau = 6 px."""
    seed = config if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, 0xCA4])))
    if config == 1:
        t = 4.0 if tau is None else tau
        return [look_at((0, 0, 3), (0, 0, 0), (0, 1, 0), 256, 256, t)]
    if config == 2:
        t = 6.0 if tau is None else tau
        return [look_at((0, -40, 1.7), (0, 0, 2.5), (0, 0, 1), 1920, 1080, t)]
    if config == 4:
        nv = 8 if n_views is None else n_views
        out = []
        for k in range(nv):
            a = 2 * math.pi * k / nv
            out.append(look_at((40 * math.cos(a), 40 * math.sin(a), 1.7), (0, 0, 2.5), (0, 0, 1),
                               1280, 720, 6.0 if tau is None else tau))
        return out
    if config in (3, 5):
        length = corridor if corridor is not None else (1000.0 if config == 3 else 3000.0)
        nv = n_views if n_views is not None else (64 if config == 3 else 32)
        res = [(640, 360), (1280, 720), (1920, 1080)]
        out = []
        for k in range(nv):
            if config == 3:
                x = length * (k + 0.5) / nv
            else:
                x = length * rng.random()
            y = -3.0 + 6.0 * rng.random()
            yaw = (0.0 if k % 2 == 0 else 180.0) + (-15.0 + 30.0 * rng.random())
            pitch = -5.0 + 10.0 * rng.random()
            if headline:
                w, hh = 1920, 1080
                t = 6.0
            else:
                w, hh = res[int(rng.integers(0, 3))] if config == 3 else (1920, 1080)
                xi = rng.random()
                lo, hi = (2.0, 15.0) if config == 3 else (3.0, 15.0)
                t = hi ** xi * lo ** (1.0 - xi)
            if tau is not None:
                t = tau
            out.append(look_dir((x, y, 1.7), yaw, pitch, w, hh, t))
        return out
    raise ValueError(config)


def perturb_interior(h: Hierarchy, seed: int = 2024, sigma: float = 0.05) -> Hierarchy:
    """The differentiation workload's target hierarchy: a copy of ``h`` whose
    interior nodes have their means moved by N(0, sigma), their scales
    multiplied by exp(N(0, sigma)) (a log-scale perturbation) and their SH
    coefficients moved by N(0, sigma); leaves, boxes and topology unchanged."""
    import dataclasses
    rng = np.random.default_rng(seed)
    inner = h.child_count > 0
    m = int(inner.sum())
    hp = dataclasses.replace(h, mean=h.mean.copy(), scale=h.scale.copy(), sh=h.sh.copy())
    hp.mean[:, inner] += rng.normal(0.0, sigma, size=(3, m)).astype(np.float32)
    hp.scale[:, inner] *= np.exp(rng.normal(0.0, sigma, size=(3, m))).astype(np.float32)
    hp.sh[:, inner] += rng.normal(0.0, sigma, size=(48, m)).astype(np.float32)
    return hp
