"""Hierarchy compaction (Sec. 5.2, "Compacting the Hierarchy"): the oracle's
step-by-step keep flags pinned by hand-derived trees and by an equivalent
formulation, and the host rebuild of the tree.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_12080_amd import compact, synth
from paper_2406_12080_amd.synth import Hierarchy
import scenes as S


def box_tree(parent, L):
    """Nested boxes [100, 100 + L] x [-L/2, L/2]^2: seen from the origin with
    focal length f, a node's granularity is f L / 100."""
    parent = np.asarray(parent, np.int32)
    n = parent.shape[0]
    L = np.asarray(L, np.float64)
    child_count = np.bincount(parent[1:], minlength=n).astype(np.int32)
    child_begin = np.zeros(n, np.int32)
    for i in range(n - 1, 0, -1):
        child_begin[parent[i]] = i
    bmin = np.stack([np.full(n, 100.0), -L / 2, -L / 2]).astype(np.float32)
    bmax = np.stack([100.0 + L, L / 2, L / 2]).astype(np.float32)
    mean = 0.5 * (bmin + bmax)
    return Hierarchy(parent=parent, child_begin=child_begin, child_count=child_count, bmin=bmin, bmax=bmax,
                     mean=mean, scale=np.ones((3, n), np.float32), rot=np.tile([[1], [0], [0], [0]], n).astype(np.float32),
                     opacity=np.full(n, 0.5, np.float32), sh=np.zeros((48, n), np.float32))


def test_granularity_of_box_tree_is_its_size():
    h = box_tree([-1, 0, 1], [100.0, 20.0, 8.0])
    assert np.allclose(O.granularity(h, S.axis_view(64, 64, 100.0)), [100.0, 20.0, 8.0], rtol=1e-15)
    assert np.allclose(O.granularity(h, S.axis_view(64, 64, 150.0)), [150.0, 30.0, 12.0], rtol=1e-15)


def test_chain_removes_the_nodes_between_two_levels():
    # root 100 > a 40 > b 38 > c 30 > d 8 > two leaves; one view, eps = L;
    # taus 3, 6, 12, 24, 48: d is the cut at 12 (8 <= 12 < 30), a at 48
    # (40 <= 48 < 100); b and c lie between d and a and are removed
    h = box_tree([-1, 0, 1, 2, 3, 4, 4], [100, 40, 38, 30, 8, 1, 1])
    keep = O.compact_keep(h, [S.axis_view(100, 100, 100.0)], 3.0, 50.0)
    assert keep.tolist() == [True, True, False, False, True, True, True]


def test_ladder_includes_tau_max():
    # the same chain with tau_max = 48 exactly: the level at 48 is taken, so
    # b and c go; stopping before it would leave them above the last cut
    h = box_tree([-1, 0, 1, 2, 3, 4, 4], [100, 40, 38, 30, 8, 1, 1])
    v = [S.axis_view(100, 100, 100.0)]
    assert O.compact_keep(h, v, 3.0, 48.0).tolist() == [True, True, False, False, True, True, True]
    assert O.compact_keep(h, v, 3.0, 47.0).all()


def test_union_of_cuts_keeps_a_node_one_view_alone_removes():
    # root 100 > A 20 > M 18 > {a1, a2} 8 > two leaves each.  View 1 sees
    # eps = L, view 2 (focal 150) eps = 1.5 L.  Taus 3.5, 7, 14, 28, 56.
    # View 1 alone: a1, a2 at 14, A at 28, so M (between them) is removed.
    # Both views at 28: view 1's cut holds A, view 2's holds M (27 <= 28 <
    # 30); M is the bottom-most node of the union, so it is kept.
    h = box_tree([-1, 0, 1, 2, 2, 3, 3, 4, 4], [100, 20, 18, 8, 8, 1, 1, 1, 1])
    v1 = S.axis_view(120, 120, 100.0)
    v2 = S.axis_view(120, 120, 150.0)
    one = O.compact_keep(h, [v1], 3.5, 60.0)
    assert one.tolist() == [True, True, False] + [True] * 6
    both = O.compact_keep(h, [v1, v2], 3.5, 60.0)
    assert both.all()


def test_no_level_keeps_everything():
    h = box_tree([-1, 0, 1, 2, 3, 4, 4], [100, 40, 38, 30, 8, 1, 1])
    assert O.compact_keep(h, [S.axis_view(100, 100, 100.0)], 64.0, 50.0).all()


def _keep_from_max_granularity(h, views, tau_min, tau_max):
    # the bottom-most nodes of the union of the cuts at tau are the nodes that
    # every view finds fine enough while some view finds their parent too
    # coarse (and the root, if every view finds it fine enough): with e(n) the
    # largest eps over the views, e(n) <= tau < e(parent); kept are the leaves,
    # those nodes at some level, and the nodes above the last level's cut
    e = np.max([O.granularity(h, v) for v in views], axis=0)
    leaf = h.child_count == 0
    par = h.parent.astype(np.int64)
    ep = np.where(par >= 0, e[np.maximum(par, 0)], np.inf)
    keep = leaf.copy()
    tau = float(np.float32(tau_min))
    last = None
    while tau <= float(np.float32(tau_max)):
        keep |= (e <= tau) & ~(ep <= tau)
        last = tau
        tau *= 2.0
    if last is None:
        return np.ones_like(keep)
    return keep | ~((e <= last) | leaf)


@pytest.mark.parametrize("case", ["c1", "c2"])
def test_steps_match_the_max_granularity_form(case):
    if case == "c1":
        h = synth.make_scene(1)
        views = [synth.look_at(e, (0, 0, 0), (0, 1, 0), 256, 256, 1.0)
                 for e in [(0, 0, 3), (2.5, 0.5, 1.5), (-1.5, 2.0, 2.0), (0.2, -3.0, 0.5), (0, 0, 10)]]
        lo, hi = 3.0, 128.0
    else:
        h = synth.make_scene(2, n_leaves=20_000)
        views = [synth.look_at((x, -40, 1.7), (0, 0, 2.5), (0, 0, 1), 640, 360, 6.0) for x in (-30, 0, 25)]
        views.append(synth.look_at((0, 0, 3.0), (10, 5, 2.0), (0, 0, 1), 640, 360, 6.0))  # eye inside the scene
        lo, hi = 3.0, 320.0
    keep = O.compact_keep(h, views, lo, hi)
    ref = _keep_from_max_granularity(h, views, lo, hi)
    assert np.array_equal(keep, ref)
    assert keep[h.child_count == 0].all() and keep[0]
    assert 0 < np.count_nonzero(~keep) < h.n_nodes
    print(case, h.n_nodes, "removed", int(np.count_nonzero(~keep)))


def test_rebuild_links_each_node_to_its_nearest_kept_ancestor():
    h = synth.make_scene(1)
    views = [synth.look_at(e, (0, 0, 0), (0, 1, 0), 256, 256, 1.0) for e in [(0, 0, 3), (2.5, 0.5, 1.5)]]
    keep = O.compact_keep(h, views, 3.0, 128.0)
    c = compact.rebuild(h, keep)
    old = np.nonzero(keep)[0]
    m = c.n_nodes
    assert m == old.shape[0] and c.n_leaves == h.n_leaves
    # the node at each new position, found by its (unique) box and attributes
    key_old = {tuple(np.concatenate([h.bmin[:, i], h.bmax[:, i], h.mean[:, i], h.sh[:3, i]]).tolist()): i for i in old}
    assert len(key_old) == old.shape[0]
    src = np.array([key_old[tuple(np.concatenate([c.bmin[:, k], c.bmax[:, k], c.mean[:, k], c.sh[:3, k]]).tolist())]
                    for k in range(m)])
    assert src[0] == 0
    pos = {int(i): k for k, i in enumerate(src)}
    for k in range(1, m):
        a = int(h.parent[src[k]])
        while not keep[a]:
            a = int(h.parent[a])
        assert c.parent[k] == pos[a]
    # breadth-first layout with contiguous children
    assert c.parent[0] == -1 and (c.parent[1:] < np.arange(1, m)).all()
    assert (np.diff(c.parent[1:]) >= 0).all()
    assert int(c.child_count.sum()) == m - 1
    for k in np.nonzero(c.child_count)[0]:
        kids = np.arange(c.child_begin[k], c.child_begin[k] + c.child_count[k])
        assert (c.parent[kids] == k).all()
    for name in ("bmin", "bmax", "mean", "scale", "rot", "sh"):
        assert np.array_equal(getattr(c, name), getattr(h, name)[:, src])
    assert np.array_equal(c.opacity, h.opacity[src])


def test_rebuild_rejects_a_removed_leaf_root_or_a_malformed_tree():
    h = box_tree([-1, 0, 1, 2, 3, 4, 4], [100, 40, 38, 30, 8, 1, 1])
    for bad in (5, 0):
        keep = np.ones(7, bool)
        keep[bad] = False
        with pytest.raises(ValueError):
            compact.rebuild(h, keep)
    h.parent[3] = 5  # a parent after its child
    with pytest.raises(ValueError):
        compact.rebuild(h, np.ones(7, bool))
    with pytest.raises(ValueError):
        compact.rebuild(h, np.ones(6, bool))


def _rebuild_numpy(h: Hierarchy, keep) -> Hierarchy:
    # independent NumPy construction of the same tree (reference for the
    # library's host code): pointer steps over removed nodes, depth passes,
    # and a level-by-level lexicographic sort
    keep = np.asarray(keep, dtype=bool).reshape(-1)
    n = h.n_nodes
    if keep.shape[0] != n:
        raise ValueError(f"keep has {keep.shape[0]} flags for {n} nodes")
    leaf = h.child_count == 0
    if not keep[0] or not keep[leaf].all():
        raise ValueError("the root and every leaf must be kept")
    parent = h.parent.astype(np.int64)
    # nearest kept proper ancestor: step over removed nodes until every
    # ancestor pointer lands on a kept node (or past the root)
    anc = parent.copy()
    while True:
        moved = anc >= 0
        moved[moved] = ~keep[anc[moved]]
        if not moved.any():
            break
        anc[moved] = parent[anc[moved]]
    ids = np.nonzero(keep)[0]
    ids = ids[ids != 0]
    # depth in the new tree (parents precede children in the old order, so
    # as many passes as levels settle it)
    depth = np.zeros(n, np.int64)
    for _ in range(int(h.info.get("levels", 0)) + 64):
        nd = depth.copy()
        nd[ids] = depth[anc[ids]] + 1
        if np.array_equal(nd, depth):
            break
        depth = nd
    else:
        raise RuntimeError("depth did not settle")
    # breadth-first order: level by level, children grouped by their
    # parent's new position, siblings in their old order
    newidx = np.full(n, -1, np.int64)
    newidx[0] = 0
    order = [np.zeros(1, np.int64)]
    placed = 1
    dmax = int(depth[ids].max(initial=0))
    for d in range(1, dmax + 1):
        lv = ids[depth[ids] == d]
        lv = lv[np.lexsort((lv, newidx[anc[lv]]))]
        newidx[lv] = placed + np.arange(lv.shape[0])
        placed += lv.shape[0]
        order.append(lv)
    order = np.concatenate(order)
    m = order.shape[0]
    new_parent = np.full(m, -1, np.int64)
    new_parent[1:] = newidx[anc[order[1:]]]
    child_count = np.bincount(new_parent[1:], minlength=m).astype(np.int32)
    child_begin = np.zeros(m, np.int32)
    has = child_count > 0
    child_begin[has] = 1 + np.searchsorted(new_parent[1:], np.nonzero(has)[0], side="left")
    info = dict(h.info)
    info.update(compacted_from=n, removed=n - m, max_children=int(child_count.max(initial=0)))

    def take(a):
        return np.ascontiguousarray(a[..., order])

    return Hierarchy(parent=new_parent.astype(np.int32), child_begin=child_begin, child_count=child_count,
                     bmin=take(h.bmin), bmax=take(h.bmax), mean=take(h.mean), scale=take(h.scale),
                     rot=take(h.rot), opacity=take(h.opacity), sh=take(h.sh), info=info)


@pytest.mark.parametrize("case", ["c1", "c2"])
def test_rebuild_matches_an_independent_numpy_construction(case):
    if case == "c1":
        h = synth.make_scene(1)
        views = [synth.look_at(e, (0, 0, 0), (0, 1, 0), 256, 256, 1.0) for e in [(0, 0, 3), (2.5, 0.5, 1.5)]]
        keep = O.compact_keep(h, views, 3.0, 128.0)
    else:
        h = synth.make_scene(2, n_leaves=20_000)
        rng = np.random.default_rng(5)
        keep = (h.child_count == 0) | (rng.random(h.n_nodes) < 0.6)  # any mask that keeps root and leaves
        keep[0] = True
    a, b = compact.rebuild(h, keep), _rebuild_numpy(h, keep)
    for name in ("parent", "child_begin", "child_count", "bmin", "bmax", "mean", "scale", "rot", "opacity", "sh"):
        assert np.array_equal(getattr(a, name), getattr(b, name)), name
    assert a.child_count.max() > 8 or case == "c1"


def test_rebuild_keeping_every_node_is_the_identity():
    h = synth.make_scene(1)
    c = compact.rebuild(h, np.ones(h.n_nodes, bool))
    for name in ("parent", "child_begin", "child_count", "bmin", "bmax", "mean", "scale", "rot", "opacity", "sh"):
        assert np.array_equal(getattr(c, name), getattr(h, name)), name
