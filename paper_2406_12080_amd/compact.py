"""Hierarchy compaction (Sec. 5.2, "Compacting the Hierarchy"): the tree
rebuilt from the keep flags of ``hgs_compact_mark``.

Every kept node's parent becomes its nearest kept ancestor, so a node may end
up with more than eight children (the alpha blending takes K from the child
count, Eq. (alphap) for K children).  Node attributes and boxes are carried
over unchanged: the leaves under a kept node are the same, so its box (the
union of their boxes) is too.  The result is in the layout ``hgs_upload``
takes: breadth-first order, root first, the children of a node contiguous
and ordered as they were.
"""
from __future__ import annotations

import numpy as np

from .synth import Hierarchy


def rebuild(h: Hierarchy, keep) -> Hierarchy:
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
