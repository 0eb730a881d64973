"""Hierarchy compaction (Sec. 5.2, "Compacting the Hierarchy"): the tree
rebuilt from the keep flags of ``hgs_compact_mark``, by the library's
``hgs_compact_rebuild`` (host code).

Every kept node's parent becomes its nearest kept ancestor, so a node may end
up with more than eight children (the alpha blending takes K from the child
count, Eq. (alphap) for K children).  Node attributes and boxes are carried
over unchanged: the leaves under a kept node are the same, so its box (the
union of their boxes) is too.  The result is in the layout ``hgs_upload``
takes: breadth-first order, root first, the children of a node contiguous
and ordered as they were.
"""
from __future__ import annotations

import ctypes

import numpy as np

from .synth import Hierarchy


def rebuild(h: Hierarchy, keep) -> Hierarchy:
    from . import hgs
    keep = np.ascontiguousarray(np.asarray(keep, dtype=bool).reshape(-1), dtype=np.uint8)
    n = h.n_nodes
    if keep.shape[0] != n:
        raise ValueError(f"keep has {keep.shape[0]} flags for {n} nodes")
    parent = np.ascontiguousarray(h.parent, np.int32)
    count = np.ascontiguousarray(h.child_count, np.int32)
    order, new_parent, child_begin, child_count = (np.empty(n, np.int32) for _ in range(4))
    m = ctypes.c_int64()
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)  # noqa: E731
    st = hgs.lib().hgs_compact_rebuild(ptr(parent), ptr(count), ptr(keep), n, ptr(order), ptr(new_parent),
                                       ptr(child_begin), ptr(child_count), ctypes.byref(m))
    if st != 0:
        raise ValueError(f"hgs_compact_rebuild failed ({st}): the root and every leaf must be kept, "
                         "and the topology must be breadth-first")
    m = m.value
    order = order[:m].astype(np.int64)
    info = dict(h.info)
    info.update(compacted_from=n, removed=n - m, max_children=int(child_count[:m].max(initial=0)))

    def take(a):
        return np.ascontiguousarray(np.take(a, order, axis=a.ndim - 1))

    return Hierarchy(parent=new_parent[:m].copy(), child_begin=child_begin[:m].copy(),
                     child_count=child_count[:m].copy(), bmin=take(h.bmin), bmax=take(h.bmax), mean=take(h.mean),
                     scale=take(h.scale), rot=take(h.rot), opacity=take(h.opacity), sh=take(h.sh), info=info)
