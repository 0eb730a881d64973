"""hgs_cut_noalloc (the cut with its working memory in the library's static
device array) against hgs_cut, through the C ABI: two calls in a row on one
device, the second on a smaller hierarchy, each node for node and weight for
weight equal to the allocating entry point; the capacity error; and the
state kept for the backward left as it was."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2406_12080_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _both(r, v):
    ids_a, t_a = r.cut(v)
    cap = int(ids_a.numel()) + 7
    ids_b = torch.full((cap,), -5, dtype=torch.int32, device="cuda")
    t_b = torch.full((cap,), -5.0, dtype=torch.float32, device="cuda")
    n = r.cut_noalloc(v, ids_b, t_b)
    torch.cuda.synchronize()
    return ids_a.cpu().numpy(), t_a.cpu().numpy(), n, ids_b.cpu().numpy(), t_b.cpu().numpy()


def test_noalloc_cut_equals_cut_twice_second_smaller():
    from paper_2406_12080_amd import hgs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    big = synth.make_scene(2, n_leaves=60_000)
    small = synth.make_scene(1)
    assert small.n_nodes < big.n_nodes
    r = hgs.Renderer(0)
    try:
        r.upload(big)
        v_big = synth.look_at((0, -40, 1.7), (0, 0, 2.5), (0, 0, 1), 640, 360, 3.0)
        ia, ta, n, ib, tb = _both(r, v_big)
        assert n == ia.shape[0] > 1000
        assert np.array_equal(ib[:n], ia) and np.array_equal(tb[:n], ta)
        assert (ib[n:] == -5).all() and (tb[n:] == -5.0).all()  # nothing past the cut
        # second call: a smaller hierarchy and a coarser cut, over what the
        # first call left in the static array
        r.upload(small)
        v_small = synth.make_views(1, tau=16.0)[0]
        ia2, ta2, n2, ib2, tb2 = _both(r, v_small)
        assert 0 < n2 == ia2.shape[0] < n
        assert np.array_equal(ib2[:n2], ia2) and np.array_equal(tb2[:n2], ta2)
        # without weights, and the capacity error (count still reported)
        ids = torch.empty(n2, dtype=torch.int32, device="cuda")
        assert r.cut_noalloc(v_small, ids, None) == n2
        assert np.array_equal(ids.cpu().numpy(), ia2)
        short = torch.empty(n2 - 1, dtype=torch.int32, device="cuda")
        with pytest.raises(hgs.HgsError) as e:
            r.cut_noalloc(v_small, short, None)
        assert e.value.status == hgs.ERR_CAPACITY
    finally:
        r.close()


def test_noalloc_cut_keeps_the_render_state():
    from paper_2406_12080_amd import hgs
    h = synth.make_scene(1)
    r = hgs.Renderer(0)
    try:
        r.upload(h)
        P = hgs.params_to_device(h)
        r.bind(*[P[k] for k in hgs.PARAM_FIELDS])
        v = synth.make_views(1, tau=4.0)[0]
        (img,), st = r.render([v])
        rid = r.last_render()
        w = torch.ones_like(img)
        g1 = {k: torch.zeros_like(P[k]) for k in hgs.PARAM_FIELDS}
        r.backward([w], g1)
        ids = torch.empty(h.n_nodes, dtype=torch.int32, device="cuda")
        assert r.cut_noalloc(synth.make_views(1, tau=64.0)[0], ids) > 0
        assert r.last_render() == rid
        g2 = {k: torch.zeros_like(P[k]) for k in hgs.PARAM_FIELDS}
        r.backward([w], g2)
        torch.cuda.synchronize()
        for k in hgs.PARAM_FIELDS:
            assert torch.equal(g1[k], g2[k]), k
    finally:
        r.close()
