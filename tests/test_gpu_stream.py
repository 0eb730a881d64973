"""Out-of-core rendering (Sec. 6.3; hgs_stream_*) through the C ABI: along a
camera path, every image equals the in-core render's bit for bit, and the
records transferred per frame equal a plain set simulation of the cache on
the oracle's cuts (needed = every cut node and its parent; transferred =
needed minus resident; the cleanup frees records unused for more than
max_age frames).  Also the capacity error and the calls refused while
streaming."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_12080_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _path(n):
    """n frames of one or two views moving through the 60k-leaf box scene."""
    out = []
    for f in range(n):
        a = 0.25 * f
        eye = (30 * np.cos(a), 30 * np.sin(a), 1.7 + 0.3 * f)
        v = synth.look_at(eye, (0, 0, 2.5), (0, 0, 1), 640, 360, 6.0 if f % 3 else 3.0)
        if f == 4:
            out.append([v, synth.look_at((0, -45, 4), (0, 0, 2.5), (0, 0, 1), 320, 180, 8.0)])
        else:
            out.append([v])
    return out


def test_streamed_frames_equal_in_core_and_transfers_match_the_cache_simulation():
    from paper_2406_12080_amd import hgs
    h = synth.make_scene(2, n_leaves=60_000)
    H = O.Hier(h)
    frames = _path(9)
    cleanup_after, max_age = 5, 2
    r = hgs.Renderer(0)
    try:
        r.upload(h)
        ref = []
        for views in frames:
            imgs, _ = r.render(views)
            ref.append([i.clone() for i in imgs])
        r.stream_begin(h.n_nodes)  # room for every node: eviction only by the cleanup
        info0 = r.stream_info()
        assert info0["resident"] == 0 and info0["frame"] == 0
        resident = {}  # node -> frame of last use (the simulation)
        parent = np.asarray(h.parent)
        for f, views in enumerate(frames, start=1):
            imgs, st = r.render(views)
            for a, b in zip(imgs, ref[f - 1]):
                assert torch.equal(a, b), f
            need = set()
            for v in views:
                ids, _ = O.cut(H, v)
                need |= set(ids.tolist())
                p = parent[ids]
                need |= set(p[p >= 0].tolist())
            want = len(need - resident.keys())
            for x in need:
                resident[x] = f
            info = r.stream_info()
            assert info["frame"] == f and info["overflow"] == 0
            assert info["requested"] == want, (f, info, want)
            assert info["resident"] == len(resident), (f, info, len(resident))
            if f == cleanup_after:
                r.stream_cleanup(max_age)
                resident = {x: lu for x, lu in resident.items() if f - lu <= max_age}
                assert r.stream_info()["resident"] == len(resident)
        # calls refused while streaming
        P = hgs.params_to_device(h)
        with pytest.raises(hgs.HgsError) as e:
            r.bind(*[P[k] for k in hgs.PARAM_FIELDS])
        assert e.value.status == hgs.ERR_STATE
        r.stream_end()
        imgs, _ = r.render(frames[0])
        assert torch.equal(imgs[0], ref[0][0])
    finally:
        r.close()


def test_a_cache_too_small_reports_capacity():
    from paper_2406_12080_amd import hgs
    h = synth.make_scene(1)
    r = hgs.Renderer(0)
    try:
        r.upload(h)
        r.stream_begin(50)
        with pytest.raises(hgs.HgsError) as e:
            r.render([synth.make_views(1, tau=4.0)[0]])
        assert e.value.status == hgs.ERR_CAPACITY
        info = r.stream_info()
        assert info["overflow"] == 1 and info["resident"] == 50
        # the root alone does not fit while the cache is full of frame 1's
        # records; after a cleanup with max_age 0 at frame 2 it does
        root_view = synth.make_views(1, tau=1e6)[0]
        with pytest.raises(hgs.HgsError):
            r.render([root_view])
        r.stream_cleanup(0)
        assert r.stream_info()["resident"] == 0
        _, st = r.render([root_view])
        info = r.stream_info()
        assert info["overflow"] == 0 and info["resident"] == 1 and st["cut"] == 1
    finally:
        r.close()
