"""Hierarchy compaction on the GPU (``hgs_compact_mark``) against the FP64
oracle's step-by-step compaction (bit-exact keep flags), and rendering of
the compacted tree against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import oracle as O
from paper_2406_12080_amd import compact, synth
import parity as PR

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hgs_mod():
    from paper_2406_12080_amd import hgs
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    hgs.lib()
    return hgs


@pytest.fixture(scope="module")
def c1():
    return synth.make_scene(1)


@pytest.fixture(scope="module")
def c2s():
    return synth.make_scene(2, n_leaves=60_000)


def c1_train_views():
    eyes = [(0, 0, 3), (2.5, 0.5, 1.5), (-1.5, 2.0, 2.0), (0.2, -3.0, 0.5), (0, 0, 10), (0.1, 0.2, 0.3)]
    return [synth.look_at(e, (0, 0, 0), (0, 1, 0), 256, 256, 1.0) for e in eyes]


def c2_train_views():
    out = [synth.look_at((x, y, 1.7), (0, 0, 2.5), (0, 0, 1), 1280, 720, 6.0)
           for x, y in [(-30, -40), (0, -40), (25, -35), (40, 0), (0, 40)]]
    out.append(synth.look_at((0, 0, 3.0), (10, 5, 2.0), (0, 0, 1), 640, 360, 6.0))  # eye inside the scene
    return out


@pytest.mark.parametrize("ladder", [(3.0, None), (1.5, 64.0), (3.0, 3.0)])
def test_keep_flags_match_oracle_c1(hgs_mod, c1, ladder):
    r = hgs_mod.Renderer(0)
    r.upload(c1)
    views = c1_train_views()
    lo, hi = ladder
    keep = r.compact_mark(views, lo, hi).cpu().numpy()
    ref = O.compact_keep(c1, views, lo, hi)
    assert np.array_equal(keep, ref)
    if hi is None:
        assert 0 < np.count_nonzero(~keep)
    r.close()


def test_keep_flags_match_oracle_c2s(hgs_mod, c2s):
    r = hgs_mod.Renderer(0)
    r.upload(c2s)
    views = c2_train_views()
    keep = r.compact_mark(views).cpu().numpy()
    ref = O.compact_keep(c2s, views)
    assert np.array_equal(keep, ref)
    print("c2s removed", int(np.count_nonzero(~keep)), "of", c2s.n_nodes)
    r.close()


def test_more_views_than_one_batch(hgs_mod, c1):
    # 1100 views: two batches of the per-node maximum; against the oracle's
    # literal steps on every view
    rng = np.random.default_rng(11)
    views = []
    for _ in range(1100):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        views.append(synth.look_at(tuple(d * rng.uniform(1.6, 12.0)), (0, 0, 0), (0, 1, 0) if abs(d[1]) < 0.9
                                   else (1, 0, 0), 128, 128, 1.0))
    r = hgs_mod.Renderer(0)
    r.upload(c1)
    keep = r.compact_mark(views, 3.0, 64.0).cpu().numpy()
    ref = O.compact_keep(c1, views, 3.0, 64.0)
    assert np.array_equal(keep, ref)
    r.close()


def test_no_level_and_bad_arguments(hgs_mod, c1):
    r = hgs_mod.Renderer(0)
    r.upload(c1)
    views = c1_train_views()
    assert r.compact_mark(views, 200.0, 100.0).all()
    for lo, hi in [(0.0, 10.0), (-1.0, 10.0), (float("nan"), 10.0), (3.0, float("inf")), (1e-30, 1e30)]:
        with pytest.raises(RuntimeError):
            r.compact_mark(views, lo, hi)
    r.close()


def test_compacted_tree_renders_like_oracle(hgs_mod, c2s):
    from paper_2406_12080_amd import hgs
    r = hgs_mod.Renderer(0)
    r.upload(c2s)
    views = c2_train_views()
    keep = r.compact_mark(views).cpu().numpy()
    r.close()
    c = compact.rebuild(c2s, keep)
    assert c.n_nodes == int(keep.sum())
    assert c.child_count.max() > 8  # Eq. (alphap) with K > 8 children
    print("children per node up to", int(c.child_count.max()))
    rc = hgs_mod.Renderer(0)
    rc.upload(c)
    for tau in (3.0, 6.0, 15.0):
        v = PR.safe_tau(c, synth.look_at((5, -38, 1.7), (0, 0, 2.5), (0, 0, 1), 482, 271, tau))
        imgs, st = rc.render([v])
        rgb = imgs[0].cpu().numpy().reshape(-1, 3).astype(np.float64)
        T = rc.buffer(hgs.BUF_T_FINAL, torch.float32).cpu().numpy().astype(np.float64)
        o = O.render(c, v)
        res = PR.check_pixels(rgb, T, o)
        print(tau, res, st)
        assert res["ok"], res
        assert st["cut"] == len(O.cut(c, v)[0])
    rc.close()
