"""The synthetic hierarchy generator: topology, boxes, merges (CPU)."""
import numpy as np
import pytest

from paper_2406_12080_amd import synth


@pytest.fixture(scope="module")
def h():
    return synth.make_scene(1, n_leaves=3000)


def test_bfs_topology(h):
    N = h.n_nodes
    assert h.parent[0] == -1 and np.all(h.parent[1:] >= 0)
    assert np.all(h.parent[1:] < np.arange(1, N))
    inner = np.nonzero(h.child_count > 0)[0]
    for i in inner:
        kids = np.arange(h.child_begin[i], h.child_begin[i] + h.child_count[i])
        assert np.all(h.parent[kids] == i)
    assert h.child_count.sum() == N - 1
    assert h.child_count.max() <= 8
    assert h.n_leaves == 3000


def test_boxes_nest_and_contain_leaf_3sigma(h):
    p = h.parent[1:]
    assert np.all(h.bmin[:, p] <= h.bmin[:, 1:]) and np.all(h.bmax[:, p] >= h.bmax[:, 1:])
    leaf = h.child_count == 0
    R = synth.quat_to_mat(h.rot[:, leaf].T.astype(np.float64))
    s = h.scale[:, leaf].T.astype(np.float64)
    var = np.einsum("nij,nj->ni", R ** 2, s ** 2)
    ext = 3 * np.sqrt(var)
    m = h.mean[:, leaf].T.astype(np.float64)
    tol = 1e-6 * ext
    assert np.all(h.bmin[:, leaf].T <= m - ext + tol)
    assert np.all(h.bmax[:, leaf].T >= m + ext - tol)


def test_merge_moments(h):
    # Eq. (merge) with weights o_i * S_i: parent mean = weighted children means
    inner = np.nonzero(h.child_count > 0)[0][:200]
    for i in inner:
        kids = np.arange(h.child_begin[i], h.child_begin[i] + h.child_count[i])
        s = h.scale[:, kids].T.astype(np.float64)
        p = 1.6075
        a, b, c = s[:, 0] ** p, s[:, 1] ** p, s[:, 2] ** p
        S = 4 * np.pi * ((a * b + a * c + b * c) / 3) ** (1 / p)
        w = h.opacity[kids].astype(np.float64) * S
        mu = (w[:, None] * h.mean[:, kids].T).sum(0) / w.sum()
        assert np.allclose(mu, h.mean[:, i], rtol=1e-5, atol=1e-6)


def test_orientation_hemisphere(h):
    q = h.rot.astype(np.float64)
    dots = (q[:, 1:] * q[:, h.parent[1:]]).sum(0)
    assert np.all(dots >= -1e-6)
    assert np.allclose(np.linalg.norm(q, axis=0), 1, atol=1e-6)
