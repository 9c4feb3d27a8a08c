"""The graded coastal generator builds a conforming mesh: every edge is
shared by at most two triangles, the boundary edges are exactly the window's
perimeter, triangles are counter-clockwise and tile the window."""
import numpy as np

from meshgen import graded


def test_graded_small_is_conforming():
    sc = graded.graded_small()
    m = sc.mesh
    xy, tri = m.xy, m.tri
    a, b, c = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    area2 = (b[:, 0] - a[:, 0]) * (c[:, 1] - a[:, 1]) - (b[:, 1] - a[:, 1]) * (c[:, 0] - a[:, 0])
    assert (area2 > 0).all()
    x0, y0 = xy.min(axis=0)
    x1, y1 = xy.max(axis=0)
    assert abs(0.5 * area2.sum() - (x1 - x0) * (y1 - y0)) < 1e-6 * (x1 - x0) * (y1 - y0)
    e = np.sort(np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]), axis=1)
    key, cnt = np.unique(e[:, 0].astype(np.int64) * len(xy) + e[:, 1], return_counts=True)
    assert cnt.max() == 2
    once = key[cnt == 1]
    bk = np.sort(m.bedges, axis=1)
    bkey = np.sort(bk[:, 0].astype(np.int64) * len(xy) + bk[:, 1])
    assert np.array_equal(np.sort(once), bkey)
    # boundary edges lie on the window's outer rectangle
    p, q = xy[m.bedges[:, 0]], xy[m.bedges[:, 1]]
    horiz = np.isclose(p[:, 1], q[:, 1]) & (np.isclose(p[:, 1], y0) | np.isclose(p[:, 1], y1))
    vert = np.isclose(p[:, 0], q[:, 0]) & (np.isclose(p[:, 0], x0) | np.isclose(p[:, 0], x1))
    assert (horiz | vert).all()
    # every node belongs to a triangle; sizes range over several levels
    assert np.unique(tri).size == len(xy)
    side = np.sqrt(0.5 * area2)
    assert side.max() / side.min() > 8.0
    # forcing: ocean, land and river edges are present
    assert set(np.unique(m.btype)) >= {0, 1, 2}


def test_graded_balance_is_two_to_one():
    feat = graded.Features(graded.seed_for(3))
    leaves = graded.build_tree(feat, 6.0, lmax=6, hmin=240.0, window=(30, 33, 3, 3))
    keys = [graded._key(*leaves[L]) for L in range(len(leaves))]
    for L in range(2, len(leaves)):
        i, j = leaves[L]
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            ni, nj = i + di, j + dj
            for k in range(2, L + 1):
                assert not np.isin(graded._key(ni >> k, nj >> k), keys[L - k]).any()
