"""Pins for the oracle's connectivity and geometry (Sec. 2.3: element-local
operator coupled through edges)."""
import numpy as np
import pytest

import meshgen
from oracle import mesh


def test_connectivity_and_geometry():
    sc = meshgen.channel_c1()
    g = mesh.build(sc.mesh.xy, sc.mesh.tri, sc.mesh.bedges, sc.mesh.btype, sc.mesh.bslot)
    E = g["n_tri"]
    assert E == 1024 and g["n_nodes"] == 585
    nbr, ne = g["nbr"], g["nbr_edge"]
    inner = nbr >= 0
    assert inner.sum() // 2 + (~inner).sum() == 1608          # edges of the channel mesh
    e, k = np.nonzero(inner)
    assert np.all(nbr[nbr[e, k], ne[e, k]] == e)              # neighbour relation is symmetric
    assert np.sum(g["btype"] == meshgen.OUTFLOW) == 8 and np.sum(g["btype"] == meshgen.LAND) == 136
    np.testing.assert_allclose(g["area"].sum(), 1000.0, rtol=1e-14)
    # outward normals of the two sides of an interior edge are opposite
    np.testing.assert_array_equal(g["normal"][e, k], -g["normal"][nbr[e, k], ne[e, k]])
    np.testing.assert_allclose(np.linalg.norm(g["normal"], axis=2), 1.0, rtol=1e-15)
    # right triangle with legs 1.5625 and 1.25: inscribed diameter 4 A / perimeter
    a, b = 1.5625, 1.25
    np.testing.assert_allclose(g["d_in"][0], 2 * a * b / (a + b + np.hypot(a, b)), rtol=1e-14)


def test_orientation_and_errors():
    xy = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], float)
    g = mesh.build(xy, np.array([[0, 2, 1], [1, 3, 2]]))
    assert g["n_flipped"] == 1 and np.all(g["detJ"] > 0)
    with pytest.raises(mesh.MeshError):
        mesh.build(xy, np.array([[0, 1, 1]]))
    with pytest.raises(mesh.MeshError):
        mesh.build(np.vstack([xy, [[0.5, -1]]]), np.array([[0, 1, 2], [1, 0, 3], [0, 1, 4]]))
    with pytest.raises(mesh.MeshError):
        mesh.build(xy, np.array([[0, 1, 2], [1, 3, 2]]), np.array([[1, 2]]), np.array([0]), np.array([0]))
    with pytest.raises(mesh.MeshError):
        mesh.build(xy, np.array([[0, 1, 7]]))
