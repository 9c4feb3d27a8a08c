"""Connectivity and FP64 geometry of an unstructured triangle mesh.

The DG operator is local to each element and couples neighbours only through
edge integrals (Sec. 2.3), so the oracle needs, per element: its CCW vertex
list, the neighbour across each local edge (and that neighbour's local edge
index), the boundary type and forcing slot of each boundary edge, the
constant Jacobian of the affine map from the reference triangle, the outward
unit normals and lengths of its three edges, and the inscribed-circle
diameter used by the CFL time step.

Local edge k joins local vertices k -> k+1 (mod 3).  The affine map is
x(r,s) = -(r+s)/2 x_a + (1+r)/2 x_b + (1+s)/2 x_c, so J is constant and
det J = area / 2.
"""
from __future__ import annotations

import numpy as np

LAND, OCEAN, RIVER, OUTFLOW = 0, 1, 2, 3


class MeshError(ValueError):
    pass


def build(xy, tri, bedges=None, btype=None, bslot=None):
    xy = np.asarray(xy, dtype=np.float64)
    tri = np.array(tri, dtype=np.int64, copy=True)
    n, m = xy.shape[0], tri.shape[0]
    if tri.ndim != 2 or tri.shape[1] != 3:
        raise MeshError("tri must be (m, 3)")
    if m and (tri.min() < 0 or tri.max() >= n):
        raise MeshError("node id out of range")
    # orient counter-clockwise
    xa, xb, xc = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    cross = (xb[:, 0] - xa[:, 0]) * (xc[:, 1] - xa[:, 1]) - (xb[:, 1] - xa[:, 1]) * (xc[:, 0] - xa[:, 0])
    if np.any(cross == 0.0):
        raise MeshError("zero-area triangle")
    flip = cross < 0.0
    tri[flip] = tri[flip][:, [0, 2, 1]]
    # edges: key = (min, max) node pair
    a = tri
    b = np.roll(tri, -1, axis=1)                     # local edge k: v_k -> v_{k+1}
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    key = (lo.astype(np.int64) * n + hi).ravel()
    order = np.argsort(key, kind="stable")
    ks = key[order]
    uniq, start, counts = np.unique(ks, return_index=True, return_counts=True)
    if np.any(counts > 2):
        raise MeshError("non-manifold edge (shared by more than two triangles)")
    nbr = np.full(3 * m, -1, dtype=np.int64)
    nbr_edge = np.full(3 * m, -1, dtype=np.int64)
    two = start[counts == 2]
    f0, f1 = order[two], order[two + 1]
    nbr[f0], nbr[f1] = f1 // 3, f0 // 3
    nbr_edge[f0], nbr_edge[f1] = f1 % 3, f0 % 3
    nbr = nbr.reshape(m, 3)
    nbr_edge = nbr_edge.reshape(m, 3)
    # boundary edges: match the user's list; unlisted boundary edges are LAND
    btype_e = np.full((m, 3), -1, dtype=np.int64)
    bslot_e = np.full((m, 3), -1, dtype=np.int64)
    isb = nbr < 0
    btype_e[isb] = LAND
    bslot_e[isb] = 0
    if bedges is not None and len(bedges):
        bedges = np.asarray(bedges, dtype=np.int64)
        bk = np.minimum(bedges[:, 0], bedges[:, 1]) * n + np.maximum(bedges[:, 0], bedges[:, 1])
        keymat = key.reshape(m, 3)
        bnd_keys = keymat[isb]
        pos = {int(k): i for i, k in enumerate(bnd_keys)}
        bidx = np.argwhere(isb)
        for j, k in enumerate(bk):
            i = pos.get(int(k))
            if i is None:
                raise MeshError(f"boundary edge {j} is not on the mesh boundary")
            e, kk = bidx[i]
            btype_e[e, kk] = int(btype[j]) if btype is not None else LAND
            bslot_e[e, kk] = int(bslot[j]) if bslot is not None else 0
    g = geometry(xy, tri)
    g.update(dict(tri=tri, nbr=nbr, nbr_edge=nbr_edge, btype=btype_e, bslot=bslot_e,
                  n_flipped=int(flip.sum()), n_nodes=n, n_tri=m))
    return g


def geometry(xy, tri):
    xa, xb, xc = xy[tri[:, 0]], xy[tri[:, 1]], xy[tri[:, 2]]
    J = np.empty((tri.shape[0], 2, 2))
    J[:, 0, 0] = 0.5 * (xb[:, 0] - xa[:, 0])
    J[:, 0, 1] = 0.5 * (xc[:, 0] - xa[:, 0])
    J[:, 1, 0] = 0.5 * (xb[:, 1] - xa[:, 1])
    J[:, 1, 1] = 0.5 * (xc[:, 1] - xa[:, 1])
    detJ = J[:, 0, 0] * J[:, 1, 1] - J[:, 0, 1] * J[:, 1, 0]
    # inverse transpose: [dphi/dx, dphi/dy] = J^{-T} [dphi/dr, dphi/ds]
    JinvT = np.empty_like(J)
    JinvT[:, 0, 0] = J[:, 1, 1] / detJ
    JinvT[:, 0, 1] = -J[:, 1, 0] / detJ
    JinvT[:, 1, 0] = -J[:, 0, 1] / detJ
    JinvT[:, 1, 1] = J[:, 0, 0] / detJ
    verts = np.stack([xa, xb, xc], axis=1)                  # (m, 3, 2)
    ev = np.roll(verts, -1, axis=1) - verts                 # edge k vector v_k -> v_{k+1}
    length = np.hypot(ev[..., 0], ev[..., 1])
    normal = np.stack([ev[..., 1] / length, -ev[..., 0] / length], axis=-1)   # outward for CCW
    area = 2.0 * detJ
    perim = length.sum(axis=1)
    return dict(J=J, detJ=detJ, JinvT=JinvT, area=area, edge_len=length, normal=normal,
                d_in=4.0 * area / perim, verts=verts,
                centroid=verts.mean(axis=1))
