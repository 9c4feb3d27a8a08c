"""Thin-layer positive-depth operator (Sec. 2.4), FP64, vectorised.

The operator is split into a depth part and a discharge part, both acting
element by element on the nodal (vertex) values of the linear part of the
solution, with H_i the depth at vertex i and Hbar their mean:

depth part
  1. all H_i >= H0          -> unchanged;
  2. Hbar <= H0             -> every H_i := Hbar;
  3. otherwise redistribute so that every H_i >= H0 and the sum is kept.
     The paper gives only these two constraints; the rule used is: sort the
     depths ascending (ties by local index), set the smallest to H0, lower
     the middle one by half the water the smallest received (but not below
     H0), and give the largest what keeps the sum.
A vertex is dry when its new depth is <= H0 (the paper says "less than";
with a strict test case 3 would never leave a dry vertex and the partial
discharge redistribution described next could not occur).  The solver
applies this test with a margin of 1e-3 H0 (the depth part puts vertices at
exactly H0, so later tests on them would otherwise be ties decided by
round-off); the functions here take the dry mask from the caller.

discharge part
  the discharge of dry vertices is removed and spread evenly over the wet
  vertices of the element (total kept); when every vertex is dry the
  discharge is zeroed.

An element is flagged dry when all three of its vertices are dry.
"""
from __future__ import annotations

import numpy as np


def depth_operator(Hv, H0):
    """Depth part on (E, 3) vertex depths.  Returns (H_new, changed_mask)."""
    Hv = np.asarray(Hv, dtype=np.float64)
    S = Hv[:, 0] + Hv[:, 1] + Hv[:, 2]
    Hbar = S / 3.0
    case1 = np.all(Hv >= H0, axis=1)
    case2 = (~case1) & (Hbar <= H0)
    case3 = (~case1) & (~case2)
    out = Hv.copy()
    out[case2] = Hbar[case2, None]
    if np.any(case3):
        h = Hv[case3]
        order = np.argsort(h, axis=1, kind="stable")
        hs = np.take_along_axis(h, order, axis=1)
        n1 = np.full(hs.shape[0], H0)
        n2 = np.maximum(H0, hs[:, 1] - (H0 - hs[:, 0]) / 2.0)
        n3 = S[case3] - n1 - n2
        new_sorted = np.stack([n1, n2, n3], axis=1)
        res = np.empty_like(h)
        np.put_along_axis(res, order, new_sorted, axis=1)
        out[case3] = res
    return out, ~case1


def discharge_operator(qv, dry):
    """Discharge part on (E, 3) vertex discharges with (E, 3) dry mask."""
    qv = np.asarray(qv, dtype=np.float64)
    n_dry = dry.sum(axis=1)
    n_wet = 3 - n_dry
    delta = np.where(dry, qv, 0.0)
    delta = delta[:, 0] + delta[:, 1] + delta[:, 2]
    out = qv.copy()
    some = (n_dry > 0) & (n_wet > 0)
    add = np.zeros_like(delta)
    add[some] = delta[some] / n_wet[some]
    out = np.where(dry, 0.0, qv + add[:, None])
    out[n_dry == 0] = qv[n_dry == 0]
    out[n_wet == 0] = 0.0
    return out, n_dry > 0
