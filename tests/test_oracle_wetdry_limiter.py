"""Pins for the positive-depth operator (Sec. 2.4) and the slope limiter.

Depth part: the three cases of Sec. 2.4, mass kept, every depth >= H0
unless all equal the mean, idempotent; a worked example computed by hand.
Discharge part: dry vertices lose their discharge to the wet ones (total
kept), all-dry elements are zeroed.  Limiter: means kept, linear data left
alone away from boundaries (nu >= 1), an isolated extremum is flattened.
"""
import numpy as np
import pytest

import meshgen
from oracle import wetdry, limiter, basis
from oracle.solver import OracleSolver

H0 = 1e-3


def test_depth_worked_example():
    # H = (-0.002, 0.005, 0.020): mean 0.0076667 > H0, one vertex below H0.
    # sorted rule: smallest -> H0 = 0.001; middle loses half of what it gave,
    # 0.005 - (0.001 + 0.002)/2 = 0.0035; largest keeps the sum: 0.0185.
    Hn, ch = wetdry.depth_operator(np.array([[-0.002, 0.005, 0.020]]), H0)
    np.testing.assert_allclose(Hn[0], [0.001, 0.0035, 0.0185], rtol=0, atol=1e-15)
    assert ch[0]
    Hn, _ = wetdry.depth_operator(np.array([[0.020, -0.002, 0.005]]), H0)   # any vertex order
    np.testing.assert_allclose(Hn[0], [0.0185, 0.001, 0.0035], rtol=0, atol=1e-15)


def test_depth_cases_and_invariants():
    rng = np.random.default_rng(0)
    H = rng.uniform(-0.01, 0.02, (20000, 3))
    H[:50] = rng.uniform(0.002, 0.02, (50, 3))          # case 1
    Hn, ch = wetdry.depth_operator(H, H0)
    assert not ch[:50].any() and np.array_equal(Hn[:50], H[:50])
    np.testing.assert_allclose(Hn.sum(1), H.sum(1), rtol=0, atol=1e-15)      # mass kept
    mean = H.sum(1) / 3
    lowmean = mean <= H0
    assert np.all(Hn[lowmean] == mean[lowmean, None])                        # case 2: flat at the mean
    assert np.all(Hn[~lowmean] >= H0 - 1e-18)                                # case 3: all >= H0
    Hn2, _ = wetdry.depth_operator(Hn, H0)                                   # idempotent
    np.testing.assert_allclose(Hn2, Hn, rtol=0, atol=1e-17)


def test_discharge_operator():
    q = np.array([[1.0, 2.0, 3.0], [1.0, 2.0, 3.0], [1.0, 2.0, 3.0], [1.0, -2.0, 3.0]])
    dry = np.array([[False, False, False], [True, False, False], [True, True, True], [False, True, True]])
    qn, ch = wetdry.discharge_operator(q, dry)
    np.testing.assert_allclose(qn[0], [1, 2, 3])
    np.testing.assert_allclose(qn[1], [0, 2.5, 3.5])
    np.testing.assert_allclose(qn[2], [0, 0, 0])
    np.testing.assert_allclose(qn[3], [2.0, 0, 0])
    assert list(ch) == [False, True, True, True]


def _limiter_solver(seed=4):
    sc = meshgen.lake_at_rest(seed=seed, nx=12, ny=8)
    m = sc.mesh
    return OracleSolver(m.xy, m.tri, m.hb, m.fric, m.bedges, m.btype, m.bslot, limiter=True,
                        tides=sc.tides)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_keeps_linear_data_and_means(p):
    s = _limiter_solver()
    T = basis.Tables(p)
    G = s.G
    rng = np.random.default_rng(2)
    a = rng.normal(size=(3, 3))
    v = G["verts"]
    vals = np.stack([a[k, 0] + a[k, 1] * v[..., 0] / 1000 + a[k, 2] * v[..., 1] / 1000 for k in range(3)], 1)
    w = np.zeros((s.E, 3, T.np))
    w[:, :, :3] = np.einsum("mi,evi->evm", T.V1inv, vals)
    st = limiter.stencil(G)
    w2 = limiter.apply(w.copy(), G, st, T)
    np.testing.assert_allclose(w2, w, rtol=0, atol=1e-12)
    # random data: means are kept exactly
    w = rng.normal(size=(s.E, 3, T.np))
    w2 = limiter.apply(w.copy(), G, st, T)
    assert np.array_equal(w2[:, :, 0], w[:, :, 0])
    # elements with a boundary edge are untouched
    bnd = np.any(G["nbr"] < 0, axis=1)
    assert np.array_equal(w2[bnd], w[bnd])


def test_limiter_flattens_isolated_extremum():
    s = _limiter_solver()
    T = basis.Tables(1)
    G = s.G
    w = np.zeros((s.E, 3, 3))
    inner = np.nonzero(np.all(G["nbr"] >= 0, axis=1))[0]
    e = inner[len(inner) // 2]
    w[e, 0, 0] = 1.0        # a bump in the mean ...
    w[e, 0, 1] = 0.3        # ... with a slope the neighbours do not support
    w[e, 0, 2] = -0.2
    w2 = limiter.apply(w.copy(), G, limiter.stencil(G), T)
    assert w2[e, 0, 0] == 1.0 and w2[e, 0, 1] == 0.0 and w2[e, 0, 2] == 0.0


def test_fully_wet_needs_a_wet_mean_at_p2():
    """A p = 2 element can be wet at its vertices and dry on average (low edge
    midpoints).  The positive-depth pass truncates it to its linear part and,
    with the mean below the margin, dries every vertex and zeroes its
    discharge means.  Such an element is not fully wet, so no neighbour's
    limiter reads its means; every fully-wet element keeps its means."""
    s = _limiter_solver()
    s.p = 2
    s.T = basis.Tables(2)
    T = s.T
    G = s.G
    s.hb_m = s.hbv @ T.lam_m.T
    inner = np.nonzero(np.all(G["nbr"] >= 0, axis=1))[0]
    e = inner[len(inner) // 2]
    # depth 1 m at every vertex and -0.5 m at every edge midpoint of e, a
    # uniform current; the rest of the mesh at 0.7 m depth, at rest
    P6 = np.vstack([T.phi_v, T.phi_m])                   # (6 points, 6 modes)
    w = np.zeros((s.E, 3, 6))
    Hpts = np.concatenate([np.full(3, 0.7), np.full(3, 0.7)])
    for k in range(s.E):
        hbp = np.concatenate([s.hbv[k], s.hb_m[k]])
        H = np.concatenate([np.full(3, 1.0), np.full(3, -0.5)]) if k == e else Hpts
        w[k, 0] = np.linalg.solve(P6, H - hbp)
    w[e, 1, 0], w[e, 2, 0] = 0.4, -0.3
    mean_depth = w[e, 0, 0] + s.hbar[e]
    assert mean_depth < 0 and np.all(T.phi_v @ w[e, 0] + s.hbv[e] > 0.9)
    s.use_limiter = True
    s.stencil = limiter.stencil(G)
    w2, flags = s.post(w)
    # e itself: truncated, every vertex at the (negative) mean, dry, discharge zeroed
    assert flags[e] and w2[e, 1, 0] == 0.0 and w2[e, 2, 0] == 0.0
    # the same definition as the limiter's: vertices and mean above the margin
    Hv = np.einsum("em,im->ei", w[:, 0], T.phi_v) + s.hbv
    full = np.all(Hv > s.H_dry, axis=1) & (w[:, 0, 0] + s.hbar > s.H_dry)
    assert not full[e]
    assert np.array_equal(w2[full][:, :, 0], w[full][:, :, 0])
