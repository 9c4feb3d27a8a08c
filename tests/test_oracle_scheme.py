"""Scheme-level pins of the FP64 oracle.

* lake at rest with bumpy bathymetry: RHS identically zero (well-balancing,
  Sec. 3.1) for p = 1, 2 and both fluxes, and it stays at rest;
* SSP stability polynomials (closed forms);
* mass budget closes to round-off (rain, boundaries, wet/dry, limiter);
* friction ODE for uniform flow on a flat bed (closed form, order 2);
* manufactured solution: L2 convergence rates p + 1 (p = 1, 2, 3);
* p = 0 equals an independent first-order finite-volume code;
* the vectorised oracle equals the element-by-element loop version.
The bathtub experiment of Sec. 3.1 is in test_oracle_bathtub.py.
"""
import math

import numpy as np
import pytest

import meshgen
from oracle import basis, physics
from oracle.loop import LoopSolver
from oracle.solver import OracleSolver, from_scenario, ssp_step, ssp_table, ssp_flux_weights

G = 9.81


def _solver(sc, **kw):
    return from_scenario(sc, **kw)


@pytest.mark.parametrize("p,flux", [(1, "roe"), (1, "llf"), (2, "roe"), (2, "llf"), (3, "roe"), (3, "llf")])
def test_lake_at_rest_rhs_vanishes(p, flux):
    sc = meshgen.lake_at_rest(p=p, flux=flux)
    s = _solver(sc)
    L, (bo, bi) = s.rhs(s.w, 0.0, np.zeros(s.E), s.flags)
    scale = G * np.abs(sc.mesh.hb).max() * np.abs(s.dhb).max()
    assert np.abs(L).max() <= 1e-12 * scale
    assert abs(bo) + abs(bi) < 1e-9
    s.step(20)
    vals = s.vertex_values()
    assert np.abs(vals[:, 1:]).max() < 1e-11
    assert np.abs(vals[:, 0] - 0.7).max() < 1e-12


@pytest.mark.parametrize("stages", [2, 3, 5])
def test_ssp_stability_polynomials(stages):
    z = np.linspace(-2.5, 0.5, 31) + 0.3j
    amp = ssp_step(np.ones_like(z), lambda w, i: w * z, 1.0, ssp_table(stages))
    if stages == 2:
        ref = 1 + z + z ** 2 / 2
    elif stages == 3:
        ref = 1 + z + z ** 2 / 2 + z ** 3 / 6
    else:                                   # s-stage second order: ((s-1)/s)(1+z/(s-1))^s + 1/s
        ref = (4 / 5) * (1 + z / 4) ** 5 + 1 / 5
    np.testing.assert_allclose(amp, ref, rtol=1e-14, atol=1e-14)
    assert abs(sum(ssp_flux_weights(ssp_table(stages))) - 1.0) < 1e-15


@pytest.mark.parametrize("name", ["c1", "mixed_p1", "mixed_p2_lim", "mixed_nodal_llf", "basin"])
def test_mass_budget_closes(name):
    if name == "c1":
        sc, n = meshgen.channel_c1(), 300
    elif name == "mixed_p1":
        sc, n = meshgen.small_mixed(), 120
    elif name == "mixed_p2_lim":
        sc, n = meshgen.small_mixed(p=2, flux="llf", limiter=True, rain_kind="parametric"), 60
    elif name == "mixed_nodal_llf":
        sc, n = meshgen.small_mixed(flux="llf", limiter=True, rain_kind="nodal"), 120
    else:
        sc, n = meshgen.basin_window(24), 100
    s = _solver(sc)
    V0 = s.volume()
    s.step(n)
    m = s.mass_totals()
    assert m["rain_in"] > 0
    resid = m["volume"] - V0 - m["rain_in"] + m["bnd_out"] - m["bnd_in"]
    assert abs(resid) <= 1e-13 * m["volume"], resid / m["volume"]


def _uniform_flow(n, H=2.0, u0=1.0, dt=10.0, steps=20):
    xy, tri, sides = meshgen.rect_grid(4, 2, 8000.0, 4000.0)     # CFL number < 0.1 at dt = 20 s
    be = np.concatenate(list(sides.values()))
    bt = np.full(len(be), meshgen.OUTFLOW)
    hb = np.full(len(xy), H)
    s = OracleSolver(xy, tri, hb, np.full(len(xy), n), be, bt, np.zeros(len(be)), dt_fixed=dt)
    s.set_initial_nodal(np.zeros(len(xy)), np.full(len(xy), H * u0), np.full(len(xy), 0.0))
    s.step(steps)
    return s.w[:, 1, 0] / H


def test_friction_ode_second_order():
    n, H, u0, T = 0.03, 2.0, 1.0, 200.0
    exact = u0 / (1 + G * n * n * u0 * T / H ** (4 / 3))
    errs = []
    for k in (10, 20, 40):
        u = _uniform_flow(n, H, u0, dt=T / k, steps=k)
        assert np.ptp(u) < 1e-14          # stays uniform
        errs.append(abs(u[0] - exact))
    assert errs[0] > errs[1] > errs[2]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


class MMS:
    """zeta = A sin(kx - wt), qx = (A w / k) sin(kx - wt), qy = 0 on a flat bed
    of depth h0 without friction; continuity holds exactly (R = 0) and the
    x-momentum source is dqx/dt + d(qx^2/H)/dx + g H dzeta/dx."""

    def __init__(self, h0=10.0, A=0.05, L=1000.0):
        self.h0, self.A, self.k = h0, A, 2 * np.pi / L
        self.w = 0.5 * self.k * np.sqrt(G * h0)

    def exact(self, x, y, t):
        th = self.k * x - self.w * t
        z = self.A * np.sin(th)
        return np.stack([z, self.A * self.w / self.k * np.sin(th), 0 * z])

    def source(self, x, y, t):
        A, k, w = self.A, self.k, self.w
        th = k * x - w * t
        qx = A * w / k * np.sin(th)
        H = self.h0 + A * np.sin(th)
        c = np.cos(th)
        fx = -A * w * w / k * c + 2 * qx * A * w * c / H - qx * qx * A * k * c / H ** 2 + G * H * A * k * c
        return np.stack([0 * fx, fx, 0 * fx])

    def ghost(self, x, y, t):
        return self.exact(x, y, t)


def _project(s, fun, t):
    """L2 projection onto the element basis with a 6x6 collapsed Gauss rule."""
    a, wa = np.polynomial.legendre.leggauss(6)
    A, B = np.meshgrid(a, a)
    WA, WB = np.meshgrid(wa, wa)
    r = (0.5 * (1 + A) * (1 - B) - 1).ravel(); sr = B.ravel()
    wq = (WA * WB * 0.5 * (1 - B)).ravel()
    phi = basis.eval_basis(s.p, r, sr)[0]
    lam = np.array(basis.barycentric(r, sr))
    v = s.G["verts"]
    x = np.einsum("ei,iq->eq", v[..., 0], lam); y = np.einsum("ei,iq->eq", v[..., 1], lam)
    f = fun(x, y, t)                                           # (3, E, nq)
    return np.einsum("veq,q,mq->evm", f, wq, phi) / basis.mass_diag(s.p)[None, None, :], (x, y, wq, phi)


@pytest.mark.parametrize("p,rate", [(1, 1.8), (2, 2.7), (3, 3.6)])
def test_mms_convergence_rate(p, rate):
    mms = MMS()
    errs = []
    for nx in (6, 12, 24):
        xy, tri, sides = meshgen.rect_grid(nx, nx // 2, 1000.0, 500.0)
        be = np.concatenate(list(sides.values()))
        s = OracleSolver(xy, tri, np.full(len(xy), mms.h0), np.zeros(len(xy)), be,
                         np.full(len(be), meshgen.OCEAN), np.zeros(len(be)), p=p, flux="llf",
                         rk_stages=2 if p == 1 else 3, cfl=0.1, mms=mms)
        w0, _ = _project(s, mms.exact, 0.0)
        s.set_state(w0)
        Tend = 15.0
        while s.t < Tend - 1e-12:
            s.dt = min(s.dt, Tend - s.t)
            s.step(1)
        ref, (x, y, wq, phi) = _project(s, mms.exact, s.t)
        zh = np.einsum("em,mq->eq", s.w[:, 0], phi)
        ze = mms.exact(x, y, s.t)[0]
        errs.append(math.sqrt(np.sum(s.G["detJ"][:, None] * wq[None] * (zh - ze) ** 2)))
    r1, r2 = math.log2(errs[0] / errs[1]), math.log2(errs[1] / errs[2])
    assert r2 > rate and r1 > rate - 0.3, (errs, r1, r2)


def _fv_first_order(xy, tri, hb, w0, dt, steps, kind, H0=1e-3):
    """Independent cell-centred finite-volume code (wall boundaries)."""
    E = len(tri)
    edges = {}
    for e, t in enumerate(tri):
        for k in range(3):
            edges.setdefault(tuple(sorted((t[k], t[(k + 1) % 3]))), []).append((e, k))
    area = np.zeros(E); grad = np.zeros((E, 2))
    for e, (a, b, c) in enumerate(tri):
        (xa, ya), (xb, yb), (xc, yc) = xy[a], xy[b], xy[c]
        area[e] = 0.5 * ((xb - xa) * (yc - ya) - (yb - ya) * (xc - xa))
        # gradient of the linear interpolant of hb
        M = np.array([[xb - xa, yb - ya], [xc - xa, yc - ya]])
        grad[e] = np.linalg.solve(M, [hb[b] - hb[a], hb[c] - hb[a]])

    def rate(U):
        out = np.zeros_like(U)
        for (i, j), lst in edges.items():
            e, k = lst[0]
            t = tri[e]
            a, b = t[k], t[(k + 1) % 3]
            dx, dy = xy[b][0] - xy[a][0], xy[b][1] - xy[a][1]
            ell = math.hypot(dx, dy); nx, ny = dy / ell, -dx / ell
            hm = np.array([0.5 * (hb[a] + hb[b])])
            UL = U[e].reshape(3, 1)
            if len(lst) == 2:
                UR = U[lst[1][0]].reshape(3, 1)
            else:
                qn = UL[1] * nx + UL[2] * ny
                UR = np.array([UL[0], UL[1] - 2 * qn * nx, UL[2] - 2 * qn * ny])
            F = physics.numerical_flux(kind, UL, UR, hm, np.array([nx]), np.array([ny]), G, H0)[:, 0]
            out[e] -= ell * F
            if len(lst) == 2:
                out[lst[1][0]] += ell * F
        out[:, 1] += area * G * U[:, 0] * grad[:, 0]
        out[:, 2] += area * G * U[:, 0] * grad[:, 1]
        return out / area[:, None]

    U = w0.copy()
    for _ in range(steps):
        U1 = U + dt * rate(U)
        U = 0.5 * U + 0.5 * (U1 + dt * rate(U1))
    return U


@pytest.mark.parametrize("kind", ["roe", "llf"])
def test_p0_equals_finite_volume(kind):
    rng = np.random.default_rng(9)
    xy, tri, sides = meshgen.rect_grid(6, 4, 600.0, 400.0, jitter=0.2, rng=rng)
    be = np.concatenate(list(sides.values()))
    hb = 5.0 + 0.002 * xy[:, 0] + np.sin(xy[:, 1] / 90.0)
    s = OracleSolver(xy, tri, hb, np.zeros(len(xy)), be, np.zeros(len(be)), np.zeros(len(be)),
                     p=0, flux=kind, dt_fixed=0.5)
    w = np.zeros((s.E, 3, 1))
    w[:, 0, 0] = rng.uniform(-0.2, 0.2, s.E); w[:, 1:, 0] = rng.normal(0, 0.3, (s.E, 2))
    s.set_state(w)
    s.step(10)
    U = _fv_first_order(xy, s.tri, hb, w[:, :, 0], 0.5, 10, kind)
    np.testing.assert_allclose(s.w[:, :, 0], U, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("case", ["p1_roe", "p2_llf_lim", "p1_llf_lim_nodal", "p2_roe", "p3_llf_lim"])
def test_vectorised_equals_loop(case):
    kw = dict(p1_roe=dict(p=1, flux="roe", limiter=False, rain_kind="gridded"),
              p2_llf_lim=dict(p=2, flux="llf", limiter=True, rain_kind="parametric"),
              p1_llf_lim_nodal=dict(p=1, flux="llf", limiter=True, rain_kind="nodal"),
              p2_roe=dict(p=2, flux="roe", limiter=False, rain_kind="none"),
              p3_llf_lim=dict(p=3, flux="llf", limiter=True, rain_kind="gridded"))[case]
    sc = meshgen.small_mixed(seed=11, nx=8, ny=5, **kw)
    m = sc.mesh
    s = from_scenario(sc)
    s.step(3)                                   # a state with fronts, flags and flow
    lp = LoopSolver(m.xy, m.tri, m.hb, m.fric, m.bedges, m.btype, m.bslot, p=s.p, flux=s.flux_kind,
                    friction=s.friction, limiter=s.use_limiter, H0=s.H0, tides=sc.tides, rivers=sc.rivers)
    R = s.element_rain(s.t)
    L1, b1 = s.rhs(s.w, s.t, R, s.flags)
    L2, b2 = lp.rhs(s.w.tolist(), s.t, R.tolist(), list(s.flags))
    scale = np.abs(L1).max()
    np.testing.assert_allclose(np.array(L2), L1, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(b2, b1, rtol=1e-12, atol=1e-12)
    trial = s.w + 0.5 * s.dt * L1
    w1, f1 = s.post(trial)
    w2, f2 = lp.post(trial.tolist())
    np.testing.assert_allclose(np.array(w2), w1, rtol=0, atol=1e-12 * np.abs(w1).max())
    assert list(f1) == list(f2)
    assert s.flags.any() and (~s.flags).any()
