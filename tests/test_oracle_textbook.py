"""The oracle against textbook solutions of the shallow water equations.

* Stoker's wet-bed dam break: the middle state (h_m, u_m) solves the
  rarefaction (Riemann invariant) and shock (Rankine-Hugoniot) relations,
  the shock moves at h_m u_m / (h_m - h_r).  Checked: the plateau depth, the
  shock position, and an L1 error that falls at about first order.
* Ritter's dry-bed dam break: h = (2 c_0 - x/t)^2 / (9 g) between -c_0 t and
  the front 2 c_0 t.  The thin-layer front lags the exact one by a distance
  that shrinks with the mesh; the volume is exact.
* Rain on the inclined plane of Sec. 3.2, condition (A): away from the ends
  the flow is uniform along the plane, so H = R t exactly and the discharge
  obeys the ODE dq/dt = g H S - g n^2 |q| q / H^(7/3) (gravity along the bed
  slope against Manning friction, the source terms of Eq. SWE).  At
  equilibrium the outflow per unit width is R L (mass conservation).
The exact solutions here are computed from these formulas with SciPy; none
of the oracle's code is used to produce them.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

import meshgen
from oracle.solver import from_scenario

G = 9.81


def stoker_star(hl, hr):
    cl = np.sqrt(G * hl)
    f = lambda hm: 2.0 * (cl - np.sqrt(G * hm)) - (hm - hr) * np.sqrt(0.5 * G * (hm + hr) / (hm * hr))  # noqa: E731
    hm = brentq(f, hr, hl, xtol=1e-15)
    um = 2.0 * (cl - np.sqrt(G * hm))
    return hm, um, hm * um / (hm - hr)


def dam_break_run(nx, hl, hr, T, ny=1, limiter=True):
    L = 200.0
    sc = meshgen.dam_break(nx, h_left=hl, h_right=hr, L=L, W=ny * L / nx, ny=ny, limiter=limiter)
    o = from_scenario(sc)
    xc = sc.mesh.xy[sc.mesh.tri, 0].mean(axis=1)
    w = np.zeros_like(o.w)
    w[:, 0, 0] = np.where(xc < 0.0, hl, hr)
    o.set_state(w)
    while o.t < T - 1e-12:
        o.dt = min(o.dt, T - o.t)
        o.step(1)
    return xc, o.w[:, 0, 0].copy(), o, L / nx


def test_stoker_wet_bed_dam_break():
    hl, hr, T = 2.0, 1.0, 10.0
    hm, um, s = stoker_star(hl, hr)
    cl, cm = np.sqrt(G * hl), np.sqrt(G * hm)
    errs = []
    for nx in (100, 200, 400):
        xc, m, o, dx = dam_break_run(nx, hl, hr, T)
        xi = xc / o.t
        exact = np.where(xi < -cl, hl, np.where(xi < um - cm, (2 * cl - xi) ** 2 / (9 * G),
                                                np.where(xi < s, hm, hr)))
        errs.append(np.abs(m - exact).sum() * dx / 2)          # two triangles per dx
        plateau = m[(xc > (um - cm) * T + 5.0) & (xc < s * T - 5.0)].mean()
        assert abs(plateau - hm) < 2e-4 * hm, (nx, plateau, hm)
        shock = xc[m > 0.5 * (hm + hr)].max()
        assert abs(shock - s * T) <= dx, (nx, shock, s * T)
    assert errs[1] < errs[0] / 1.4 and errs[2] < errs[1] / 1.4, errs


def test_stoker_dam_break_exercises_the_limiter():
    """Stoker's dam break on a strip two quads wide, so that half the
    triangles have no wall edge and the slope limiter (Sec. 2.3) acts on
    them.  With the limiter the element means stay within 1.5e-2 below h_r
    and 2e-3 above h_l (the overshoot of an unlimited p = 1 run is about
    four times larger, which the same run checks), the plateau holds h_m to
    1e-5, the shock sits within one cell of the exact one and the L1 error
    halves with the mesh."""
    hl, hr, T = 2.0, 1.0, 10.0
    hm, um, s = stoker_star(hl, hr)
    cl, cm = np.sqrt(G * hl), np.sqrt(G * hm)
    errs = []
    for nx in (100, 200):
        xc, m, o, dx = dam_break_run(nx, hl, hr, T, ny=2)
        xi = xc / o.t
        exact = np.where(xi < -cl, hl, np.where(xi < um - cm, (2 * cl - xi) ** 2 / (9 * G),
                                                np.where(xi < s, hm, hr)))
        errs.append(np.abs(m - exact).sum() * dx / 4)           # four triangles per dx
        assert m.min() >= hr - 1.5e-2 and m.max() <= hl + 2e-3, (nx, m.min(), m.max())
        plateau = m[(xc > (um - cm) * T + 5.0) & (xc < s * T - 5.0)].mean()
        assert abs(plateau - hm) < 1e-5 * hm, (nx, plateau, hm)
        shock = xc[m > 0.5 * (hm + hr)].max()
        assert abs(shock - s * T) <= dx, (nx, shock, s * T)
    assert errs[1] < errs[0] / 1.8, errs
    _, m_free, _, _ = dam_break_run(200, hl, hr, T, ny=2, limiter=False)
    assert m_free.min() < hr - 3e-2 or m_free.max() > hl + 1e-2, (m_free.min(), m_free.max())


def test_ritter_dry_bed_dam_break():
    h0, T = 1.0, 6.0
    c0 = np.sqrt(G * h0)
    errs, lags = [], []
    for nx in (100, 200, 400):
        xc, m, o, dx = dam_break_run(nx, h0, 0.0, T)
        xi = xc / o.t
        exact = np.where(xi < -c0, h0, np.where(xi < 2 * c0, (2 * c0 - xi) ** 2 / (9 * G), 0.0))
        errs.append(np.abs(m - exact).sum() * dx / 2)
        # where the exact depth is 1 cm
        x_exact = T * (2 * c0 - 3 * np.sqrt(G * 0.01))
        lags.append(x_exact - xc[m > 0.01].max())
        assert abs(o.volume() - h0 * 100.0 * dx) < 1e-12 * h0 * 100.0 * dx
        assert m.min() >= 0.0
    assert errs[1] < errs[0] / 1.4 and errs[2] < errs[1] / 1.4, errs
    assert lags[0] > lags[1] > lags[2] > 0.0 and lags[2] < 2.0, lags


def test_inclined_plane_condition_a():
    S, n, R, Lp, W = 0.015, 0.009, 8.33e-4, 24.0, 0.196
    sc = meshgen.inclined_plane(96, L=Lp, W=W, slope=S, rain=R, manning=n)
    o = from_scenario(sc)
    xc = sc.mesh.xy[sc.mesh.tri, 0].mean(axis=1)
    hbm = sc.mesh.hb[sc.mesh.tri].mean(axis=1)
    mid = (xc > 11.0) & (xc < 13.0)

    def rhs(t, y):
        h = R * t
        return [G * h * S - G * n * n * abs(y[0]) * y[0] / h ** (7.0 / 3.0)]
    t0 = 0.05                      # start on the friction-dominated branch
    ode = solve_ivp(rhs, (t0, 20.0), [np.sqrt(S) / n * (R * t0) ** (5.0 / 3.0)], method="Radau",
                    rtol=1e-10, atol=1e-14, dense_output=True)
    for T, qtol in ((5.0, 1e-4), (10.0, 1e-5), (15.0, 1e-5)):
        while o.t < T - 1e-12:
            o.dt = min(o.dt, T - o.t)
            o.step(1)
        H = o.w[mid, 0, 0] + hbm[mid]
        assert np.abs(H / (R * T) - 1.0).max() < 1e-7, T
        q = o.w[mid, 1, 0]
        assert np.abs(q / ode.sol(T)[0] - 1.0).max() < qtol, (T, q.mean(), ode.sol(T)[0])
        assert np.abs(o.w[mid, 2, 0]).max() < 1e-6 * np.abs(q).max()     # nothing across the flume
    while o.t < 40.0 - 1e-12:
        o.dt = min(o.dt, 40.0 - o.t)
        o.step(1)
    b0, t1 = o.bnd_out, o.t
    o.step(5)
    q_out = (o.bnd_out - b0) / (o.t - t1) / W
    assert abs(q_out / (R * Lp) - 1.0) < 5e-3, q_out
