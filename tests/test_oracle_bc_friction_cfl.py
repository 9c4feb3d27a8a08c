"""Pins of three oracle parts that the other tests leave free.

* Quadratic friction (Sec. 3.1: quadratic coefficient 0.001; reading A3,
  tau_b = C_f |u| / H): spatially uniform flow over a flat bed with
  transmissive boundaries has no flux divergence, so the discharge obeys
  the ODE dq/dt = -tau_b q, i.e. du/dt = -C_f u |u| / H at fixed H, whose
  solution is u(t) = u0 / (1 + C_f u0 t / H).  The scheme must reach it at
  second order in dt.
* River boundary (Sec. 2.1, Eq. river_bc; reading A4: the ghost normal
  discharge is 2 q_river - q_n, the mass flux is q_river).  Two identities
  fix the ghost: with q_river = 0 the river edge is a land edge (the ghost is
  the mirror image, Sec. 2.1 "zero normal flow"), and when the interior
  already carries q_n = q_river the ghost equals the interior state, so a
  uniform stream entering through a river edge is an exact steady state.
  A linear ghost a q_river + b q_n meets both only for a = 2, b = -1.
* CFL time step (Sec. 1, the CFL condition; reading A26): dt = CFL min_e
  d_e / lambda_e with lambda_e the largest |u| + sqrt(g H) over the wet
  vertices, |u| the speed (magnitude of the velocity vector), d_e the
  inscribed-circle diameter 4 area / perimeter.  Checked against a value
  worked out by hand on a two-triangle mesh.
"""
import math

import numpy as np

import meshgen
from oracle.solver import OracleSolver

G = 9.81


# ------------------------------------------------------------ friction
def _uniform_flow_quadratic(cf, H, u0, dt, steps):
    xy, tri, sides = meshgen.rect_grid(4, 2, 8000.0, 4000.0)
    be = np.concatenate(list(sides.values()))
    bt = np.full(len(be), meshgen.OUTFLOW)
    s = OracleSolver(xy, tri, np.full(len(xy), H), np.full(len(xy), cf), be, bt, np.zeros(len(be)),
                     friction="quadratic", dt_fixed=dt)
    s.set_initial_nodal(np.zeros(len(xy)), np.full(len(xy), H * u0), np.zeros(len(xy)))
    s.step(steps)
    return s.w[:, 1, 0] / H


def test_quadratic_friction_ode_second_order():
    # H = 2 m so that a wrong power of H (1/H^2, 1/H^(4/3)) changes the decay
    cf, H, u0, T = 0.01, 2.0, 1.5, 200.0
    exact = u0 / (1.0 + cf * u0 * T / H)         # 1.5 / (1 + 1.5) = 0.6 m/s
    assert abs(exact - 0.6) < 1e-15
    errs = []
    for k in (10, 20, 40):
        u = _uniform_flow_quadratic(cf, H, u0, T / k, k)
        assert np.ptp(u) < 1e-14                 # stays uniform
        errs.append(abs(u[0] - exact))
    assert errs[0] > errs[1] > errs[2]
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5, errs
    assert errs[2] < 2e-4


# --------------------------------------------------------------- river
def _channel(side_type, q_series, *, flux="llf"):
    """4 km x 2 km flat channel (8 x 4 quads, jittered), 10 m deep.  The left
    side gets ``side_type`` (slot 0: river series ``q_series``), the right
    side is transmissive, top and bottom are land."""
    rng = np.random.default_rng(17)
    xy, tri, sides = meshgen.rect_grid(8, 4, 4000.0, 2000.0, jitter=0.15, rng=rng)
    be, bt, bs = [], [], []
    for name, ty in (("bottom", meshgen.LAND), ("right", meshgen.OUTFLOW), ("top", meshgen.LAND),
                     ("left", side_type)):
        be.append(sides[name]); bt.append(np.full(len(sides[name]), ty)); bs.append(np.zeros(len(sides[name])))
    be, bt, bs = np.concatenate(be), np.concatenate(bt), np.concatenate(bs)
    rivers = {0: q_series} if side_type == meshgen.RIVER else {}
    s = OracleSolver(xy, tri, np.full(len(xy), 10.0), np.zeros(len(xy)), be, bt, bs, flux=flux,
                     friction="quadratic", dt_fixed=2.0, rivers=rivers)
    return s, xy


def test_river_with_zero_flux_is_a_land_boundary():
    """q_river = 0: the ghost is the mirror of the interior state, as on land."""
    for flux in ("llf", "roe"):
        out = []
        for ty in (meshgen.RIVER, meshgen.LAND):
            s, xy = _channel(ty, (np.array([0.0, 1e6]), np.array([0.0, 0.0])), flux=flux)
            # a surface bump and an oblique current toward the left wall
            z = 0.3 * np.exp(-((xy[:, 0] - 1000.0) ** 2 + (xy[:, 1] - 900.0) ** 2) / 600.0 ** 2)
            s.set_initial_nodal(z, -2.0 - 0.5 * np.sin(xy[:, 1] / 500.0), 0.8 * np.cos(xy[:, 0] / 700.0))
            s.step(25)
            out.append((s.w.copy(), s.mass_totals()))
        (wr, mr), (wl, ml) = out
        assert np.abs(wr - wl).max() <= 1e-13 * np.abs(wl).max(), flux
        # the river edges are where the flow meets the wall: the run is not trivial
        assert np.abs(wl[:, 1:, 0]).max() > 1.0
        for k in ("bnd_in", "bnd_out", "volume"):
            assert abs(mr[k] - ml[k]) <= 1e-13 * max(1.0, abs(ml[k])), (flux, k)


def test_uniform_inflow_through_a_river_edge_is_steady():
    """Interior q_n equal to q_river: the ghost equals the interior state, so
    the uniform stream (qx = q0, flat surface, no friction) is steady."""
    q0 = 3.0
    for flux in ("llf", "roe"):
        # outward normal of the left side is -x: inflow q0 is q_river = -q0
        s, xy = _channel(meshgen.RIVER, (np.array([0.0, 1e6]), np.array([-q0, -q0])), flux=flux)
        s.set_initial_nodal(np.zeros(len(xy)), np.full(len(xy), q0), np.zeros(len(xy)))
        L, (bo, bi) = s.rhs(s.w, 0.0, np.zeros(s.E), s.flags)
        scale = q0 * q0 / 10.0 + 0.5 * G * 10.0     # momentum flux of the stream
        assert np.abs(L).max() <= 1e-13 * scale / 500.0, (flux, np.abs(L).max())
        # inflow on the left, the same outflow on the right (2 km wide)
        assert abs(bi - 2000.0 * q0) < 1e-9 and abs(bo - 2000.0 * q0) < 1e-9
        s.step(20)
        vals = s.vertex_values()
        assert np.abs(vals[:, 1] - q0).max() < 1e-11 and np.abs(vals[:, 2]).max() < 1e-11
        assert np.abs(vals[:, 0]).max() < 1e-11


# ----------------------------------------------------------------- CFL
def test_cfl_time_step_worked_by_hand():
    """Unit square cut along its diagonal into two right triangles with legs
    of 1 m: area 1/2, perimeter 2 + sqrt(2), inscribed diameter
    d = 4 (1/2) / (2 + sqrt(2)) = 2 - sqrt(2) = 0.585786437627 m.
    Flat bed 1 m deep at nodes 0, 1 and 3, 4 m deep at node 2 (surface
    raised by 3 m there), velocity (3, 4) m/s everywhere (q = H (3, 4)), so
    |u| = 5 m/s at every vertex.  Both triangles contain node 2, where
    sqrt(g H) = sqrt(39.24) = 6.264183905346 m/s is the largest, so
    lambda = 11.264183905346 m/s and dt = 0.3 d / lambda =
    0.3 x 0.585786437627 / 11.264183905346 = 0.0156013017 s."""
    xy = np.array([[0.0, 0.0], [1.0, 0.0], [1.0, 1.0], [0.0, 1.0]])
    tri = np.array([[0, 1, 2], [0, 2, 3]])
    H = np.array([1.0, 1.0, 4.0, 1.0])
    s = OracleSolver(xy, tri, np.ones(4), np.zeros(4), cfl=0.3)
    s.set_initial_nodal(H - 1.0, 3.0 * H, 4.0 * H)
    assert abs(s.dt - 0.0156013017) < 1e-10, s.dt
    # the same state with the velocity turned by 90 degrees gives the same dt
    s.set_initial_nodal(H - 1.0, -4.0 * H, 3.0 * H)
    assert abs(s.dt - 0.0156013017) < 1e-10, s.dt
