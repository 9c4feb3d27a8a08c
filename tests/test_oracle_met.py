"""Pins of the wind and pressure forcing of the oracle (oracle.met).

* the vortex: the cyclostrophic Holland wind peaks at the radius of maximum
  wind with sqrt(B dp / (rho_a e)) (calculus on s exp(-s)), the pressure
  deficit is dp (1 - 1/e) there and dp at the centre, the circulation is
  counter-clockwise, and with dp = 0 only the background wind is left;
* the drag law at hand-computed speeds and its cap;
* two discrete equilibria in closed basins, where every term of the scheme
  is integrated exactly, so the right-hand side must vanish to round-off:
  - inverse barometer: flat bed, still water whose surface is -psi under a
    stationary pressure low (no wind): g H grad zeta = -g H grad psi;
  - wind set-up: uniform 10 m/s wind, free surface rising downwind with
    slope a = tau / (g H) over a bed rising with the same slope (so H is
    constant), tau = 1.15e-3 * 1.42e-3 * 10^2 m^2/s^2 worked out by hand;
  a wrong sign, a missing depth factor or a wrong stress magnitude leaves a
  residual of the order of the forcing itself;
* mass: wind and pressure move water but add none (closed basin).
"""
import numpy as np
import pytest

from meshgen.generators import Mesh, rect_grid, _bnd
from oracle import met
from oracle.solver import OracleSolver

G = 9.81


def test_vortex_peak_and_pressure():
    dp, rm, B = 4000.0, 30e3, 1.3
    r = np.linspace(0.2 * rm, 5.0 * rm, 200001)
    Wx, Wy, dpa = met.vortex(r, np.zeros_like(r), 0.0, 0.0, dp, rm, B, 1.0, 0.0, 0.0)
    V = np.hypot(Wx, Wy)
    k = int(np.argmax(V))
    assert abs(r[k] - rm) <= (r[1] - r[0])
    assert V[k] == pytest.approx(np.sqrt(B * dp / (met.RHO_AIR * np.e)), rel=1e-9)
    _, _, at_rm = met.vortex(rm, 0.0, 0.0, 0.0, dp, rm, B, 1.0, 0.0, 0.0)
    assert at_rm == pytest.approx(-dp * (1.0 - np.exp(-1.0)), rel=1e-14)
    wx0, wy0, at_c = met.vortex(0.0, 0.0, 0.0, 0.0, dp, rm, B, 1.0, 0.0, 0.0)
    assert at_c == -dp and wx0 == 0.0 and wy0 == 0.0


def test_vortex_turns_counter_clockwise():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(-1e5, 1e5, 50), rng.uniform(-1e5, 1e5, 50)
    xc, yc = 1e4, -2e4
    Wx, Wy, _ = met.vortex(x, y, xc, yc, 3000.0, 25e3, 1.5, 1.0, 0.0, 0.0)
    dx, dy = x - xc, y - yc
    speed = np.hypot(Wx, Wy)
    assert np.all(np.abs(dx * Wx + dy * Wy) <= 1e-12 * np.hypot(dx, dy) * speed)   # tangential
    assert np.all(dx * Wy - dy * Wx > 0.0)                                         # counter-clockwise
    Wx, Wy, dpa = met.vortex(x, y, xc, yc, 0.0, 25e3, 1.5, 1.0, 3.0, -4.0)
    assert np.all(Wx == 3.0) and np.all(Wy == -4.0) and np.all(dpa == 0.0)


def test_drag_law_values():
    assert met.drag_coefficient(10.0) == pytest.approx(1.42e-3, rel=1e-12)
    assert met.drag_coefficient(20.0) == pytest.approx(2.09e-3, rel=1e-12)
    assert met.drag_coefficient(0.0) == pytest.approx(0.75e-3, rel=1e-12)
    assert met.drag_coefficient(60.0) == pytest.approx(3.5e-3, rel=1e-12)


def _closed_basin(nx, ny, Lx, Ly, hb_fn):
    xy, tri, sides = rect_grid(nx, ny, Lx, Ly, jitter=0.15, rng=np.random.default_rng(5), diagonal="short")
    hb = hb_fn(xy[:, 0], xy[:, 1])
    be, bt, bs = _bnd(sides, {})                      # land on every side
    return Mesh(xy, tri, hb, np.full(len(hb), 0.025), be, bt, bs)


def _rhs(mesh, zeta, records, p=1, flux="llf"):
    s = OracleSolver(mesh.xy, mesh.tri, mesh.hb, mesh.fric, mesh.bedges, mesh.btype, mesh.bslot,
                     p=p, flux=flux, friction="manning", H0=0.01, met=records)
    z = np.zeros_like(zeta)
    s.set_initial_nodal(zeta, z, z)
    m = met.met_nodes(records, s.xy, 0.0, s.g)
    L, _ = s.rhs(s.w, 0.0, np.zeros(s.E), s.flags, m)
    return s, L, m


@pytest.mark.parametrize("flux", ["llf", "roe"])
def test_inverse_barometer_equilibrium(flux):
    mesh = _closed_basin(24, 24, 100e3, 100e3, lambda x, y: np.full_like(x, 20.0))
    rec = np.array([[0.0, 50e3, 45e3, 4000.0, 20e3, 1.5, 0.0, 0.0, 0.0]])
    _, _, psi = met.met_nodes(rec, mesh.xy, 0.0, G)
    s, L, m = _rhs(mesh, -psi, rec, flux=flux)
    scale = G * 20.0 * 4000.0 / (met.RHO_WATER * G * 20e3)          # g H |grad psi| near rm
    assert np.max(np.abs(psi)) > 0.3                                 # a 0.4 m bulge
    assert np.max(np.abs(L[:, 1:])) <= 1e-11 * scale
    # the same state with the pressure term's sign flipped is far from balance
    s2, L2, _ = _rhs(mesh, psi, rec, flux=flux)
    assert np.max(np.abs(L2[:, 1:])) > 0.5 * scale


@pytest.mark.parametrize("flux", ["llf", "roe"])
def test_wind_setup_equilibrium(flux):
    tau = 1.15e-3 * 1.42e-3 * 10.0 ** 2              # rho_a/rho_w C_d(10 m/s) |W| W, by hand
    h0, c = 10.0, -0.05
    H = h0 + c
    a = tau / (G * H)
    mesh = _closed_basin(20, 6, 100e3, 30e3, lambda x, y: h0 - a * x)
    zeta = a * mesh.xy[:, 0] + c                       # H = hb + zeta = h0 + c everywhere
    rec = np.array([[0.0, -1e9, 0.0, 0.0, 1e4, 1.0, 1.0, 10.0, 0.0]])
    s, L, m = _rhs(mesh, zeta, rec, flux=flux)
    assert m[0] == pytest.approx(np.full(len(zeta), tau), rel=1e-12)
    assert np.max(np.abs(L[:, 1:])) <= 1e-10 * tau / H
    # a 7 m/s wind (0.44 of the stress) over the same set-up is out of balance
    rec2 = rec.copy()
    rec2[0, 7] = 7.0
    _, L2, _ = _rhs(mesh, zeta, rec2, flux=flux)
    assert np.max(np.abs(L2[:, 1, 0])) > 0.2 * tau / H


def test_storm_moves_water_but_adds_none():
    mesh = _closed_basin(16, 16, 80e3, 80e3, lambda x, y: 15.0 + 5.0 * np.sin(x / 2e4) * np.cos(y / 3e4))
    rec = np.array([[0.0, 20e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0],
                    [4.0e3, 60e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0]])
    s = OracleSolver(mesh.xy, mesh.tri, mesh.hb, mesh.fric, mesh.bedges, mesh.btype, mesh.bslot,
                     p=1, flux="roe", friction="manning", H0=0.01, met=rec, cfl=0.3)
    z = np.zeros(len(mesh.hb))
    s.set_initial_nodal(z, z, z)
    v0 = s.volume()
    s.step(20)
    assert np.max(np.abs(s.w[:, 1:, 0])) > 1e-3                       # the storm has moved the water
    assert abs(s.volume() - v0) <= 1e-12 * v0
