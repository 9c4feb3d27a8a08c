"""Seeded generators for meshes, bathymetry and forcing (no solver arithmetic).

Every generator returns plain NumPy arrays wrapped in the two dataclasses
below.  Seeds follow one rule: workload ``c`` uses ``23070 + c``; member
``i`` of an ensemble uses ``(23070 + c) * 1000 + i`` (see :func:`seed_for`).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

# Boundary partition of the domain (Sec. 2.1): ocean = specified elevation,
# land = zero normal flow, river = specified normal flux (Eq. river_bc);
# OUTFLOW is a transmissive boundary used by the channel workload.
LAND, OCEAN, RIVER, OUTFLOW = 0, 1, 2, 3

MM_PER_HOUR = 1.0 / 3.6e6  # (mm/h) -> (m/s)


def seed_for(config_id: int, member: Optional[int] = None) -> int:
    base = 2307 * 10 + int(config_id)
    return base if member is None else base * 1000 + int(member)


@dataclass
class Mesh:
    xy: np.ndarray          # (n, 2) float64 node coordinates [m]
    tri: np.ndarray         # (m, 3) int32 node ids (0-based)
    hb: np.ndarray          # (n,) float64 bathymetry, positive downward [m]
    fric: np.ndarray        # (n,) float64 Manning n or quadratic C_f
    bedges: np.ndarray      # (nb, 2) int32 boundary edge node pairs
    btype: np.ndarray       # (nb,) int32 LAND/OCEAN/RIVER/OUTFLOW
    bslot: np.ndarray       # (nb,) int32 forcing slot (tide / river series)

    @property
    def n_nodes(self) -> int:
        return int(self.xy.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


@dataclass
class Scenario:
    name: str
    mesh: Mesh
    zeta0: np.ndarray       # (n,) initial nodal free surface [m]
    qx0: np.ndarray         # (n,) initial nodal discharge [m^2/s]
    qy0: np.ndarray
    params: Dict[str, object]
    rain: Dict[str, object] = field(default_factory=lambda: {"kind": "none"})
    # slot -> (mean level, (k,3) rows of amplitude, period, phase): mean + sum a sin(2 pi t/T + phase)
    tides: Dict[int, Tuple[float, np.ndarray]] = field(default_factory=dict)
    rivers: Dict[int, Tuple[np.ndarray, np.ndarray]] = field(default_factory=dict)  # slot -> (t, q)
    n_steps: int = 0
    # storm wind and pressure records (t, xc, yc, dp, rm, B, wf, wbx, wby), or None
    met: Optional[np.ndarray] = None


def default_params(**kw) -> Dict[str, object]:
    """Solver settings; p = 2 defaults to three SSP stages at CFL 0.15,
    p = 3 to three stages at CFL 0.1."""
    p = dict(p=1, flux="roe", friction="manning", limiter=False, cfl=0.3,
             dt_fixed=0.0, dt_max=1.0e30, H0=1.0e-3, g=9.81, rk_stages=2)
    if kw.get("p", 1) == 2:
        p.update(rk_stages=3, cfl=0.15)
    if kw.get("p", 1) == 3:
        p.update(rk_stages=3, cfl=0.1)
    p.update(kw)
    return p


# ---------------------------------------------------------------------------
# structured / jittered triangulations of a rectangle
# ---------------------------------------------------------------------------
def rect_grid(nx: int, ny: int, Lx: float, Ly: float, *, x0: float = 0.0,
              y0: float = 0.0, jitter: float = 0.0,
              rng: Optional[np.random.Generator] = None,
              diagonal: str = "ne"):
    """Rectangle split into nx*ny quads, each cut into two CCW triangles.

    ``diagonal='ne'`` cuts every quad along (i,j)->(i+1,j+1); ``'short'``
    cuts along the shorter diagonal after jittering.  Interior nodes are moved
    by U(-jitter*dx, +jitter*dx) in each direction.  Returns
    ``xy, tri, sides`` where ``sides`` maps bottom/right/top/left to (k,2)
    node-pair arrays in boundary order.
    """
    dx, dy = Lx / nx, Ly / ny
    ii, jj = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1))
    x = x0 + ii.astype(np.float64) * dx
    y = y0 + jj.astype(np.float64) * dy
    if jitter > 0.0:
        rng = rng if rng is not None else np.random.default_rng(0)
        jx = rng.uniform(-jitter * dx, jitter * dx, size=x.shape)
        jy = rng.uniform(-jitter * dy, jitter * dy, size=y.shape)
        inner = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny)
        x = np.where(inner, x + jx, x)
        y = np.where(inner, y + jy, y)
    xy = np.stack([x.ravel(), y.ravel()], axis=1)
    nid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    ci, cj = np.meshgrid(np.arange(nx), np.arange(ny))
    ci, cj = ci.ravel(), cj.ravel()
    n00, n10 = nid(ci, cj), nid(ci + 1, cj)
    n11, n01 = nid(ci + 1, cj + 1), nid(ci, cj + 1)
    if diagonal == "ne":
        use_ne = np.ones(ci.shape, dtype=bool)
    elif diagonal == "short":
        d_ne = np.sum((xy[n11] - xy[n00]) ** 2, axis=1)
        d_nw = np.sum((xy[n01] - xy[n10]) ** 2, axis=1)
        use_ne = d_ne <= d_nw
    else:
        raise ValueError(diagonal)
    t1 = np.where(use_ne[:, None], np.stack([n00, n10, n11], 1), np.stack([n00, n10, n01], 1))
    t2 = np.where(use_ne[:, None], np.stack([n00, n11, n01], 1), np.stack([n10, n11, n01], 1))
    tri = np.empty((2 * ci.size, 3), dtype=np.int32)
    tri[0::2] = t1
    tri[1::2] = t2
    i = np.arange(nx)
    j = np.arange(ny)
    sides = {
        "bottom": np.stack([nid(i, 0), nid(i + 1, 0)], 1).astype(np.int32),
        "right": np.stack([nid(nx, j), nid(nx, j + 1)], 1).astype(np.int32),
        "top": np.stack([nid(i + 1, ny), nid(i, ny)], 1).astype(np.int32),
        "left": np.stack([nid(0, j + 1), nid(0, j)], 1).astype(np.int32),
    }
    return xy, tri, sides


def _bnd(sides, types: Dict[str, Tuple[int, int]]):
    be, bt, bs = [], [], []
    for name in ("bottom", "right", "top", "left"):
        t, s = types.get(name, (LAND, 0))
        be.append(sides[name])
        bt.append(np.full(len(sides[name]), t, np.int32))
        bs.append(np.full(len(sides[name]), s, np.int32))
    return (np.concatenate(be).astype(np.int32), np.concatenate(bt),
            np.concatenate(bs))


# ---------------------------------------------------------------------------
# workload 0: rain on a sloping channel (stand-in for the inclined plane)
# ---------------------------------------------------------------------------
def channel_c1(nx: int = 64, ny: int = 8) -> Scenario:
    """100 m x 10 m channel, bed slope 0.001 falling toward x = 100 m.

    64 x 8 rectangles cut along the NE diagonal (1,024 triangles, 585 nodes);
    walls at y = 0, y = 10 m and x = 0, free outflow at x = 100 m; Manning
    n = 0.02; uniform rain 100 mm/h; initial depth 0.01 m, at rest; Roe flux,
    no limiter, SSP-RK2 at CFL 0.3 for 1000 steps.
    """
    xy, tri, sides = rect_grid(nx, ny, 100.0, 10.0)
    zb = 0.001 * (100.0 - xy[:, 0])          # bed elevation (up)
    hb = -zb                                  # positive downward
    be, bt, bs = _bnd(sides, {"right": (OUTFLOW, 0)})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.02), be, bt, bs)
    depth0 = 0.01
    zeta0 = depth0 - hb
    rain = 100.0 * MM_PER_HOUR
    return Scenario("channel_c1", mesh, zeta0, np.zeros_like(hb), np.zeros_like(hb),
                    default_params(flux="roe", friction="manning", limiter=False, cfl=0.3),
                    rain={"kind": "nodal", "r": np.full(len(hb), rain)}, n_steps=1000)


# ---------------------------------------------------------------------------
# Sec. 3.1: filling a "bathtub"
# ---------------------------------------------------------------------------
def bathtub() -> Scenario:
    """(0,50 km) x (0,8 km), 25 x 4 rectangles -> 200 triangles; walls.

    The printed bump exp(-100 (x-25000)^2) cannot be seen by nodes spaced
    2 km apart, so x is measured in units of the domain length:
    hb = 5 - exp(-100 ((x - 25000)/50000)^2).  Quadratic friction 0.001,
    dt = 5 s, rain 7.0556e-6 m/s for 24 h followed by 48 h without forcing.
    """
    xy, tri, sides = rect_grid(25, 4, 50000.0, 8000.0)
    hb = 5.0 - np.exp(-100.0 * ((xy[:, 0] - 25000.0) / 50000.0) ** 2)
    be, bt, bs = _bnd(sides, {})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.001), be, bt, bs)
    z = np.zeros(len(hb))
    return Scenario("bathtub", mesh, z.copy(), z.copy(), z.copy(),
                    default_params(flux="roe", friction="quadratic", limiter=False, dt_fixed=5.0),
                    rain={"kind": "nodal", "r": np.full(len(hb), 7.0556e-6),
                          "until": 86400.0}, n_steps=51840)


# ---------------------------------------------------------------------------
# workload 1 and its scaled versions: jittered basin with a shelf and a coast
# ---------------------------------------------------------------------------
def basin_bathymetry(x, y, rng, L=200e3):
    """Shelf profile of the 200 km basin: -3000 m ocean, tanh shelf centred at
    x = 150 km (width 10 km) rising to +20 m land, plus 32 seeded Gaussian
    bumps (a ~ U(-500, 500) m, sigma ~ U(3, 15) km); clipped to [-3000, 20].
    Lengths scale with L / 200 km."""
    s = L / 200e3
    zb = -3000.0 + 3020.0 * (1.0 + np.tanh((x - 150e3 * s) / (10e3 * s))) / 2.0
    a = rng.uniform(-500.0, 500.0, 32)
    sig = rng.uniform(3e3, 15e3, 32) * s
    cx = rng.uniform(0.0, L, 32)
    cy = rng.uniform(0.0, L, 32)
    for k in range(32):
        zb = zb + a[k] * np.exp(-((x - cx[k]) ** 2 + (y - cy[k]) ** 2) / (2.0 * sig[k] ** 2))
    return np.clip(zb, -3000.0, 20.0)


def parametric_track(x_start, y_start, vx, vy, peak, t_end=1.0e6, *,
                     rm=30e3, re=100e3, t0_frac=0.5, n_rec=2):
    """Storm records (t, xc, yc, peak, T0, rm, re) on a straight track.

    Rates in m/s; the centre moves with (vx, vy).  Records are spaced
    evenly over [0, t_end] so that linear interpolation reproduces the
    straight track exactly.
    """
    t = np.linspace(0.0, t_end, n_rec)
    rec = np.zeros((n_rec, 7))
    rec[:, 0] = t
    rec[:, 1] = x_start + vx * t
    rec[:, 2] = y_start + vy * t
    rec[:, 3] = peak
    rec[:, 4] = t0_frac * peak
    rec[:, 5] = rm
    rec[:, 6] = re
    return rec


def vortex_track(x_start, y_start, vx, vy, dp, t_end=1.0e6, *, rm=30e3, B=1.3, wf=1.0,
                 wb=(0.0, 0.0), n_rec=2):
    """Wind and pressure records (t, xc, yc, dp, rm, B, wf, wbx, wby) on a
    straight track: central pressure deficit dp (Pa), radius of maximum
    wind rm (m), shape B, factor wf on the vortex wind and a uniform
    background wind wb (m/s)."""
    t = np.linspace(0.0, t_end, n_rec)
    rec = np.zeros((n_rec, 9))
    rec[:, 0] = t
    rec[:, 1] = x_start + vx * t
    rec[:, 2] = y_start + vy * t
    rec[:, 3] = dp
    rec[:, 4] = rm
    rec[:, 5] = B
    rec[:, 6] = wf
    rec[:, 7] = wb[0]
    rec[:, 8] = wb[1]
    return rec


def basin(N: int = 708, seed: int = seed_for(1), *, L: float = 200e3,
          window=None, jitter: float = 0.2, flux: str = "llf", limiter: bool = True,
          peak_mmh: float = 50.0, track=None, n_steps: int = 5000, p: int = 1,
          wind: bool = False) -> Scenario:
    """Jittered N x N grid cut along the shorter diagonals.

    Without ``window`` the grid covers the whole L x L basin: N = 708 gives
    1,002,528 triangles.  With ``window=(x0, y0, size)`` it covers that
    square of the same basin (same bathymetry and storm), which keeps the
    element size of the full workload on a smaller mesh.  Bathymetry: see
    :func:`basin_bathymetry`; dry land starts with zero depth.  Ocean
    boundary (zero elevation, slot 0) on the west side, land elsewhere,
    Manning 0.025, parametric rain (peak 50 mm/h, r_m = 30 km,
    r_e = 100 km) whose centre starts at (0.3 L, 0.5 L) and moves east at
    5 m/s.  ``wind=True`` adds the storm's wind and pressure on the same
    track: pressure deficit 4,000 Pa, radius of maximum wind 30 km (scaled
    with L), B = 1.3 (peak wind 40 m/s).
    """
    rng = np.random.default_rng(seed)
    x0, y0, size = (0.0, 0.0, L) if window is None else window
    xy, tri, sides = rect_grid(N, N, size, size, x0=x0, y0=y0, jitter=jitter, rng=rng,
                               diagonal="short")
    zb = basin_bathymetry(xy[:, 0], xy[:, 1], np.random.default_rng(seed + 1), L)
    hb = -zb
    be, bt, bs = _bnd(sides, {"left": (OCEAN, 0)})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.025), be, bt, bs)
    zeta0 = np.maximum(0.0, -hb)
    peak = peak_mmh * MM_PER_HOUR
    if track is None:
        track = parametric_track(0.3 * L, 0.5 * L, 5.0, 0.0, peak,
                                 rm=30e3 * L / 200e3, re=100e3 * L / 200e3)
    met = vortex_track(0.3 * L, 0.5 * L, 5.0, 0.0, 4000.0, rm=30e3 * L / 200e3) if wind else None
    return Scenario(f"basin_{N}", mesh, zeta0, np.zeros_like(hb), np.zeros_like(hb),
                    default_params(p=p, flux=flux, friction="manning", limiter=limiter, H0=0.05),
                    rain={"kind": "parametric", "records": track},
                    tides={0: (0.0, np.zeros((0, 3)))}, n_steps=n_steps, met=met)


def basin_window(N: int, seed: int = seed_for(1), **kw) -> Scenario:
    """N x N piece of the 200 km basin at its own element size (282.5 m),
    placed across the coast (x from 160 km)."""
    size = N * 200e3 / 708
    return basin(N, seed, window=(160e3, 100e3 - 0.5 * size, size), **kw)


# ---------------------------------------------------------------------------
# small mixed-boundary scenario for parity tests
# ---------------------------------------------------------------------------
def gridded_field(rng, x0, y0, dx, dy, nx, ny, n_rec, dt_rec, *, n_cells=6,
                  peak_range=(20.0, 100.0), radius_range=(0.2, 0.5), drift=(5.0, 0.0)):
    """Smooth seeded rain lattice (n_rec, ny, nx), float32, m/s.

    Gaussian rain cells drifting with ``drift`` m/s between hourly-type
    records; values clipped to [0, 100] mm/h.
    """
    Lx, Ly = dx * (nx - 1), dy * (ny - 1)
    cx = rng.uniform(x0, x0 + Lx, n_cells)
    cy = rng.uniform(y0, y0 + Ly, n_cells)
    pk = rng.uniform(*peak_range, n_cells)
    rad = rng.uniform(*radius_range, n_cells) * max(Lx, Ly)
    gx = x0 + dx * np.arange(nx)
    gy = y0 + dy * np.arange(ny)
    X, Y = np.meshgrid(gx, gy)
    vals = np.zeros((n_rec, ny, nx), dtype=np.float64)
    for r in range(n_rec):
        sx, sy = drift[0] * r * dt_rec, drift[1] * r * dt_rec
        f = np.zeros_like(X)
        for k in range(n_cells):
            f += pk[k] * np.exp(-((X - cx[k] - sx) ** 2 + (Y - cy[k] - sy) ** 2) / (2 * rad[k] ** 2))
        vals[r] = np.clip(f, 0.0, 100.0)
    t_rec = dt_rec * np.arange(n_rec, dtype=np.float64)
    return dict(kind="gridded", x0=x0, y0=y0, dx=dx, dy=dy, nx=nx, ny=ny,
                t_rec=t_rec, vals=(vals * MM_PER_HOUR).astype(np.float32))


def small_mixed(seed: int = 7, nx: int = 24, ny: int = 12, *, p: int = 1,
                flux: str = "roe", limiter: bool = False, friction: str = "manning",
                rain_kind: str = "gridded", dry_island: bool = True,
                dt_fixed: float = 0.0, wind: bool = False) -> Scenario:
    """10 km x 5 km jittered basin touching every boundary type.

    Left side: OCEAN (slot 0, two tidal constituents).  Right side: lower
    half RIVER (slot 1, inflow series), the two top edges OUTFLOW, LAND in
    between.  Top and bottom: LAND.  The bed deepens seaward with bumps and an island that rises
    above the surface, so wet/dry fronts exist from the start.  ``wind``
    adds a storm vortex (pressure deficit 3,000 Pa, radius of maximum wind
    2 km, B = 1.4, peak wind 37 m/s) crossing the basin at (4, 2) m/s over a
    (3, -1) m/s background wind.
    """
    rng = np.random.default_rng(seed)
    Lx, Ly = 10e3, 5e3
    xy, tri, sides = rect_grid(nx, ny, Lx, Ly, jitter=0.25, rng=rng, diagonal="short")
    x, y = xy[:, 0], xy[:, 1]
    hb = 12.0 - 10.0 * x / Lx + 1.5 * np.sin(2 * np.pi * y / Ly) * np.cos(np.pi * x / Lx)
    if dry_island:
        hb = hb - 14.0 * np.exp(-(((x - 0.55 * Lx) / (0.12 * Lx)) ** 2 + ((y - 0.5 * Ly) / (0.18 * Ly)) ** 2))
    right = sides["right"]
    ymid = 0.5 * (xy[right[:, 0], 1] + xy[right[:, 1], 1])
    be, bt, bs = [], [], []
    for name in ("bottom", "top"):
        be.append(sides[name]); bt.append(np.full(len(sides[name]), LAND)); bs.append(np.zeros(len(sides[name])))
    be.append(sides["left"]); bt.append(np.full(len(sides["left"]), OCEAN)); bs.append(np.zeros(len(sides["left"])))
    low = ymid < 0.5 * Ly
    top = ymid > Ly - 2.5 * Ly / ny
    be.append(right); bt.append(np.where(low, RIVER, np.where(top, OUTFLOW, LAND)))
    bs.append(np.where(low, 1, 0))
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.03 if friction == "manning" else 0.002),
                np.concatenate(be).astype(np.int32), np.concatenate(bt).astype(np.int32),
                np.concatenate(bs).astype(np.int32))
    zeta0 = np.maximum(0.05 * np.cos(np.pi * y / Ly), -hb)     # dry where the bed is above
    qx0 = np.where(hb + zeta0 > 0.5, 0.02 * np.sin(np.pi * y / Ly), 0.0)
    qy0 = np.where(hb + zeta0 > 0.5, -0.01 * np.cos(np.pi * x / Lx), 0.0)
    if rain_kind == "gridded":
        rain = gridded_field(rng, -500.0, -500.0, 1000.0, 1000.0, 12, 7, 4, 600.0)
    elif rain_kind == "parametric":
        rain = {"kind": "parametric",
                "records": parametric_track(2e3, 1e3, 3.0, 1.5, 60 * MM_PER_HOUR, 2e4,
                                            rm=1.5e3, re=4e3, n_rec=3)}
    elif rain_kind == "nodal":
        rain = {"kind": "nodal", "r": rng.uniform(0, 80, len(hb)) * MM_PER_HOUR}
    else:
        rain = {"kind": "none"}
    tides = {0: (0.02, np.array([[0.30, 44712.0, 0.3], [0.10, 43200.0, 1.1]]))}
    rivers = {1: (np.array([0.0, 120.0, 600.0, 3600.0]), np.array([-0.2, -0.8, -1.5, -0.5]))}
    met = (vortex_track(-2e3, 1e3, 4.0, 2.0, 3000.0, 2e4, rm=2e3, B=1.4, wb=(3.0, -1.0), n_rec=3)
           if wind else None)
    return Scenario(f"small_mixed_{seed}", mesh, zeta0, qx0, qy0,
                    default_params(p=p, flux=flux, friction=friction, limiter=limiter,
                                   dt_fixed=dt_fixed, H0=0.05),
                    rain=rain, tides=tides, rivers=rivers, n_steps=200, met=met)


def lake_at_rest(seed: int = 3, nx: int = 16, ny: int = 10, level: float = 0.7,
                 p: int = 1, flux: str = "roe") -> Scenario:
    """Jittered rectangle with a bumpy, fully submerged bed and a flat surface."""
    rng = np.random.default_rng(seed)
    xy, tri, sides = rect_grid(nx, ny, 4000.0, 2500.0, jitter=0.25, rng=rng, diagonal="short")
    x, y = xy[:, 0], xy[:, 1]
    hb = 6.0 + 3.0 * np.sin(x / 600.0) * np.cos(y / 450.0) + 0.001 * x
    be, bt, bs = _bnd(sides, {"left": (OCEAN, 0)})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.025), be, bt, bs)
    zeta0 = np.full(len(hb), level)
    return Scenario("lake_at_rest", mesh, zeta0, np.zeros_like(hb), np.zeros_like(hb),
                    default_params(p=p, flux=flux, friction="manning", limiter=False),
                    tides={0: (level, np.zeros((0, 3)))})


# ---------------------------------------------------------------------------
# textbook checks: dam breaks on a strip, rain on an inclined plane
# ---------------------------------------------------------------------------
def dam_break(nx: int = 200, *, h_left: float = 2.0, h_right: float = 1.0, L: float = 200.0,
              W: float = 2.0, H0: float = 1e-3, limiter: bool = True, ny: int = 1) -> Scenario:
    """Quasi-1D strip x in (-L/2, L/2), nx x ny quads, flat bed at the datum
    (hb = 0), walls all round, fluid at rest with depth h_left for x < 0 and
    h_right for x > 0 (h_right = 0 is a dry bed).  No friction, no rain.
    The nodal zeta0 puts the nodes on x = 0 on the right; a piecewise
    constant start (element means h_left / h_right, the dam on the quad
    boundary at x = 0 for even nx) is set from the element centroids."""
    xy, tri, sides = rect_grid(nx, ny, L, W, x0=-L / 2)
    be, bt, bs = _bnd(sides, {})
    hb = np.zeros(len(xy))
    mesh = Mesh(xy, tri, hb, np.zeros(len(hb)), be, bt, bs)
    # node values are set so that each element holds one side's depth: the
    # dam sits on the quad boundary at x = 0 (nx even)
    zeta0 = np.where(xy[:, 0] < 0.0, h_left, h_right).astype(np.float64)
    sc = Scenario("dam_break", mesh, zeta0, np.zeros(len(hb)), np.zeros(len(hb)),
                  default_params(flux="roe", friction="manning", limiter=limiter, cfl=0.3, H0=H0),
                  n_steps=0)
    return sc


def inclined_plane(nx: int = 96, *, L: float = 24.0, W: float = 0.196, slope: float = 0.015,
                   rain: float = 8.33e-4, manning: float = 0.009, H0: float = 1e-4) -> Scenario:
    """Rain on an initially dry plane (Sec. 3.2, condition (A)): a 24 m flume
    of width 0.196 m at sin(theta) = 0.015, uniform rain 0.0833 cm/s,
    Manning n = 0.009.  The bed falls toward x = L (hb = slope * x, positive
    downward); walls on the sides and the upper end, free outflow at x = L;
    dry start (zeta = -hb).  A dry plane has no wave speed, so the step is
    capped at 0.02 s (the paper ran at a fixed 0.001 s)."""
    xy, tri, sides = rect_grid(nx, 1, L, W)
    hb = slope * xy[:, 0]
    be, bt, bs = _bnd(sides, {"right": (OUTFLOW, 0)})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), manning), be, bt, bs)
    z = np.zeros(len(hb))
    return Scenario("inclined_plane", mesh, -hb, z.copy(), z.copy(),
                    default_params(flux="roe", friction="manning", limiter=False, cfl=0.3, H0=H0,
                                   dt_max=0.02),
                    rain={"kind": "nodal", "r": np.full(len(hb), rain)}, n_steps=0)


# ---------------------------------------------------------------------------
# ensembles and request traces built from the basin generator
# ---------------------------------------------------------------------------
def log_uniform_sizes(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """n triangle counts drawn log-uniformly from [lo, hi] (seeded)."""
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(np.log(lo), np.log(hi), n))


def basin_member(config_id: int, i: int, n_tri: float, *, p: int = 1) -> Scenario:
    """Member i of an ensemble: the basin generator at about n_tri triangles
    (N x N grid with 2 N^2 ~ n_tri), its own seed, a rain peak ~ U(10, 120)
    mm/h and a storm track with a seeded start in the western half and a
    seeded heading, at 5 m/s; time step at most 0.5 s."""
    seed = seed_for(config_id, i)
    rng = np.random.default_rng(seed + 7)
    N = max(4, int(round(np.sqrt(n_tri / 2.0))))
    L = 200e3
    peak = rng.uniform(10.0, 120.0)
    ang = rng.uniform(-0.5 * np.pi, 0.5 * np.pi)
    track = parametric_track(rng.uniform(0.1, 0.5) * L, rng.uniform(0.2, 0.8) * L, 5.0 * np.cos(ang),
                             5.0 * np.sin(ang), peak * MM_PER_HOUR)
    sc = basin(N, seed, peak_mmh=peak, track=track, p=p)
    sc.name = f"member_{config_id}_{i}"
    # coarse members would take CFL steps of several seconds, where explicit
    # Manning friction in thin layers is unstable; cap at the 0.5 s step of
    # the paper's large-mesh run
    sc.params["dt_max"] = 0.5
    return sc


def ensemble_plan(n: int = 64, lo: float = 1e4, hi: float = 5e5, config_id: int = 4):
    """Sizes and orders of an ensemble: log-uniform sizes, even members p = 1,
    odd members p = 2.  Returns a list of (i, n_tri, p)."""
    sizes = log_uniform_sizes(n, lo, hi, seed_for(config_id))
    return [(i, float(sizes[i]), 1 if i % 2 == 0 else 2) for i in range(n)]


def request_trace(n_req: int = 400, rate: float = 20.0, n_meshes: int = 64, steps=(500, 5000),
                  config_id: int = 5):
    """Poisson arrivals (mean ``rate`` per second) of flood scenarios: for each
    request its arrival time [s], the index of its mesh in the pool, its step
    count ~ U{steps} and its storm (peak ~ U(10, 120) mm/h, seeded track).
    The pool holds ``n_meshes`` basin meshes of log-uniform sizes in
    [5e3, 2e6] triangles (see :func:`serving_pool_sizes`)."""
    rng = np.random.default_rng(seed_for(config_id))
    t = np.cumsum(rng.exponential(1.0 / rate, n_req))
    mesh = rng.integers(0, n_meshes, n_req)
    nst = rng.integers(steps[0], steps[1] + 1, n_req)
    peak = rng.uniform(10.0, 120.0, n_req)
    ang = rng.uniform(-0.5 * np.pi, 0.5 * np.pi, n_req)
    x0 = rng.uniform(0.1, 0.5, n_req)
    y0 = rng.uniform(0.2, 0.8, n_req)
    return [dict(id=k, arrival=float(t[k]), mesh=int(mesh[k]), n_steps=int(nst[k]),
                 track=parametric_track(x0[k] * 200e3, y0[k] * 200e3, 5.0 * np.cos(ang[k]),
                                        5.0 * np.sin(ang[k]), peak[k] * MM_PER_HOUR))
            for k in range(n_req)]


def serving_pool_sizes(n_meshes: int = 64, lo: float = 5e3, hi: float = 2e6, config_id: int = 5):
    return log_uniform_sizes(n_meshes, lo, hi, seed_for(config_id, 999))
