"""Forcing: nodal rain, element rain, tides and river fluxes (FP64).

Rain enters through nodes (Sec. 2.3): a rate r is given at every mesh node
and the element source is the plain average of its three vertex values,
Eq. rain.  It is added in every element, wet or dry.  Node rates come from
  * a user array (held until replaced);
  * a storm-centred radial profile whose parameters are interpolated
    linearly in time between storm records and evaluated at each node from
    its distance to the centre (Sec. 2.5).  The R-CLIPER expressions are in
    a figure that is not available, so the profile has the same shape with
    explicit parameters: R = T0 + (peak - T0) r / r_m inside r_m and
    peak exp(-(r - r_m)/r_e) beyond;
  * a rain lattice read at record times and interpolated linearly onto each
    node (Sec. 3.3): bilinear in space (zero outside the lattice) and linear
    in time between records (held constant before the first and after the
    last record).
Rain is evaluated once per time step at t^n and held for all stages.

Boundary forcing, evaluated at each stage time: ocean elevation
mean + sum a sin(2 pi t / T + phase); river normal flux (m^2/s, outward
positive, Eq. river_bc) linear in time between samples and held beyond.
"""
from __future__ import annotations

import numpy as np


def interp_records(t_rec, values, t):
    """Linear interpolation of rows of ``values`` at time t (clamped)."""
    t_rec = np.asarray(t_rec, dtype=np.float64)
    values = np.asarray(values, dtype=np.float64)
    if len(t_rec) == 1 or t <= t_rec[0]:
        return values[0].copy(), 0, 0, 0.0
    if t >= t_rec[-1]:
        return values[-1].copy(), len(t_rec) - 1, len(t_rec) - 1, 0.0
    k = int(np.searchsorted(t_rec, t, side="right") - 1)
    th = (t - t_rec[k]) / (t_rec[k + 1] - t_rec[k])
    return (1.0 - th) * values[k] + th * values[k + 1], k, k + 1, th


def rain_parametric_nodes(xy, records, t):
    rec = np.asarray(records, dtype=np.float64)
    v, _, _, _ = interp_records(rec[:, 0], rec[:, 1:], t)
    xc, yc, peak, T0, rm, re = v
    r = np.hypot(xy[:, 0] - xc, xy[:, 1] - yc)
    inner = T0 + (peak - T0) * r / rm
    outer = peak * np.exp(-(r - rm) / re)
    return np.where(r < rm, inner, outer)


def lattice_bilinear(vals2d, x0, y0, dx, dy, nx, ny, x, y):
    fx = (x - x0) / dx
    fy = (y - y0) / dy
    inside = (fx >= 0.0) & (fx <= nx - 1) & (fy >= 0.0) & (fy <= ny - 1)
    i = np.clip(np.floor(fx), 0, max(nx - 2, 0)).astype(np.int64)
    j = np.clip(np.floor(fy), 0, max(ny - 2, 0)).astype(np.int64)
    ax = fx - i
    ay = fy - j
    i1 = np.minimum(i + 1, nx - 1)
    j1 = np.minimum(j + 1, ny - 1)
    v = vals2d.astype(np.float64)
    f = ((1.0 - ay) * ((1.0 - ax) * v[j, i] + ax * v[j, i1])
         + ay * ((1.0 - ax) * v[j1, i] + ax * v[j1, i1]))
    return np.where(inside, f, 0.0)


def rain_gridded_nodes(xy, spec, t):
    t_rec = np.asarray(spec["t_rec"], dtype=np.float64)
    vals = np.asarray(spec["vals"])
    args = (spec["x0"], spec["y0"], spec["dx"], spec["dy"], spec["nx"], spec["ny"], xy[:, 0], xy[:, 1])
    if len(t_rec) == 1 or t <= t_rec[0]:
        return lattice_bilinear(vals[0], *args)
    if t >= t_rec[-1]:
        return lattice_bilinear(vals[-1], *args)
    k = int(np.searchsorted(t_rec, t, side="right") - 1)
    th = (t - t_rec[k]) / (t_rec[k + 1] - t_rec[k])
    return (1.0 - th) * lattice_bilinear(vals[k], *args) + th * lattice_bilinear(vals[k + 1], *args)


def rain_nodes(rain, xy, t):
    kind = rain.get("kind", "none")
    if kind == "none":
        return np.zeros(xy.shape[0])
    if kind == "nodal":
        return np.asarray(rain["r"], dtype=np.float64)
    if kind == "parametric":
        return rain_parametric_nodes(xy, rain["records"], t)
    if kind == "gridded":
        return rain_gridded_nodes(xy, rain, t)
    raise ValueError(kind)


def element_rain(r_nodes, tri):
    """Eq. rain: R_e = (r(n1) + r(n2) + r(n3)) / 3."""
    return (r_nodes[tri[:, 0]] + r_nodes[tri[:, 1]] + r_nodes[tri[:, 2]]) / 3.0


def tide_level(spec, t):
    mean, rows = spec
    z = float(mean)
    for a, T, ph in np.asarray(rows, dtype=np.float64).reshape(-1, 3):
        z += a * np.sin(2.0 * np.pi * t / T + ph)
    return z


def river_flux(spec, t):
    ts, qs = spec
    ts = np.asarray(ts, dtype=np.float64)
    qs = np.asarray(qs, dtype=np.float64)
    v, _, _, _ = interp_records(ts, qs[:, None], t)
    return float(v[0])
