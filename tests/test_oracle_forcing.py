"""Pins for the forcing evaluation (Sec. 2.3 Eq. rain, Sec. 2.5, Sec. 3.3).

Linear interpolation reproduces the records at record times and straight
tracks exactly; bilinear lattice interpolation reproduces any bilinear field
and is zero outside the lattice; the radial profile is continuous at r_m
with the peak there; element rain is the mean of the three vertex values.
"""
import numpy as np

import meshgen
from oracle import forcing


def test_interp_records_and_track():
    rec = meshgen.parametric_track(1000.0, 2000.0, 5.0, -2.0, 3e-5, t_end=1e4, n_rec=5)
    for row in rec:
        v, _, _, _ = forcing.interp_records(rec[:, 0], rec[:, 1:], row[0])
        np.testing.assert_allclose(v, row[1:], rtol=1e-15)
    v, _, _, _ = forcing.interp_records(rec[:, 0], rec[:, 1:], 3333.0)
    np.testing.assert_allclose(v[:2], [1000 + 5 * 3333.0, 2000 - 2 * 3333.0], rtol=1e-14)
    v, _, _, _ = forcing.interp_records(rec[:, 0], rec[:, 1:], 2e4)     # held after the last record
    np.testing.assert_allclose(v, rec[-1, 1:])


def test_parametric_profile_shape():
    rec = np.array([[0.0, 0.0, 0.0, 1e-5, 4e-6, 30e3, 100e3]])
    xy = np.array([[0.0, 0.0], [30e3 - 1e-6, 0.0], [30e3, 0.0], [0.0, 130e3], [15e3, 0.0]])
    r = forcing.rain_parametric_nodes(xy, rec, 0.0)
    np.testing.assert_allclose(r[0], 4e-6)                         # T0 at the centre
    np.testing.assert_allclose(r[1], 1e-5, rtol=1e-9)              # continuous at r_m
    np.testing.assert_allclose(r[2], 1e-5)
    np.testing.assert_allclose(r[3], 1e-5 * np.exp(-1.0), rtol=1e-14)
    np.testing.assert_allclose(r[4], 7e-6, rtol=1e-14)


def test_bilinear_lattice():
    nx, ny, x0, y0, dx, dy = 5, 4, -100.0, 50.0, 20.0, 30.0
    gx = x0 + dx * np.arange(nx); gy = y0 + dy * np.arange(ny)
    X, Y = np.meshgrid(gx, gy)
    f = lambda x, y: 1e-6 * (1 + 0.01 * x + 0.02 * y + 1e-4 * x * y)  # noqa: E731
    vals = f(X, Y)[None].repeat(2, 0)
    spec = dict(x0=x0, y0=y0, dx=dx, dy=dy, nx=nx, ny=ny, t_rec=np.array([0.0, 10.0]), vals=vals)
    rng = np.random.default_rng(0)
    pts = np.stack([rng.uniform(gx[0], gx[-1], 50), rng.uniform(gy[0], gy[-1], 50)], 1)
    pts = np.vstack([pts, [[gx[-1], gy[-1]], [gx[0], gy[0]], [gx[-1] + 1e-9, gy[0]], [gx[0], gy[0] - 1]]])
    r = forcing.rain_gridded_nodes(pts, spec, 5.0)
    np.testing.assert_allclose(r[:-2], f(pts[:-2, 0], pts[:-2, 1]), rtol=1e-13)
    assert r[-2] == 0.0 and r[-1] == 0.0
    # linear in time between records
    spec["vals"] = np.stack([vals[0], 3 * vals[0]])
    r = forcing.rain_gridded_nodes(pts[:3], spec, 2.5)
    np.testing.assert_allclose(r, 1.5 * f(pts[:3, 0], pts[:3, 1]), rtol=1e-13)


def test_tide_river_and_element_mean():
    spec = (0.1, np.array([[0.5, 100.0, 0.0], [0.2, 50.0, np.pi / 2]]))
    assert abs(forcing.tide_level(spec, 25.0) - (0.1 + 0.5 + 0.2 * np.cos(np.pi + np.pi / 2 * 0 + 0) * 0 + 0.2 * np.sin(np.pi + np.pi / 2))) < 1e-15
    riv = (np.array([0.0, 10.0]), np.array([-1.0, -3.0]))
    assert forcing.river_flux(riv, -5.0) == -1.0 and forcing.river_flux(riv, 20.0) == -3.0
    assert abs(forcing.river_flux(riv, 2.5) + 1.5) < 1e-15
    r = np.array([1.0, 2.0, 6.0, 9.0])
    tri = np.array([[0, 1, 2], [1, 2, 3]])
    np.testing.assert_allclose(forcing.element_rain(r, tri), [3.0, 17.0 / 3.0])
