"""Storm wind stress and atmospheric pressure on the GPU against the oracle.

* small mixed basins (every boundary type, wet/dry fronts, limiter or p = 2)
  crossed by a storm vortex over a background wind: one step to 1e-12 and
  fifty steps to 1e-10 (FP64), both stage-kernel variants, the per-edge one
  on 256- and 64-element tiles; a closed wet basin in FP32 to 1e-4;
* the two discrete equilibria of the oracle pins (inverse barometer under a
  stationary low, wind set-up over a bed of the same slope) stay at rest on
  the GPU;
* clearing the wind gives back the run without it, bit for bit; bad records
  are refused;
* the full-size 1M-triangle basin with the storm's wind and pressure, in
  the autotuned configuration the bench times: one step from a GPU state,
  every element against the oracle.
"""
import numpy as np
import pytest

import meshgen
from meshgen.generators import Mesh, Scenario, _bnd, default_params, rect_grid
from oracle import met
from oracle.solver import from_scenario
from tests.parity import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2307_14302_amd as pkg
    return pkg


CASES = {
    "p1_llf_param_lim": dict(p=1, flux="llf", limiter=True, rain_kind="parametric", wind=True),
    "p2_roe_gridded": dict(p=2, flux="roe", limiter=False, rain_kind="gridded", wind=True),
}


@pytest.mark.parametrize("variant,tile", [(0, 256), (1, 256), (1, 64)])
@pytest.mark.parametrize("case", list(CASES))
def test_storm_parity_fp64(dg, case, variant, tile):
    sc = meshgen.small_mixed(seed=5, nx=20, ny=10, **CASES[case])
    print(f"case {case} variant {variant} tile {tile}: E={sc.mesh.n_tri}", flush=True)
    gpu = dg.Solver.from_scenario(sc, precision="fp64")
    gpu.set_variant(variant)
    if variant == 1:
        gpu.set_tile(tile)
    orc = from_scenario(sc)
    gpu.step(1)
    orc.step(1)
    e1 = rel_l2(gpu.state("modal"), orc.w, orc)
    assert e1.max() < 1e-12, e1
    gpu.step(49)
    orc.step(49)
    err = rel_l2(gpu.state("modal"), orc.w, orc)
    print(case, "rel L2 after 50 steps", err, flush=True)
    assert err.max() < 1e-10, err
    np.testing.assert_array_equal(gpu.flags().astype(bool), orc.flags)
    mg, mo = gpu.mass(), orc.mass_totals()
    for k in ("t", "volume", "rain_in", "bnd_in", "bnd_out"):
        assert abs(mg[k] - mo[k]) <= 1e-10 * max(1.0, abs(mo[k])), (k, mg[k], mo[k])
    gpu.close()


def _closed(nx, ny, Lx, Ly, hb_fn, zeta_fn, records, flux="llf", p=1):
    xy, tri, sides = rect_grid(nx, ny, Lx, Ly, jitter=0.15, rng=np.random.default_rng(5), diagonal="short")
    hb = hb_fn(xy[:, 0], xy[:, 1])
    be, bt, bs = _bnd(sides, {})
    mesh = Mesh(xy, tri, hb, np.full(len(hb), 0.025), be, bt, bs)
    z = np.zeros(len(hb))
    return Scenario("closed", mesh, zeta_fn(xy[:, 0], xy[:, 1]), z, z.copy(),
                    default_params(p=p, flux=flux, friction="manning", H0=0.01, cfl=0.3),
                    met=np.asarray(records, dtype=np.float64))


def test_moving_storm_closed_basin_fp32(dg):
    rec = [[0.0, 20e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0],
           [4.0e3, 60e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0]]
    sc = _closed(32, 32, 80e3, 80e3, lambda x, y: 15.0 + 5.0 * np.sin(x / 2e4) * np.cos(y / 3e4),
                 lambda x, y: np.zeros_like(x), rec, flux="roe")
    gpu = dg.Solver.from_scenario(sc, precision="fp32")
    orc = from_scenario(sc)
    gpu.step(100)
    orc.step(100)
    err = rel_l2(gpu.state("modal"), orc.w, orc)
    print("closed basin FP32 rel L2", err, flush=True)
    assert np.abs(orc.w[:, 1:, 0]).max() > 1e-2        # the storm drives a real flow
    assert err.max() < 1e-4, err
    gpu.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-5)])
def test_equilibria_stay_at_rest(dg, precision, tol):
    # inverse barometer: flat 20 m bed, surface -psi under a stationary low
    rec = np.array([[0.0, 50e3, 45e3, 4000.0, 20e3, 1.5, 0.0, 0.0, 0.0]])
    psi = lambda x, y: met.met_nodes(rec, np.stack([x, y], 1), 0.0, 9.81)[2]   # noqa: E731
    sc = _closed(24, 24, 100e3, 100e3, lambda x, y: np.full_like(x, 20.0), lambda x, y: -psi(x, y), rec)
    # wind set-up: uniform 10 m/s wind, surface slope tau / (g H) over a bed of the same slope
    tau = 1.15e-3 * 1.42e-3 * 100.0
    H = 9.95
    a = tau / (9.81 * H)
    rec2 = np.array([[0.0, -1e9, 0.0, 0.0, 1e4, 1.0, 1.0, 10.0, 0.0]])
    sc2 = _closed(20, 6, 100e3, 30e3, lambda x, y: 10.0 - a * x, lambda x, y: a * x - 0.05, rec2)
    for s, scale in ((sc, 0.4 * np.sqrt(9.81 * 20.0)), (sc2, 0.17 * np.sqrt(9.81 * 10.0))):
        gpu = dg.Solver.from_scenario(s, precision=precision)
        gpu.step(50)
        q = gpu.state("modal")[:, 1:, :]
        print(precision, "largest discharge after 50 steps", np.abs(q).max(), flush=True)
        # a discharge of the order of (surface anomaly) x (wave speed) means the balance is lost
        assert np.abs(q).max() <= tol * scale
        gpu.close()


def test_clear_wind_restores_the_plain_run(dg):
    sc = meshgen.small_mixed(seed=8, nx=16, ny=8, flux="llf", limiter=True, rain_kind="parametric", wind=True)
    a = dg.Solver.from_scenario(sc, precision="fp32")
    a.set_wind(None)
    plain = meshgen.small_mixed(seed=8, nx=16, ny=8, flux="llf", limiter=True, rain_kind="parametric")
    b = dg.Solver.from_scenario(plain, precision="fp32")
    a.step(20)
    b.step(20)
    assert np.array_equal(a.state(), b.state())
    a.set_wind(sc.met)
    a.step(5)
    assert not np.array_equal(a.state(), b.state())
    a.close(); b.close()


def test_bad_wind_records_are_refused(dg):
    from paper_2307_14302_amd import _native as N
    sc = meshgen.small_mixed(seed=8, nx=8, ny=4)
    s = dg.Solver.from_scenario(sc)
    good = np.array([[0.0, 1e3, 1e3, 2000.0, 1e3, 1.3, 1.0, 0.0, 0.0]])
    s.set_wind(good)
    for col, val, msg in ((5, 0.0, "shape"), (5, 3.5, "shape"), (4, 0.0, "radius"), (3, -1.0, "deficit"),
                          (1, np.nan, "non-finite")):
        bad = good.copy()
        bad[0, col] = val
        with pytest.raises(N.DgsweError, match=msg):
            s.set_wind(bad)
    two = np.vstack([good, good])
    with pytest.raises(N.DgsweError, match="increase"):
        s.set_wind(two)
    s.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 2e-5)])
def test_full_size_basin_with_storm_one_step(dg, precision, tol):
    """1,002,528 triangles with the storm's wind and pressure on the rain
    track, in the launch configuration the bench times (autotuned stage
    kernel): 20 GPU steps, then one step on both sides from the same
    state."""
    sc = meshgen.basin(708, wind=True)
    gpu = dg.Solver.from_scenario(sc, precision=precision)
    variant, _ = gpu.autotune(2)
    print(precision, f"autotuned: variant {variant}, tile {gpu.tile()}, fused {gpu.fused()}", flush=True)
    gpu.step(20)
    w = gpu.state()
    m0 = gpu.mass()
    orc = from_scenario(sc)
    orc.set_state(w, m0["t"], post=False)
    orc.dt = m0["dt_next"]
    gpu.step(1)
    orc.step(1)
    err = rel_l2(gpu.state(), orc.w, orc)
    print(precision, "full-size storm one-step rel L2", err, flush=True)
    assert err.max() < tol, err
    gpu.close()
