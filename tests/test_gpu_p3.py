"""Cubic elements (p = 3, ten Dubiner modes, collapsed 4 x 4 area rule, four
Gauss points per edge, SSP(3,3) at CFL 0.1: the generators' default) on the GPU against the oracle.

* small mixed basins (every boundary type, wet/dry fronts; Roe with gridded
  rain, LLF with the limiter and parametric rain, and with a storm's wind
  and pressure): one step to 1e-12, fifty steps to 1e-10 (FP64), flags and
  budgets equal;
* a closed wet basin under a moving storm in FP32 to 1e-4;
* lake at rest stays at rest;
* both stage kernels (per element; per edge with the tile's traces staged
  in LDS) in every case; the autotuner times both;
* a 20,000-triangle window of the benchmark basin: one step from a GPU
  state, every element against the oracle.
"""
import numpy as np
import pytest

import meshgen
from meshgen.generators import Mesh, Scenario, _bnd, default_params, rect_grid
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
    "roe_gridded": dict(flux="roe", limiter=False, rain_kind="gridded"),
    "llf_param_lim": dict(flux="llf", limiter=True, rain_kind="parametric"),
    "llf_lim_storm": dict(flux="llf", limiter=True, rain_kind="parametric", wind=True),
}


def _mixed(case, **kw):
    return meshgen.small_mixed(seed=5, nx=20, ny=10, p=3, **CASES[case], **kw)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_p3_parity_fp64(dg, case, variant):
    sc = _mixed(case)
    print(f"p=3 case {case} variant {variant}: E={sc.mesh.n_tri}", flush=True)
    gpu = dg.Solver.from_scenario(sc, precision="fp64")
    gpu.set_variant(variant)
    orc = from_scenario(sc)
    e0 = rel_l2(gpu.state("modal"), orc.w, orc)
    assert e0.max() < 1e-13, e0
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


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_p3_closed_basin_storm_fp32(dg, variant):
    rec = [[0.0, 20e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0],
           [4.0e3, 60e3, 40e3, 5000.0, 15e3, 1.4, 1.0, 2.0, 1.0]]
    xy, tri, sides = rect_grid(24, 24, 80e3, 80e3, jitter=0.15, rng=np.random.default_rng(5), diagonal="short")
    hb = 15.0 + 5.0 * np.sin(xy[:, 0] / 2e4) * np.cos(xy[:, 1] / 3e4)
    be, bt, bs = _bnd(sides, {})
    z = np.zeros(len(hb))
    sc = Scenario("closed_p3", Mesh(xy, tri, hb, np.full(len(hb), 0.025), be, bt, bs), z, z.copy(), z.copy(),
                  default_params(p=3, flux="roe", friction="manning", H0=0.01), met=np.asarray(rec))
    gpu = dg.Solver.from_scenario(sc, precision="fp32")
    gpu.set_variant(variant)
    orc = from_scenario(sc)
    gpu.step(100)
    orc.step(100)
    err = rel_l2(gpu.state("modal"), orc.w, orc)
    print("p=3 closed basin FP32 rel L2", err, flush=True)
    assert np.abs(orc.w[:, 1:, 0]).max() > 1e-2
    assert err.max() < 1e-4, err
    gpu.close()


@pytest.mark.parametrize("precision,tol,variant", [("fp64", 1e-11, 0), ("fp64", 1e-11, 1), ("fp32", 1e-4, 0),
                                                   ("fp32", 1e-4, 1), ("fp32", 1e-4, 2)])
def test_p3_lake_at_rest(dg, precision, tol, variant):
    sc = meshgen.lake_at_rest(p=3)
    gpu = dg.Solver.from_scenario(sc, precision=precision)
    gpu.set_variant(variant)
    gpu.step(50)
    v = gpu.state("vertex")
    assert np.abs(v[:, 1:]).max() < tol
    assert np.abs(v[:, 0] - 0.7).max() < tol
    gpu.close()


def test_p3_kernels_agree_and_autotune(dg):
    """The two stage kernels differ only in summation order; the autotuner
    times both and leaves the state as it was."""
    sc = _mixed("llf_lim_storm")
    a = dg.Solver.from_scenario(sc, precision="fp64")
    b = dg.Solver.from_scenario(sc, precision="fp64")
    a.set_variant(0); b.set_variant(1)
    a.step(30); b.step(30)
    err = rel_l2(a.state(), b.state(), from_scenario(sc))
    assert err.max() < 1e-12, err
    w = b.state()
    v, ms = b.autotune(2)
    assert v in (0, 1) and ms[0] > 0.0 and ms[1] > 0.0
    assert np.array_equal(b.state(), w)
    a.close(); b.close()


@pytest.mark.parametrize("precision,tol,variant", [("fp64", 1e-11, 0), ("fp64", 1e-11, 1), ("fp32", 5e-5, 0),
                                                   ("fp32", 5e-5, 1), ("fp32", 5e-5, 2)])
def test_p3_basin_window_one_step(dg, precision, tol, variant):
    sc = meshgen.basin_window(100, p=3)
    gpu = dg.Solver.from_scenario(sc, precision=precision)
    gpu.set_variant(variant)
    gpu.step(10)
    w = gpu.state()
    m0 = gpu.mass()
    orc = from_scenario(sc)
    orc.set_state(w, m0["t"], post=False)
    orc.dt = m0["dt_next"]
    gpu.step(1)
    orc.step(1)
    err = rel_l2(gpu.state(), orc.w, orc)
    print(precision, "p=3 basin window one-step rel L2", err, flush=True)
    assert err.max() < tol, err
    gpu.close()


@pytest.mark.parametrize("case", list(CASES))
def test_p3_matrix_core_area_integrals_fp32(dg, case):
    """Stage variant 2: the area integrals as 16x16x4 matrix products on the
    matrix cores (FP32).  Against the oracle to the FP32 bar after one and
    after 30 steps, and against the vector kernel on the same 64-element
    tiles (variant 1), from which it differs only in the order of the area
    sums: to 1e-5 of the state scale after 30 steps."""
    sc = _mixed(case)
    a = dg.Solver.from_scenario(sc, precision="fp32")
    b = dg.Solver.from_scenario(sc, precision="fp32")
    a.set_variant(2)
    b.set_variant(1); b.set_tile(64)
    assert a.variant() == 2 and a.tile() == 64 and b.tile() == 64
    orc = from_scenario(sc)
    a.step(1); b.step(1); orc.step(1)
    e1 = rel_l2(a.state(), orc.w, orc)
    d1 = rel_l2(a.state(), b.state(), orc)
    a.step(29); b.step(29); orc.step(29)
    ea = rel_l2(a.state(), orc.w, orc)
    eb = rel_l2(b.state(), orc.w, orc)
    d = rel_l2(a.state(), b.state(), orc)
    print(f"p=3 {case} FP32 matrix-core area: one step {e1} (vs vector {d1}); 30 steps {ea} "
          f"(vector kernel {eb}, between them {d})", flush=True)
    assert e1.max() < 5e-6, e1
    assert ea.max() < 1e-4 and eb.max() < 1e-4, (ea, eb)
    assert d.max() < 1e-5, d
    ma, mb = a.mass(), b.mass()
    for k in ("t", "volume", "rain_in"):
        assert abs(ma[k] - mb[k]) <= 1e-6 * max(1.0, abs(mb[k])), (k, ma[k], mb[k])
    a.close(); b.close()


def test_p3_matrix_core_variant_scope_and_autotune(dg):
    """Variant 2 is refused where it is not built (FP64, p < 3); on a p = 3
    FP32 context the autotuner times it as its seventh configuration and
    leaves the state as it was."""
    import paper_2307_14302_amd._native as N
    sc = _mixed("llf_param_lim")
    c64 = dg.Solver.from_scenario(sc, precision="fp64")
    with pytest.raises(N.DgsweError, match="EINVAL"):
        c64.set_variant(2)
    p1 = dg.Solver.from_scenario(meshgen.small_mixed(seed=5, nx=12, ny=6, p=1), precision="fp32")
    with pytest.raises(N.DgsweError, match="EINVAL"):
        p1.set_variant(2)
    b = dg.Solver.from_scenario(sc, precision="fp32")
    b.step(5)
    w = b.state()
    v, ms = b.autotune(2)
    assert v in (0, 1, 2) and ms[6] > 0.0 and ms[0] > 0.0 and ms[5] > 0.0
    assert np.array_equal(b.state(), w)
    c64.close(); p1.close(); b.close()
