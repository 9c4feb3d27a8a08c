"""dgswe_step_noalloc, the allocation-free step (for callers that cannot
allocate device memory), called through the C ABI: it must give the states,
flags and totals of dgswe_step bit for bit, on two calls in a row (the second
on a smaller mesh, so the static scratch holds the first call's contents), in
FP64 and FP32, on the limiter's post-pass path and on the path without it;
a set-up call after it sees the last step's partials; meshes beyond its
scratch are refused."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2307_14302_amd as pkg
    return pkg


@pytest.mark.parametrize("tile", [256, 64])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_step_equals_step(dg, precision, tile):
    from paper_2307_14302_amd import _native as N
    cases = [(meshgen.basin_window(40), 30),                                              # limiter on
             (meshgen.small_mixed(seed=9, nx=12, ny=6, rain_kind="gridded"), 20)]          # smaller, no limiter
    for sc, n in cases:
        print(f"{precision} {sc.name} E={sc.mesh.n_tri} limiter={sc.params['limiter']} {n} steps", flush=True)
        a = dg.Solver.from_scenario(sc, precision=precision)
        b = dg.Solver.from_scenario(sc, precision=precision)
        for s in (a, b):
            s.set_variant(1)
            s.set_tile(tile)
        a.step(n)
        N.call("dgswe_step_noalloc", b.h, n)
        assert np.array_equal(a.state(), b.state())
        assert np.array_equal(a.flags(), b.flags())
        assert a.mass() == b.mass()
        # a set-up call after the steps recomputes totals from the last
        # step's partials, which the context holds after either call
        for s in (a, b):
            s.set_rain({"kind": "none"})
        assert a.mass() == b.mass()
        a.step(3)
        N.call("dgswe_step_noalloc", b.h, 3)
        assert np.array_equal(a.state(), b.state()) and a.mass() == b.mass()
        a.close(); b.close()


def test_noalloc_refuses_meshes_beyond_its_scratch(dg):
    from paper_2307_14302_amd import _native as N
    xy, tri, _ = meshgen.rect_grid(1100, 1100, 100e3, 100e3)          # 2,420,000 triangles
    s = dg.Solver(dict(precision="fp32", dt_fixed=1.0))
    s.upload_mesh(xy, np.full(len(xy), 5.0), np.full(len(xy), 0.02), tri)
    s.set_initial_nodal(np.zeros(len(xy)), np.zeros(len(xy)), np.zeros(len(xy)))
    with pytest.raises(N.DgsweError, match="2094848 triangles at most") as ei:
        N.call("dgswe_step_noalloc", s.h, 1)
    assert ei.value.code == N.DGSWE_EINVAL
    assert s.mass()["steps"] == 0
    s.close()
