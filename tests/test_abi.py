"""The C ABI library loads and exports every function include/dgswe.h
declares; host-only calls behave as documented (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dgswe.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dgswe_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("dgswe_create", "dgswe_upload_mesh", "dgswe_set_rain_nodal", "dgswe_set_rain_parametric",
                 "dgswe_set_rain_gridded", "dgswe_step", "dgswe_read_state", "dgswe_mass_totals",
                 "dgswe_batch_step", "dgswe_footprint_bytes"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2307_14302_amd import _native as N
    lib = C.CDLL(N.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the binding wraps every declared function
    assert set(declared_functions()) <= set(N.SIGNATURES)


def test_host_only_calls():
    from paper_2307_14302_amd import _native as N
    p = N.Params()
    assert N.lib.dgswe_default_params(C.byref(p)) == 0
    assert (p.p, p.precision, p.flux, p.rk_stages, p.limiter) == (1, N.FP64, N.ROE, 2, 0)
    assert abs(p.cfl - 0.3) < 1e-15 and abs(p.H0 - 1e-3) < 1e-18 and abs(p.g - 9.81) < 1e-15
    f64 = N.lib.dgswe_footprint_bytes(C.byref(p), 1_000_000, 500_000)
    p.precision = N.FP32
    f32 = N.lib.dgswe_footprint_bytes(C.byref(p), 1_000_000, 500_000)
    assert 0 < f32 < f64
    p.p = 7
    assert N.lib.dgswe_footprint_bytes(C.byref(p), 10, 10) == N.DGSWE_EINVAL
    assert b"p must be" in N.lib.dgswe_last_error()
    assert N.lib.dgswe_default_params(None) == N.DGSWE_EINVAL


def test_create_rejects_bad_params_before_touching_the_device():
    from paper_2307_14302_amd import _native as N
    p = N.Params()
    N.lib.dgswe_default_params(C.byref(p))
    h = C.c_void_p()
    for field, bad in (("rk_stages", 4), ("flux", 9), ("H0", -1.0), ("precision", 5)):
        q = N.Params.from_buffer_copy(p)
        setattr(q, field, bad)
        assert N.lib.dgswe_create(C.byref(q), None, C.byref(h)) == N.DGSWE_EINVAL
        assert not h.value


def test_product_path_has_no_fallback():
    """The binding loads only the in-tree HIP library and never the oracle."""
    src = open(os.path.join(ROOT, "paper_2307_14302_amd", "_native.py")).read()
    src += open(os.path.join(ROOT, "paper_2307_14302_amd", "solver.py")).read()
    assert "oracle" not in src
    assert "import numpy" in src  # argument marshalling only


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU and says so for --gpus N > 1 (before any
    device work)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 1" in r.stderr
