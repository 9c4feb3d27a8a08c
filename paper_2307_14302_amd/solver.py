"""Python front end of the HIP DG solver: argument marshalling only.

Every computation happens in libdgswe.so (include/dgswe.h).  ``Solver`` owns
one context (one mesh, one state); ``Batch`` steps many contexts together.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, Optional

import numpy as np

from . import _native as N
from ._native import call, dptr, fptr, iptr

_FLUX = {"roe": N.ROE, "llf": N.LLF}
_FRICTION = {"manning": N.MANNING, "quadratic": N.QUADRATIC}
_PREC = {"fp64": N.FP64, "fp32": N.FP32, "f64": N.FP64, "f32": N.FP32}


def params_from_dict(d: Dict[str, object]) -> N.Params:
    p = N.Params()
    N.lib.dgswe_default_params(C.byref(p))
    for k, v in d.items():
        if k == "flux":
            p.flux = _FLUX[v] if isinstance(v, str) else int(v)
        elif k == "friction":
            p.friction = _FRICTION[v] if isinstance(v, str) else int(v)
        elif k == "precision":
            p.precision = _PREC[v] if isinstance(v, str) else int(v)
        elif k == "limiter":
            p.limiter = int(bool(v))
        elif k in ("p", "rk_stages"):
            setattr(p, k, int(v))
        elif k in ("cfl", "dt_fixed", "dt_max", "H0", "g"):
            setattr(p, k, float(v))
    return p


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):       # torch.cuda.Stream
        return C.c_void_p(int(stream.cuda_stream)) if stream.cuda_stream else None
    return C.c_void_p(int(stream))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Solver:
    def __init__(self, params: Dict[str, object], stream=None):
        self.params = dict(params)
        self._p = params_from_dict(self.params)
        self.np = (self._p.p + 1) * (self._p.p + 2) // 2
        h = C.c_void_p()
        call("dgswe_create", C.byref(self._p), _stream_handle(stream), C.byref(h))
        self.h = h
        self.n_tri = 0
        self.n_nodes = 0

    # ------------------------------------------------------------- set-up
    def bind_workspace(self, ptr: int, nbytes: int):
        """Place every device array of this context in caller-owned device
        memory (e.g. ``t.data_ptr()`` of a torch tensor kept alive by the
        caller); call before the mesh is uploaded."""
        call("dgswe_workspace_bind", self.h, C.c_void_p(int(ptr)), C.c_size_t(int(nbytes)))
        return self

    def upload_mesh(self, xy, hb, fric, tri, bedges=None, btype=None, bslot=None):
        xy, hb, fric, tri = _f64(xy), _f64(hb), _f64(fric), _i32(tri)
        nb = 0 if bedges is None else len(bedges)
        be = _i32(bedges if nb else np.zeros((1, 2)))
        bt = _i32(btype if nb else np.zeros(1))
        bs = _i32(bslot if nb else np.zeros(1))
        call("dgswe_upload_mesh", self.h, xy.shape[0], dptr(xy), dptr(hb), dptr(fric), tri.shape[0], iptr(tri),
             nb, iptr(be), iptr(bt), iptr(bs))
        self.n_tri, self.n_nodes = int(tri.shape[0]), int(xy.shape[0])
        return self

    def share_mesh(self, other: "Solver"):
        call("dgswe_share_mesh", self.h, other.h)
        self.n_tri, self.n_nodes = other.n_tri, other.n_nodes
        return self

    def set_initial_nodal(self, zeta, qx, qy):
        z, a, b = _f64(zeta), _f64(qx), _f64(qy)
        call("dgswe_set_initial_nodal", self.h, dptr(z), dptr(a), dptr(b))

    def set_state(self, w, t: float = 0.0, totals: Optional[Dict[str, float]] = None, layout: str = "modal"):
        """State (modal (n_tri, 3, Np) or vertex (n_tri, 3, 3) values) at time
        t; ``totals`` (a dict as returned by :meth:`mass`) continues the
        budgets, step count and step size of an earlier run."""
        w = _f64(w)
        acc = None
        if totals is not None:
            m = N.Mass()
            for k, _ in N.Mass._fields_:
                if k in totals:
                    setattr(m, k, totals[k])
            acc = C.byref(m)
        call("dgswe_set_state", self.h, N.MODAL if layout == "modal" else N.VERTEX, dptr(w), float(t), acc)

    def set_rain(self, rain: Optional[Dict[str, object]]):
        kind = (rain or {}).get("kind", "none")
        if kind == "none":
            call("dgswe_clear_rain", self.h)
        elif kind == "nodal":
            r = _f64(rain["r"])
            call("dgswe_set_rain_nodal", self.h, dptr(r))
        elif kind == "parametric":
            rec = _f64(rain["records"])
            call("dgswe_set_rain_parametric", self.h, rec.shape[0], dptr(rec))
        elif kind == "gridded":
            t = _f64(rain["t_rec"])
            v = np.ascontiguousarray(rain["vals"], dtype=np.float32)
            call("dgswe_set_rain_gridded", self.h, float(rain["x0"]), float(rain["y0"]), float(rain["dx"]),
                 float(rain["dy"]), int(rain["nx"]), int(rain["ny"]), t.shape[0], dptr(t), fptr(v))
        else:
            raise ValueError(kind)

    def set_wind(self, records):
        """Storm wind and pressure records (t, xc, yc, dp, rm, B, wf, wbx, wby),
        one row each, or None to turn the forcing off."""
        if records is None:
            call("dgswe_clear_wind", self.h)
            return
        rec = _f64(np.asarray(records, dtype=np.float64).reshape(-1, 9))
        call("dgswe_set_wind_vortex", self.h, rec.shape[0], dptr(rec))

    def set_tide(self, slot: int, mean: float, rows):
        rows = _f64(np.asarray(rows, dtype=np.float64).reshape(-1, 3))
        buf = rows if rows.size else np.zeros(3)
        call("dgswe_set_ocean_tide", self.h, int(slot), float(mean), rows.shape[0], dptr(buf))

    def set_river(self, slot: int, t, q):
        t, q = _f64(t), _f64(q)
        call("dgswe_set_river_flux", self.h, int(slot), t.shape[0], dptr(t), dptr(q))

    # -------------------------------------------------------------- run
    def step(self, n: int = 1):
        call("dgswe_step", self.h, int(n))

    def sync(self):
        call("dgswe_sync", self.h)

    # ---------------------------------------------------------- results
    def state(self, layout: str = "modal") -> np.ndarray:
        if layout == "modal":
            out = np.empty((self.n_tri, 3, self.np))
            call("dgswe_read_state", self.h, N.MODAL, dptr(out))
        else:
            out = np.empty((self.n_tri, 3, 3))
            call("dgswe_read_state", self.h, N.VERTEX, dptr(out))
        return out

    def flags(self) -> np.ndarray:
        out = np.zeros(self.n_tri, dtype=np.uint8)
        call("dgswe_read_flags", self.h, out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out

    def mass(self) -> Dict[str, float]:
        m = N.Mass()
        call("dgswe_mass_totals", self.h, C.byref(m))
        return m.as_dict()

    def info(self):
        v = [C.c_int64() for _ in range(4)]
        call("dgswe_info", self.h, *[C.byref(x) for x in v])
        return dict(n_tri=v[0].value, n_nodes=v[1].value, n_edges=v[2].value, n_flipped=v[3].value)

    def set_variant(self, variant: int):
        call("dgswe_set_tuning", self.h, N.TUNE_STAGE_VARIANT, int(variant))

    def autotune(self, n_steps: int = 5):
        """Pick the fastest stage-kernel configuration for this mesh; the
        state is left as it was.  Returns (variant, (ms/step per-element,
        per-edge with post passes, per-edge fused, per-edge on tiles of 512,
        128 and 64 elements, per-edge with matrix-core area integrals; 0
        where it does not apply))."""
        v = C.c_int()
        ms = (C.c_double * 7)()
        call("dgswe_autotune", self.h, int(n_steps), C.byref(v), ms)
        return v.value, tuple(ms)

    def set_fused(self, on: bool):
        """Post-processing fused into the next stage (limiter on, p <= 2)."""
        call("dgswe_set_tuning", self.h, N.TUNE_FUSED_POST, int(bool(on)))

    def fused(self) -> int:
        v = C.c_int()
        call("dgswe_get_tuning", self.h, N.TUNE_FUSED_POST, C.byref(v))
        return v.value

    def set_tile(self, tile: int):
        """Elements per workgroup of the per-edge stage kernel: 64, 128, 256
        or (p = 1) 512; a tile other than 256 turns fused post-processing
        off."""
        call("dgswe_set_tuning", self.h, N.TUNE_STAGE_TILE, int(tile))

    def tile(self) -> int:
        v = C.c_int()
        call("dgswe_get_tuning", self.h, N.TUNE_STAGE_TILE, C.byref(v))
        return v.value

    def variant(self) -> int:
        v = C.c_int()
        call("dgswe_get_tuning", self.h, N.TUNE_STAGE_VARIANT, C.byref(v))
        return v.value

    def profiling(self, on=True):
        """False/0 off, True/1 every kernel, 2 the stage kernel only."""
        call("dgswe_set_profiling", self.h, int(on))

    def kernel_stats(self, name: str):
        n, ms = C.c_int64(), C.c_double()
        call("dgswe_kernel_stats", self.h, name.encode(), C.byref(n), C.byref(ms))
        return n.value, ms.value

    def footprint(self) -> int:
        return int(N.lib.dgswe_footprint_bytes(C.byref(self._p), self.n_tri, self.n_nodes))

    @staticmethod
    def footprint_of(params: Dict[str, object], like: "Solver") -> int:
        """Device bytes of a context with ``params`` on the mesh of ``like``."""
        p = params_from_dict(params)
        return int(N.lib.dgswe_footprint_bytes(C.byref(p), like.n_tri, like.n_nodes))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            call("dgswe_destroy", self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- helpers
    @classmethod
    def from_scenario(cls, sc, stream=None, mesh_from: Optional["Solver"] = None, workspace=None, **over):
        """Build a solver from a workload description with attributes
        mesh (xy, tri, hb, fric, bedges, btype, bslot), zeta0/qx0/qy0,
        params, rain, tides, rivers and (optional) met.  workspace =
        (device pointer, bytes) places the context's arrays there."""
        prm = dict(sc.params)
        prm.update(over)
        s = cls(prm, stream=stream)
        if workspace is not None:
            s.bind_workspace(*workspace)
        m = sc.mesh
        if mesh_from is not None:
            s.share_mesh(mesh_from)
        else:
            s.upload_mesh(m.xy, m.hb, m.fric, m.tri, m.bedges, m.btype, m.bslot)
        for slot, (mean, rows) in sc.tides.items():
            s.set_tide(slot, mean, rows)
        for slot, (t, q) in sc.rivers.items():
            s.set_river(slot, t, q)
        s.set_rain(sc.rain)
        if getattr(sc, "met", None) is not None:
            s.set_wind(sc.met)
        s.set_initial_nodal(sc.zeta0, sc.qx0, sc.qy0)
        return s


class Batch:
    def __init__(self, params: Dict[str, object], budget_bytes: int = 0, stream=None):
        p = params_from_dict(params)
        h = C.c_void_p()
        call("dgswe_batch_create", C.byref(p), _stream_handle(stream), int(budget_bytes), C.byref(h))
        self.h = h
        self.members: Dict[int, Solver] = {}

    def add(self, s: Solver, n_steps: int) -> int:
        slot = C.c_int32()
        call("dgswe_batch_add", self.h, s.h, int(n_steps), C.byref(slot))
        self.members[slot.value] = s
        return slot.value

    def step(self, n: int = 1):
        call("dgswe_batch_step", self.h, int(n))

    def poll(self):
        cap = max(1, len(self.members))
        buf = np.zeros(cap, dtype=np.int32)
        n = C.c_int32()
        call("dgswe_batch_poll", self.h, iptr(buf), cap, C.byref(n))
        return [int(x) for x in buf[: min(n.value, cap)]]

    def read(self, slot: int, layout: str = "modal"):
        """State and totals of a live member, by slot."""
        s = self.members.get(slot)
        out = np.empty((s.n_tri, 3, s.np if layout == "modal" else 3)) if s is not None else None
        m = N.Mass()
        call("dgswe_batch_read", self.h, int(slot), N.MODAL if layout == "modal" else N.VERTEX,
             dptr(out) if out is not None else None, C.byref(m))
        return out, m.as_dict()

    def retire(self, slot: int) -> Solver:
        call("dgswe_batch_retire", self.h, int(slot))
        return self.members.pop(slot)

    def info(self):
        n, f = C.c_int32(), C.c_int64()
        call("dgswe_batch_info", self.h, C.byref(n), C.byref(f))
        return n.value, f.value

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            call("dgswe_batch_destroy", self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
