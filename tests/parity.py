"""Helpers shared by the GPU parity tests (comparison norms only).

Parity norm: at vertex values (p = 1) or at the area quadrature points of
the degree's own rule (p >= 2: 9 points at p = 2, 16 at p = 3, so that every
mode of the element enters the comparison),
  err_zeta = ||zeta_gpu - zeta_orc|| / max(||zeta_orc||, 1e-3 sqrt(n) D)
  err_q    = ||q_gpu - q_orc||       / max(||q_orc||,    1e-3 sqrt(n) D c)
with q the discharge vector (qx, qy) at every point, D the RMS water depth
of the oracle state and c = sqrt(g D).  The momentum error is taken on the
vector field, so that a component that vanishes identically (a 1-D flow)
does not turn round-off into a relative error of order one; the floors keep
a fluid at rest from dividing by round-off.

Wet/dry flags: where FP32 and the FP64 oracle take a threshold decision on
different sides, the flip is reported with its margin (the oracle's largest
vertex depth minus the dry margin H0 (1 + 1e-3)), see :func:`flag_flips`.
"""
import numpy as np

from oracle import basis


def point_values(w, p):
    """Vertex values (p <= 1) or area-point values (p >= 2) of modal states."""
    if p >= 2:
        T = basis.Tables(p)
        return np.einsum("evm,mq->evq", w, T.phi_q)
    T = basis.Tables(1)
    return np.einsum("evm,im->evi", w[:, :, :3], T.phi_v)


def point_hb(orc):
    if orc.p >= 2:
        return orc.hb_q
    return orc.hbv


def rel_l2(w_gpu, w_orc, orc, g=9.81):
    """(err_zeta, err_q) as defined in the module docstring."""
    a, b = point_values(w_gpu, orc.p), point_values(w_orc, orc.p)
    H = b[:, 0] + point_hb(orc)
    n = H.size
    D = max(np.sqrt(np.mean(H * H)), 1e-3)
    c = np.sqrt(g * D)
    fz = 1e-3 * np.sqrt(n) * D
    fq = 1e-3 * np.sqrt(n) * D * c
    ez = np.linalg.norm(a[:, 0] - b[:, 0]) / max(np.linalg.norm(b[:, 0]), fz)
    eq = np.linalg.norm(a[:, 1:] - b[:, 1:]) / max(np.linalg.norm(b[:, 1:]), fq)
    return np.array([ez, eq])


def flag_flips(gpu_flags, orc):
    """Elements whose dry flag differs from the oracle's, with the margin of
    the oracle's decision: an element is dry when every vertex depth is at
    most H_dry, so the margin is (largest vertex depth) - H_dry.  Returns
    (ids, margins)."""
    g = np.asarray(gpu_flags).astype(bool)
    ids = np.nonzero(g != orc.flags)[0]
    Hv = np.einsum("em,im->ei", orc.w[:, 0, :], orc.T.phi_v) + orc.hbv
    return ids, Hv[ids].max(axis=1) - orc.H_dry


def fp32_storage_error(sc, steps, orc):
    """The FP32 error scale of a scenario: rel L2 (as :func:`rel_l2`) between
    the FP64 oracle ``orc`` after ``steps`` steps and the same oracle run with
    its bathymetry and its state after every stage rounded to FP32, i.e. what
    FP32 storage alone costs on this workload.  Limiter and wet/dry decisions
    are discontinuous, so on violent transients this alone can exceed 1e-4."""
    from oracle.solver import OracleSolver
    m = sc.mesh
    prm = dict(sc.params)
    r32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)  # noqa: E731
    s = OracleSolver(m.xy, m.tri, r32(m.hb), m.fric, m.bedges, m.btype, m.bslot, p=prm["p"], flux=prm["flux"],
                     friction=prm["friction"], limiter=prm["limiter"], cfl=prm["cfl"], dt_fixed=prm["dt_fixed"],
                     dt_max=prm["dt_max"], H0=prm["H0"], g=prm["g"], rk_stages=prm.get("rk_stages", 2),
                     rain=sc.rain, tides=sc.tides, rivers=sc.rivers, met=getattr(sc, "met", None))
    post = s.post
    s.post = lambda w: (lambda r: (r32(r[0]), r[1]))(post(w))
    s.set_initial_nodal(sc.zeta0, sc.qx0, sc.qy0)
    s.step(steps)
    return rel_l2(s.w, orc.w, orc)
