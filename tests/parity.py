"""Helpers shared by the GPU parity tests (comparison norms only).

Parity norm: at vertex values (p = 1) or area-point values (p = 2),
  err_zeta = ||zeta_gpu - zeta_orc|| / max(||zeta_orc||, 1e-3 sqrt(n) D)
  err_q    = ||q_gpu - q_orc||       / max(||q_orc||,    1e-3 sqrt(n) D c)
with q the discharge vector (qx, qy) at every point, D the RMS water depth
of the oracle state and c = sqrt(g D).  The momentum error is taken on the
vector field, so that a component that vanishes identically (a 1-D flow)
does not turn round-off into a relative error of order one; the floors keep
a fluid at rest from dividing by round-off.
"""
import numpy as np

from oracle import basis


def point_values(w, p):
    """Vertex values (p <= 1) or area-point values (p = 2) of modal states."""
    if p == 2:
        T = basis.Tables(2)
        return np.einsum("evm,mq->evq", w, T.phi_q)
    T = basis.Tables(1)
    return np.einsum("evm,im->evi", w[:, :, :3], T.phi_v)


def point_hb(orc):
    if orc.p == 2:
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
