"""Wind stress and atmospheric pressure forcing (FP64 oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 2.1 lets the momentum equations carry source terms F_x, F_y, wind
stresses among them, and Sec. 2.3 / Sec. 3.3 drive them with a parametric
hurricane wind and pressure model (GAHM), whose expressions the paper does
not print.  This module uses the symmetric form of the vortex that GAHM
generalises (Holland 1980), plus a uniform background wind, and the usual
depth-integrated forms of the two forces:

    F = tau_s / rho_w - (H / rho_w) grad p_a
      = (rho_a / rho_w) C_d |W| W - g H grad psi,      psi = (p_a - p_n) / (rho_w g).

Storm records (t, xc, yc, dp, rm, B, wf, wbx, wby) are interpolated
linearly in time (held before the first and after the last record) and
evaluated once per time step at t^n, at the mesh nodes, like the rain
(Sec. 2.5).  At distance r from the centre, with s = (rm / r)^B:

    p_a - p_n = -dp (1 - exp(-s))                      (pressure deficit dp)
    V         = sqrt(B dp s exp(-s) / rho_a)           (cyclostrophic wind)
    W         = wf V (-(y - yc), x - xc) / r + (wbx, wby)

i.e. counter-clockwise circulation (northern hemisphere).  V peaks at
r = rm with sqrt(B dp / (rho_a e)).  Drag: C_d = (0.75 + 0.067 |W|) 1e-3,
capped at 3.5e-3.  rho_a = 1.15 kg/m^3, rho_w = 1000 kg/m^3.

Inside an element the nodal stress and psi are linear (the element is
linear in x, y), so grad psi is constant per element; the sources are taken
at the area points of the quadrature rule, with H = zeta + h_b there.
"""
from __future__ import annotations

import numpy as np

from .forcing import interp_records

RHO_AIR = 1.15
RHO_WATER = 1000.0
CD_MAX = 3.5e-3


def drag_coefficient(speed):
    return np.minimum((0.75 + 0.067 * np.asarray(speed, dtype=np.float64)) * 1e-3, CD_MAX)


def vortex(x, y, xc, yc, dp, rm, B, wf, wbx, wby):
    """Wind (Wx, Wy) in m/s and pressure anomaly p_a - p_n in Pa at (x, y)."""
    dx = np.asarray(x, dtype=np.float64) - xc
    dy = np.asarray(y, dtype=np.float64) - yc
    r = np.hypot(dx, dy)
    rs = np.maximum(r, 1e-6 * rm)          # the centre itself: s huge, exp(-s) = 0
    s = (rm / rs) ** B
    e = np.exp(-s)
    dpa = -dp * (1.0 - e)
    V = np.sqrt(B * dp * s * e / RHO_AIR)
    Wx = wf * V * (-dy) / rs + wbx
    Wy = wf * V * dx / rs + wby
    return Wx, Wy, dpa


def stress_and_head(x, y, rec, g):
    """Nodal kinematic stress tau_s / rho_w and pressure head psi."""
    Wx, Wy, dpa = vortex(x, y, *rec)
    sp = np.hypot(Wx, Wy)
    k = (RHO_AIR / RHO_WATER) * drag_coefficient(sp) * sp
    return k * Wx, k * Wy, dpa / (RHO_WATER * g)


def met_nodes(records, xy, t, g):
    """(tau_x, tau_y, psi) at every node for storm records at time t."""
    rec = np.asarray(records, dtype=np.float64).reshape(-1, 9)
    v, _, _, _ = interp_records(rec[:, 0], rec[:, 1:], t)
    return stress_and_head(xy[:, 0], xy[:, 1], v, g)
