"""Physical flux, numerical fluxes and bottom friction (FP64, vectorised).

State at a point: w = (zeta, qx, qy) with qx = H u, qy = H v and
H = zeta + hb (Sec. 2.2).  The flux matrix is

    F(w) = [[qx, qy], [qx u + P, qx v], [qy u, qy v + P]],
    P    = g/2 (H^2 - hb^2) = g/2 zeta (zeta + 2 hb),

i.e. the pressure term of Eq. SWE (the flux matrix printed in Sec. 2.2
drops the factor 1/2; Eq. SWE is followed).  The second form is the same
polynomial without the cancellation of H^2 - hb^2 in deep water.

Velocities are q / max(H, H0) (thin-layer reading: a dry point has a
vanishing velocity, not an infinite one).  Wave speeds use sqrt(g max(H,0)).

Numerical fluxes (Sec. 2.3 names Roe and local Lax-Friedrichs):
  * LLF:  Fhat = (Fn(w-) + Fn(w+))/2 - lam/2 (w+ - w-),
          lam = max(|un-| + c-, |un+| + c+);
  * Roe:  textbook Roe linearisation in the frame (n, t) with
          Roe-averaged velocity and c~ = sqrt(g (H- + H+)/2), no entropy fix.
"""
from __future__ import annotations

import numpy as np


def flux_xy(zeta, qx, qy, hb, g, H0):
    H = zeta + hb
    Hs = np.maximum(H, H0)
    u, v = qx / Hs, qy / Hs
    P = 0.5 * g * zeta * (zeta + 2.0 * hb)
    Fx = np.stack([qx, qx * u + P, qy * u])
    Fy = np.stack([qy, qx * v, qy * v + P])
    return Fx, Fy


def flux_n(zeta, qx, qy, hb, nx, ny, g, H0):
    """Normal flux F(w).n, shape (3, ...)."""
    H = zeta + hb
    Hs = np.maximum(H, H0)
    qn = qx * nx + qy * ny
    un = qn / Hs
    P = 0.5 * g * zeta * (zeta + 2.0 * hb)
    return np.stack([qn, qx * un + P * nx, qy * un + P * ny])


def llf(wl, wr, hb, nx, ny, g, H0):
    """Local Lax-Friedrichs flux.  wl, wr: (3, ...) states; returns (3, ...)."""
    fl = flux_n(wl[0], wl[1], wl[2], hb, nx, ny, g, H0)
    fr = flux_n(wr[0], wr[1], wr[2], hb, nx, ny, g, H0)
    Hl, Hr = wl[0] + hb, wr[0] + hb
    unl = (wl[1] * nx + wl[2] * ny) / np.maximum(Hl, H0)
    unr = (wr[1] * nx + wr[2] * ny) / np.maximum(Hr, H0)
    lam = np.maximum(np.abs(unl) + np.sqrt(g * np.maximum(Hl, 0.0)),
                     np.abs(unr) + np.sqrt(g * np.maximum(Hr, 0.0)))
    return 0.5 * (fl + fr) - 0.5 * lam * (np.asarray(wr) - np.asarray(wl))


def roe(wl, wr, hb, nx, ny, g, H0):
    """Roe flux for the shallow water system (no entropy fix)."""
    fl = flux_n(wl[0], wl[1], wl[2], hb, nx, ny, g, H0)
    fr = flux_n(wr[0], wr[1], wr[2], hb, nx, ny, g, H0)
    Hl = np.maximum(wl[0] + hb, H0)
    Hr = np.maximum(wr[0] + hb, H0)
    qnl = wl[1] * nx + wl[2] * ny
    qtl = -wl[1] * ny + wl[2] * nx
    qnr = wr[1] * nx + wr[2] * ny
    qtr = -wr[1] * ny + wr[2] * nx
    sl, sr = np.sqrt(Hl), np.sqrt(Hr)
    un = (sl * (qnl / Hl) + sr * (qnr / Hr)) / (sl + sr)
    ut = (sl * (qtl / Hl) + sr * (qtr / Hr)) / (sl + sr)
    c = np.sqrt(0.5 * g * (Hl + Hr))
    dH = wr[0] - wl[0]                 # continuous bathymetry: dH = d zeta
    dqn = qnr - qnl
    dqt = qtr - qtl
    a1 = ((un + c) * dH - dqn) / (2.0 * c)
    a3 = (dqn - (un - c) * dH) / (2.0 * c)
    a2 = dqt - ut * dH
    l1, l2, l3 = np.abs(un - c), np.abs(un), np.abs(un + c)
    # dissipation sum |lam_k| a_k r_k with r1 = (1, un-c, ut), r2 = (0,0,1), r3 = (1, un+c, ut)
    d0 = l1 * a1 + l3 * a3
    dn = l1 * a1 * (un - c) + l3 * a3 * (un + c)
    dt_ = l1 * a1 * ut + l2 * a2 + l3 * a3 * ut
    dx = dn * nx - dt_ * ny
    dy = dn * ny + dt_ * nx
    return 0.5 * (fl + fr) - 0.5 * np.stack([d0, dx, dy])


def numerical_flux(kind, wl, wr, hb, nx, ny, g, H0):
    if kind == "roe":
        return roe(wl, wr, hb, nx, ny, g, H0)
    if kind == "llf":
        return llf(wl, wr, hb, nx, ny, g, H0)
    raise ValueError(kind)


def friction_tau(kind, coef, zeta, qx, qy, hb, g, H0):
    """Bottom friction factor tau_b (Eq. SWE) at points.

    Manning (Sec. 3 uses it in all cases): tau_b = g n^2 |u| / H^{4/3}.
    Quadratic (Sec. 3.1, coefficient 0.001): tau_b = C_f |u| / H.
    H is floored at H0 as for the velocities.
    """
    Hs = np.maximum(zeta + hb, H0)
    speed = np.sqrt(qx * qx + qy * qy) / Hs
    if kind == "manning":
        return g * coef * coef * speed / (Hs * np.cbrt(Hs))
    if kind == "quadratic":
        return coef * speed / Hs
    raise ValueError(kind)
