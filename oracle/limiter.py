"""Optional slope limiter (Sec. 2.3), FP64, vectorised.

The paper states only that an optional slope limiter is available for flows
with shocks and cites Cockburn and Shu for the Runge-Kutta DG framework.
The limiter used is the Cockburn-Shu triangle limiter, applied
componentwise to (zeta, qx, qy) on the linear part of the solution:

  for each edge midpoint m_i of element 0 with barycentre b_0, write
  m_i - b_0 = a_j (b_j - b_0) + a_k (b_k - b_0) with a_j, a_k >= 0, using
  the barycentres of the neighbour across edge i and one other neighbour;
  the limited midpoint deviation is
      D_i = minmod( w(m_i) - wbar_0 , nu [a_j (wbar_j - wbar_0) + a_k (wbar_k - wbar_0)] )
  with nu = 1.5 (no TVB constant).  If every D_i equals the unlimited
  deviation the element is left untouched.  Otherwise, if the D_i do not sum
  to zero, positive and negative parts are scaled by min(1, N/P) and
  min(1, P/N) (P, N the sums of the positive and negative parts), and the
  linear part is rebuilt from the mean and the three deviations (least
  squares over the three midpoints; exact when they sum to zero).  For
  p = 2 a limited component also loses its quadratic modes.

Elements with a boundary edge, or whose barycentre decomposition has no
non-negative pair, are not limited.  minmod(0, .) = 0.
"""
from __future__ import annotations

import numpy as np

NU = 1.5


def stencil(g):
    """Per element and midpoint: neighbour slots (j, k), weights (a_j, a_k).

    Returns (ok (E,), jk (E,3,2) int, alpha (E,3,2)).
    """
    nbr = g["nbr"]
    verts = g["verts"]
    E = nbr.shape[0]
    cen = (verts[:, 0] + verts[:, 1] + verts[:, 2]) / 3.0
    ok = np.all(nbr >= 0, axis=1)
    jk = np.zeros((E, 3, 2), dtype=np.int64)
    alpha = np.zeros((E, 3, 2))
    safe = np.where(nbr >= 0, nbr, 0)
    bn = cen[safe]                                      # (E, 3, 2) neighbour barycentres
    for i in range(3):
        mid = 0.5 * (verts[:, i] + verts[:, (i + 1) % 3])
        mx, my = mid[:, 0] - cen[:, 0], mid[:, 1] - cen[:, 1]
        found = np.zeros(E, dtype=bool)
        for off in (1, 2):
            j, k = i, (i + off) % 3
            ax, ay = bn[:, j, 0] - cen[:, 0], bn[:, j, 1] - cen[:, 1]
            bx, by = bn[:, k, 0] - cen[:, 0], bn[:, k, 1] - cen[:, 1]
            det = ax * by - ay * bx
            with np.errstate(divide="ignore", invalid="ignore"):
                aj = (mx * by - my * bx) / det
                ak = (ax * my - ay * mx) / det
            good = (~found) & (det != 0.0) & (aj >= 0.0) & (ak >= 0.0)
            jk[good, i] = (j, k)
            alpha[good, i, 0] = aj[good]
            alpha[good, i, 1] = ak[good]
            found |= good
        ok &= found
    return ok, jk, alpha


def minmod(a, b):
    same = ((a > 0) & (b > 0)) | ((a < 0) & (b < 0))
    return np.where(same, np.sign(a) * np.minimum(np.abs(a), np.abs(b)), 0.0)


def apply(w, g, st, tables, active=None):
    """Limit the state w (E, 3, Np) in place and return it.

    ``active`` (E,) restricts limiting to the marked elements.
    """
    ok, jk, alpha = st
    nbr = g["nbr"]
    if active is not None:
        ok = ok & active
    idx = np.nonzero(ok)[0]
    if idx.size == 0:
        return w
    wbar = w[:, :, 0]                                   # phi_00 = 1: mode 0 is the mean
    phim = tables.phi_m[:, 1:3]                          # (3 midpoints, 2 linear modes)
    pinv = np.linalg.pinv(phim)                          # (2, 3)
    we = w[idx]                                          # (n, 3, Np)
    d = np.einsum("nvm,im->nvi", we[:, :, 1:3], phim)   # unlimited deviations
    nb = nbr[idx]                                        # (n, 3)
    wb0 = wbar[idx]                                      # (n, 3 vars)
    dbar = np.zeros_like(d)
    for i in range(3):
        j = nb[np.arange(idx.size), jk[idx, i, 0]]
        k = nb[np.arange(idx.size), jk[idx, i, 1]]
        dbar[:, :, i] = (alpha[idx, i, 0][:, None] * (wbar[j] - wb0)
                         + alpha[idx, i, 1][:, None] * (wbar[k] - wb0))
    D = minmod(d, NU * dbar)
    same = np.all(D == d, axis=2)                        # (n, vars)
    s = D[:, :, 0] + D[:, :, 1] + D[:, :, 2]
    P = np.maximum(D, 0.0).sum(axis=2)
    N = np.maximum(-D, 0.0).sum(axis=2)
    resc = (~same) & (s != 0.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        tp = np.where(resc, np.minimum(1.0, N / np.where(P > 0, P, 1.0)), 1.0)
        tn = np.where(resc, np.minimum(1.0, P / np.where(N > 0, N, 1.0)), 1.0)
    tp = np.where(resc & (P == 0.0), 1.0, tp)
    tn = np.where(resc & (N == 0.0), 1.0, tn)
    Dr = tp[:, :, None] * np.maximum(D, 0.0) - tn[:, :, None] * np.maximum(-D, 0.0)
    D = np.where(resc[:, :, None], Dr, D)
    lin = np.einsum("li,nvi->nvl", pinv, D)              # (n, vars, 2)
    changed = ~same
    new = we.copy()
    new[:, :, 1:3] = np.where(changed[:, :, None], lin, we[:, :, 1:3])
    if we.shape[2] > 3:
        new[:, :, 3:] = np.where(changed[:, :, None], 0.0, we[:, :, 3:])
    w[idx] = new
    return w
