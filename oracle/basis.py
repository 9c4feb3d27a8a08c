"""Dubiner orthogonal modal basis and quadrature on the reference triangle.

Sec. 2.2, Eq. dubiner: the solution is expanded in an orthogonal Dubiner
basis phi_ij of polynomial order i + j, which makes the element mass matrix
diagonal; higher order is obtained by adding terms.

Reference triangle: vertices v0 = (-1,-1), v1 = (1,-1), v2 = (-1,1).  The
collapsed coordinate is a = 2 (1 + r) / (1 - s) - 1 and

    phi_ij(r, s) = P_i(a) ((1 - s)/2)^i  P_j^{(2i+1, 0)}(s),

with P_i the Legendre and P_j^{(alpha,0)} the Jacobi polynomials.  The
product P_i(a) ((1-s)/2)^i is a polynomial in (r, s); it is evaluated with
the homogeneous Legendre recurrence in x = r + (1 + s)/2 and b = (1 - s)/2,
which avoids the coordinate singularity at v2.  Modes are ordered by total
order and, inside one order, by decreasing i:
(0,0), (1,0), (0,1), (2,0), (1,1), (0,2).
"""
from __future__ import annotations

import numpy as np

REF_VERTS = np.array([[-1.0, -1.0], [1.0, -1.0], [-1.0, 1.0]])
REF_AREA = 2.0


def n_modes(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def mode_list(p: int):
    out = []
    for d in range(p + 1):
        for i in range(d, -1, -1):
            out.append((i, d - i))
    return out


def mass_diag(p: int) -> np.ndarray:
    """Closed-form diagonal mass: int phi_ij^2 = 2 / ((2i+1)(i+j+1))."""
    return np.array([2.0 / ((2 * i + 1) * (i + j + 1)) for i, j in mode_list(p)])


def jacobi(n: int, alpha: float, beta: float, x):
    """P_n^{(alpha,beta)}(x) by the standard three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if n == 0:
        return p0
    p1 = 0.5 * ((alpha + beta + 2.0) * x + (alpha - beta))
    for k in range(2, n + 1):
        a1 = 2.0 * k * (k + alpha + beta) * (2.0 * k + alpha + beta - 2.0)
        a2 = (2.0 * k + alpha + beta - 1.0) * (alpha * alpha - beta * beta)
        a3 = (2.0 * k + alpha + beta - 2.0) * (2.0 * k + alpha + beta - 1.0) * (2.0 * k + alpha + beta)
        a4 = 2.0 * (k + alpha - 1.0) * (k + beta - 1.0) * (2.0 * k + alpha + beta)
        p0, p1 = p1, ((a2 + a3 * x) * p1 - a4 * p0) / a1
    return p1


def djacobi(n: int, alpha: float, beta: float, x):
    """d/dx P_n^{(alpha,beta)} = (n + alpha + beta + 1)/2 P_{n-1}^{(alpha+1,beta+1)}."""
    x = np.asarray(x, dtype=np.float64)
    if n == 0:
        return np.zeros_like(x)
    return 0.5 * (n + alpha + beta + 1.0) * jacobi(n - 1, alpha + 1.0, beta + 1.0, x)


def _collapsed_legendre(i: int, r, s):
    """Q_i = P_i(a) b^i with its r- and s-derivatives (forward mode)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    x = r + 0.5 * (1.0 + s)
    b = 0.5 * (1.0 - s)
    # (value, d/dx, d/db)
    q0 = (np.ones_like(r), np.zeros_like(r), np.zeros_like(r))
    if i == 0:
        q = q0
    else:
        q1 = (x.copy(), np.ones_like(r), np.zeros_like(r))
        for n in range(1, i):
            v = ((2 * n + 1) * x * q1[0] - n * b * b * q0[0]) / (n + 1)
            dx = ((2 * n + 1) * (q1[0] + x * q1[1]) - n * b * b * q0[1]) / (n + 1)
            db = ((2 * n + 1) * x * q1[2] - n * (2.0 * b * q0[0] + b * b * q0[2])) / (n + 1)
            q0, q1 = q1, (v, dx, db)
        q = q1
    val, dqx, dqb = q
    # dx/dr = 1, dx/ds = 1/2, db/ds = -1/2
    return val, dqx, 0.5 * dqx - 0.5 * dqb


def eval_basis(p: int, r, s):
    """phi, dphi/dr, dphi/ds with shape (n_modes, *r.shape)."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    phi, dr, ds = [], [], []
    for i, j in mode_list(p):
        q, qr, qs = _collapsed_legendre(i, r, s)
        pj = jacobi(j, 2.0 * i + 1.0, 0.0, s)
        dpj = djacobi(j, 2.0 * i + 1.0, 0.0, s)
        phi.append(q * pj)
        dr.append(qr * pj)
        ds.append(qs * pj + q * dpj)
    return np.array(phi), np.array(dr), np.array(ds)


# ---------------------------------------------------------------------------
# quadrature (the paper does not name its rules; the choice is a reading)
# ---------------------------------------------------------------------------
def area_rule(p: int):
    """Area rule on the reference triangle: points (r, s) and weights.

    p <= 1: the 3-point interior rule with barycentric points
    (2/3,1/6,1/6) and permutations, weight 2/3 each (exact for degree 2).
    p = 2, 3: Gauss-Legendre (p+1) x (p+1) mapped by the Duffy collapse
    r = (1 + a)(1 - b)/2 - 1, s = b with Jacobian (1 - b)/2 (exact for
    degree 2p: 4 and 6).  Points are listed with b outermost.
    """
    if p <= 1:
        bary = np.array([[2 / 3, 1 / 6, 1 / 6], [1 / 6, 2 / 3, 1 / 6], [1 / 6, 1 / 6, 2 / 3]])
        pts = bary @ REF_VERTS
        w = np.full(3, REF_AREA / 3.0)
        return pts[:, 0].copy(), pts[:, 1].copy(), w
    if p in (2, 3):
        n = p + 1
        a, wa = np.polynomial.legendre.leggauss(n)
        rs, ss, ws = [], [], []
        for ib in range(n):
            for ia in range(n):
                b = a[ib]
                rs.append(0.5 * (1.0 + a[ia]) * (1.0 - b) - 1.0)
                ss.append(b)
                ws.append(wa[ia] * wa[ib] * 0.5 * (1.0 - b))
        return np.array(rs), np.array(ss), np.array(ws)
    raise ValueError("p must be 0, 1, 2 or 3")


def edge_rule(p: int):
    """(p+1)-point Gauss-Legendre on t in [-1, 1], ascending t."""
    return np.polynomial.legendre.leggauss(p + 1)


def edge_point(k: int, t):
    """Reference point on local edge k (v_k -> v_{k+1}) at parameter t."""
    t = np.asarray(t, dtype=np.float64)
    va, vb = REF_VERTS[k], REF_VERTS[(k + 1) % 3]
    return (0.5 * (1.0 - t) * va[0] + 0.5 * (1.0 + t) * vb[0],
            0.5 * (1.0 - t) * va[1] + 0.5 * (1.0 + t) * vb[1])


def barycentric(r, s):
    """Barycentric coordinates of (r, s) with respect to v0, v1, v2."""
    r = np.asarray(r, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    return -0.5 * (r + s), 0.5 * (1.0 + r), 0.5 * (1.0 + s)


class Tables:
    """All basis values the solver needs for one p."""

    def __init__(self, p: int):
        self.p = p
        self.np = n_modes(p)
        self.mass = mass_diag(p)
        self.qr, self.qs, self.qw = area_rule(p)
        self.phi_q, self.dphi_dr_q, self.dphi_ds_q = eval_basis(p, self.qr, self.qs)   # (Np, nq)
        self.lam_q = np.array(barycentric(self.qr, self.qs))                           # (3, nq)
        self.gt, self.gw = edge_rule(p)
        ng = len(self.gt)
        self.phi_e = np.zeros((3, ng, self.np))
        self.lam_e = np.zeros((3, ng, 3))
        for k in range(3):
            er, es = edge_point(k, self.gt)
            self.phi_e[k] = eval_basis(p, er, es)[0].T
            self.lam_e[k] = np.array(barycentric(er, es)).T
        # vertex values of the first three (linear) modes and their inverse
        self.phi_v = eval_basis(p, REF_VERTS[:, 0], REF_VERTS[:, 1])[0].T             # (3, Np)
        n1 = min(3, self.np)
        self.V1 = self.phi_v[:, :n1]
        self.V1inv = np.linalg.inv(self.V1) if n1 == 3 else None
        # edge midpoints (for the slope limiter and the p=2 depth test)
        mids = np.array([0.5 * (REF_VERTS[k] + REF_VERTS[(k + 1) % 3]) for k in range(3)])
        self.phi_m = eval_basis(p, mids[:, 0], mids[:, 1])[0].T                        # (3, Np)
        self.lam_m = np.array(barycentric(mids[:, 0], mids[:, 1])).T                   # (3, 3)
