"""Brute-force, element-by-element version of the oracle (tiny meshes only).

TEST INFRASTRUCTURE ONLY.  The vectorised oracle in :mod:`oracle.solver` is
checked against this plain-loop version on meshes of a few dozen elements:
it rebuilds connectivity with a dictionary, evaluates every trace, flux,
quadrature sum, positive-depth step and limiter step one element (and one
point) at a time with Python floats, so indexing and broadcasting mistakes
in the vectorised code show up as disagreements.  It uses the pinned basis
tables and the pinned point fluxes of :mod:`oracle.physics`.
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, physics, forcing

LAND, OCEAN, RIVER, OUTFLOW = 0, 1, 2, 3


def _flux(kind, a, b, hb, nx, ny, g, H0):
    F = physics.numerical_flux(kind, np.array(a, float).reshape(3, 1), np.array(b, float).reshape(3, 1),
                               np.array([hb]), np.array([nx]), np.array([ny]), g, H0)
    return [float(F[0, 0]), float(F[1, 0]), float(F[2, 0])]


def _fn(w, hb, nx, ny, g, H0):
    F = physics.flux_n(w[0], w[1], w[2], hb, nx, ny, g, H0)
    return [float(F[0]), float(F[1]), float(F[2])]


class LoopSolver:
    def __init__(self, xy, tri, hb, fric, bedges, btype, bslot, *, p=1, flux="roe",
                 friction="manning", limiter=False, H0=1e-3, g=9.81, tides=None, rivers=None):
        self.xy = [tuple(map(float, q)) for q in np.asarray(xy)]
        self.hbn = [float(v) for v in hb]
        self.p, self.kind, self.fric_kind = p, flux, friction
        self.use_lim, self.H0, self.g = limiter, float(H0), float(g)
        self.H_dry = self.H0 * (1.0 + 1e-3)
        self.F_eps = 1e-3 * self.H0 * math.sqrt(self.g * self.H0)
        self.tides, self.rivers = dict(tides or {}), dict(rivers or {})
        self.T = basis.Tables(p)
        self.tri = []
        for a, b, c in np.asarray(tri):
            (xa, ya), (xb, yb), (xc, yc) = self.xy[a], self.xy[b], self.xy[c]
            if (xb - xa) * (yc - ya) - (yb - ya) * (xc - xa) < 0:
                b, c = c, b
            self.tri.append((int(a), int(b), int(c)))
        self.E = len(self.tri)
        edges = {}
        for e, t in enumerate(self.tri):
            for k in range(3):
                key = tuple(sorted((t[k], t[(k + 1) % 3])))
                edges.setdefault(key, []).append((e, k))
        bmap = {}
        for (a, b), ty, sl in zip(np.asarray(bedges), btype, bslot):
            bmap[tuple(sorted((int(a), int(b))))] = (int(ty), int(sl))
        self.nb = [[None] * 3 for _ in range(self.E)]
        for key, lst in edges.items():
            if len(lst) == 2:
                (e1, k1), (e2, k2) = lst
                self.nb[e1][k1] = ("in", e2, k2)
                self.nb[e2][k2] = ("in", e1, k1)
            else:
                e1, k1 = lst[0]
                self.nb[e1][k1] = ("bd",) + bmap.get(key, (LAND, 0))
        self.fric = []
        self.geo = []
        for t in self.tri:
            f = [float(fric[i]) for i in t]
            self.fric.append((f[0] + f[1] + f[2]) / 3.0)
            P = [self.xy[i] for i in t]
            J = [[0.5 * (P[1][0] - P[0][0]), 0.5 * (P[2][0] - P[0][0])],
                 [0.5 * (P[1][1] - P[0][1]), 0.5 * (P[2][1] - P[0][1])]]
            det = J[0][0] * J[1][1] - J[0][1] * J[1][0]
            JiT = [[J[1][1] / det, -J[1][0] / det], [-J[0][1] / det, J[0][0] / det]]
            el = []
            for k in range(3):
                dx = P[(k + 1) % 3][0] - P[k][0]
                dy = P[(k + 1) % 3][1] - P[k][1]
                L = math.hypot(dx, dy)
                el.append((L, dy / L, -dx / L))
            self.geo.append((P, det, JiT, el))

    # ---------------------------------------------------------------- helpers
    def _hb_at(self, e, lam):
        t = self.tri[e]
        return sum(lam[i] * self.hbn[t[i]] for i in range(3))

    def _trace(self, w, e, k, gidx):
        return [sum(w[e][v][m] * self.T.phi_e[k][gidx][m] for m in range(self.T.np)) for v in range(3)]

    def _wall(self, a, hb, nx, ny):
        qn = a[1] * nx + a[2] * ny
        return _flux(self.kind, a, [a[0], a[1] - 2 * qn * nx, a[2] - 2 * qn * ny], hb, nx, ny, self.g, self.H0)

    # -------------------------------------------------------------------- RHS
    def rhs(self, w, t, R, dry):
        T, g, H0 = self.T, self.g, self.H0
        ng = len(T.gt)
        L = []
        bout = bin_ = 0.0
        for e in range(self.E):
            P, det, JiT, el = self.geo[e]
            edge = [[0.0] * T.np for _ in range(3)]
            for k in range(3):
                ell, nx, ny = el[k]
                info = self.nb[e][k]
                fmass = 0.0
                for gi in range(ng):
                    hb = self._hb_at(e, T.lam_e[k][gi])
                    a = self._trace(w, e, k, gi)
                    if info[0] == "bd":
                        ty, sl = info[1], info[2]
                        qn = a[1] * nx + a[2] * ny
                        if ty == LAND:
                            F = self._wall(a, hb, nx, ny)
                        elif ty == OUTFLOW:
                            F = _fn(a, hb, nx, ny, g, H0)
                        elif ty == OCEAN:
                            lev = forcing.tide_level(self.tides.get(sl, (0.0, np.zeros((0, 3)))), t)
                            F = _flux(self.kind, a, [lev, a[1], a[2]], hb, nx, ny, g, H0)
                        else:
                            qr = forcing.river_flux(self.rivers[sl], t)
                            qg = 2 * qr - qn
                            F = _flux(self.kind, a, [a[0], a[1] + (qg - qn) * nx, a[2] + (qg - qn) * ny],
                                      hb, nx, ny, g, H0)
                            F[0] = qr
                        fmass += 0.5 * ell * T.gw[gi] * F[0]
                    else:
                        _, n2, k2 = info
                        b = self._trace(w, n2, k2, ng - 1 - gi)
                        F = self._interior(a, b, dry[e], dry[n2], hb, nx, ny)
                    for v in range(3):
                        for m in range(T.np):
                            edge[v][m] += 0.5 * ell * T.gw[gi] * F[v] * T.phi_e[k][gi][m]
                if info[0] == "bd":
                    if fmass > 0:
                        bout += fmass
                    else:
                        bin_ -= fmass
            # area integrals
            dhr = 0.5 * (self.hbn[self.tri[e][1]] - self.hbn[self.tri[e][0]])
            dhs = 0.5 * (self.hbn[self.tri[e][2]] - self.hbn[self.tri[e][0]])
            dhx = JiT[0][0] * dhr + JiT[0][1] * dhs
            dhy = JiT[1][0] * dhr + JiT[1][1] * dhs
            vol = [[0.0] * T.np for _ in range(3)]
            for q in range(len(T.qw)):
                wq = [sum(w[e][v][m] * T.phi_q[m][q] for m in range(T.np)) for v in range(3)]
                hb = self._hb_at(e, T.lam_q[:, q])
                H = wq[0] + hb
                Hs = max(H, H0)
                u, vv = wq[1] / Hs, wq[2] / Hs
                Pp = 0.5 * g * wq[0] * (wq[0] + 2 * hb)
                Fx = [wq[1], wq[1] * u + Pp, wq[2] * u]
                Fy = [wq[2], wq[1] * vv, wq[2] * vv + Pp]
                sp = math.hypot(wq[1], wq[2]) / Hs
                if self.fric_kind == "manning":
                    tau = g * self.fric[e] ** 2 * sp / (Hs * Hs ** (1.0 / 3.0))
                else:
                    tau = self.fric[e] * sp / Hs
                S = [R[e], g * wq[0] * dhx - tau * wq[1], g * wq[0] * dhy - tau * wq[2]]
                for m in range(T.np):
                    dx = JiT[0][0] * T.dphi_dr_q[m][q] + JiT[0][1] * T.dphi_ds_q[m][q]
                    dy = JiT[1][0] * T.dphi_dr_q[m][q] + JiT[1][1] * T.dphi_ds_q[m][q]
                    for v in range(3):
                        vol[v][m] += T.qw[q] * det * (dx * Fx[v] + dy * Fy[v] + S[v] * T.phi_q[m][q])
            L.append([[(vol[v][m] - edge[v][m]) / (det * T.mass[m]) for m in range(T.np)] for v in range(3)])
        return L, (bout, bin_)

    def _interior(self, a, b, dry_me, dry_nb, hb, nx, ny):
        """Outward flux for this element at one Gauss point."""
        g, H0 = self.g, self.H0
        if not dry_me and not dry_nb:
            return _flux(self.kind, a, b, hb, nx, ny, g, H0)
        if dry_me and dry_nb:
            return self._wall(a, hb, nx, ny)
        if not dry_me:          # me wet, neighbour dry
            F = _flux(self.kind, a, [b[0], 0.0, 0.0], hb, nx, ny, g, H0)
            return F if F[0] > self.F_eps else self._wall(a, hb, nx, ny)
        # me dry, neighbour wet: seen from the neighbour's side
        F = _flux(self.kind, b, [a[0], 0.0, 0.0], hb, -nx, -ny, g, H0)
        return [-x for x in F] if F[0] > self.F_eps else self._wall(a, hb, nx, ny)

    # ------------------------------------------------------------------- post
    def post(self, w):
        T, H0 = self.T, self.H0
        w = [[list(row) for row in we] for we in w]
        if self.use_lim:
            w = self._limit(w)
        dry = []
        for e in range(self.E):
            t = self.tri[e]
            hbv = [self.hbn[i] for i in t]
            if self.p >= 2:
                trunc = False
                for i in range(3):
                    Hv = sum(w[e][0][m] * T.phi_v[i][m] for m in range(T.np)) + hbv[i]
                    Hm = sum(w[e][0][m] * T.phi_m[i][m] for m in range(T.np)) + 0.5 * (hbv[i] + hbv[(i + 1) % 3])
                    if Hv <= self.H_dry or Hm <= self.H_dry:
                        trunc = True
                if trunc:
                    for v in range(3):
                        for m in range(3, T.np):
                            w[e][v][m] = 0.0
            vals = [[sum(w[e][v][m] * T.phi_v[i][m] for m in range(T.np)) for i in range(3)] for v in range(3)]
            H = [vals[0][i] + hbv[i] for i in range(3)]
            S = H[0] + H[1] + H[2]
            if all(h >= H0 for h in H):
                Hn, chg = H, False
            elif S / 3.0 <= H0:
                Hn, chg = [S / 3.0] * 3, True
            else:
                order = sorted(range(3), key=lambda i: (H[i], i))
                Hn = [0.0] * 3
                Hn[order[0]] = H0
                Hn[order[1]] = max(H0, H[order[1]] - (H0 - H[order[0]]) / 2.0)
                Hn[order[2]] = S - Hn[order[0]] - Hn[order[1]]
                chg = True
            if chg:
                z = [Hn[i] - hbv[i] for i in range(3)]
                for m in range(3):
                    w[e][0][m] = sum(T.V1inv[m][i] * z[i] for i in range(3))
            d = [Hn[i] <= self.H_dry for i in range(3)]
            nd = sum(d)
            if nd:
                for v in (1, 2):
                    q = vals[v]
                    if nd == 3:
                        qn = [0.0, 0.0, 0.0]
                    else:
                        delta = sum(q[i] for i in range(3) if d[i])
                        qn = [0.0 if d[i] else q[i] + delta / (3 - nd) for i in range(3)]
                    for m in range(3):
                        w[e][v][m] = sum(T.V1inv[m][i] * qn[i] for i in range(3))
            dry.append(nd == 3)
        return w, dry

    def _limit(self, w):
        T, H0 = self.T, self.H0
        full = []
        for e in range(self.E):
            hbv = [self.hbn[i] for i in self.tri[e]]
            fw = all(sum(w[e][0][m] * T.phi_v[i][m] for m in range(T.np)) + hbv[i] > self.H_dry for i in range(3))
            if self.p >= 2:
                fw = fw and w[e][0][0] + (hbv[0] + hbv[1] + hbv[2]) / 3.0 > self.H_dry
            full.append(fw)
        cen = [tuple(sum(P[i][d] for i in range(3)) / 3.0 for d in range(2)) for P, _, _, _ in self.geo]
        out = [[list(r) for r in we] for we in w]
        pinv = np.linalg.pinv(T.phi_m[:, 1:3])
        for e in range(self.E):
            if any(x[0] != "in" for x in self.nb[e]):
                continue
            nbs = [x[1] for x in self.nb[e]]
            if not full[e] or not all(full[n] for n in nbs):
                continue
            P = self.geo[e][0]
            choice = []
            for i in range(3):
                mx = 0.5 * (P[i][0] + P[(i + 1) % 3][0]) - cen[e][0]
                my = 0.5 * (P[i][1] + P[(i + 1) % 3][1]) - cen[e][1]
                got = None
                for off in (1, 2):
                    j, k = i, (i + off) % 3
                    ax, ay = cen[nbs[j]][0] - cen[e][0], cen[nbs[j]][1] - cen[e][1]
                    bx, by = cen[nbs[k]][0] - cen[e][0], cen[nbs[k]][1] - cen[e][1]
                    det = ax * by - ay * bx
                    if det == 0.0:
                        continue
                    aj = (mx * by - my * bx) / det
                    ak = (ax * my - ay * mx) / det
                    if aj >= 0.0 and ak >= 0.0:
                        got = (j, k, aj, ak)
                        break
                choice.append(got)
            if any(c is None for c in choice):
                continue
            for v in range(3):
                wb = w[e][v][0]
                d = [w[e][v][1] * T.phi_m[i][1] + w[e][v][2] * T.phi_m[i][2] for i in range(3)]
                D = []
                for i, (j, k, aj, ak) in enumerate(choice):
                    db = 1.5 * (aj * (w[nbs[j]][v][0] - wb) + ak * (w[nbs[k]][v][0] - wb))
                    a = d[i]
                    D.append(math.copysign(min(abs(a), abs(db)), a) if (a > 0 and db > 0) or (a < 0 and db < 0) else 0.0)
                if all(D[i] == d[i] for i in range(3)):
                    continue
                s = D[0] + D[1] + D[2]
                if s != 0.0:
                    Pp = sum(max(0.0, x) for x in D)
                    Nn = sum(max(0.0, -x) for x in D)
                    tp = 1.0 if Pp == 0.0 else min(1.0, Nn / Pp)
                    tn = 1.0 if Nn == 0.0 else min(1.0, Pp / Nn)
                    D = [tp * max(0.0, x) - tn * max(0.0, -x) for x in D]
                lin = pinv @ np.array(D)
                out[e][v][1], out[e][v][2] = float(lin[0]), float(lin[1])
                for m in range(3, T.np):
                    out[e][v][m] = 0.0
        return out
