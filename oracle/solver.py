"""FP64 DG solver for the rain-augmented shallow water equations (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One time step follows the evaluation order of Sec. 2.3: for every stage,
boundary edge integrals, interior edge integrals, forcing (including the
nodal rain of Eq. rain), area integrals, then the new stage solution; the
positive-depth operator of Sec. 2.4 (after the optional limiter) is applied
after every Runge-Kutta stage and once to the initial state.

Per element e with reference-to-physical Jacobian J (Sec. 2.2, Eq.
elem_weak_form with the diagonal Dubiner mass of Eq. dubiner):

    det J m_k dw_k/dt =  sum_q W_q det J grad(phi_k).F(w_q)          (volume)
                       + sum_q W_q det J s(w_q) phi_k(q)               (sources)
                       - sum_edges sum_g (l/2) w_g Fhat_g phi_k(g)     (edges)

with s = (R_e, g zeta dhb/dx - tau_b qx, g zeta dhb/dy - tau_b qy): the
source vector of Sec. 2.2 plus the friction term that Eq. SWE carries on its
left-hand side (the printed source vector omits it); with meteorological
forcing the momentum rows also take F = tau_s/rho_w - g H grad psi.  Sums run over
quadrature points in table order and over local edges 0, 1, 2.

Time integration (Sec. 2.2, Eq. RKSSP; Sec. 3 uses a two-stage second-order
SSPRK): every two-stage second-order explicit RK method has the stability
polynomial 1 + z + z^2/2, and the SSP-optimal one is the Shu-Osher scheme

    w1      = w^n + dt L(w^n, t^n)
    w^{n+1} = w^n/2 + (w1 + dt L(w1, t^n + dt))/2

(:func:`ssp_table` also holds SSP(3,3) for p = 2 and SSP(5,2)).  Boundary
forcing is evaluated at the stage times; rain at t^n for every stage.  dt = dt_fixed if given, else
min(dt_max, CFL min_e d_e / lam_e) with d_e the inscribed-circle diameter and
lam_e the largest |u| + sqrt(g H) over the element's wet vertices.

Readings of silent or garbled points (also listed in the design notes):
  * pressure g/2 (H^2 - hb^2) as in Eq. SWE (the flux matrix drops the 1/2);
  * friction included in the source (Eq. SWE), Manning g n^2 |u| / H^{4/3}
    or quadratic C_f |u| / H, explicit at the area points;
  * bathymetry continuous and linear per element; element friction
    coefficient = mean of the three nodal values;
  * velocities q / max(H, H0); wave speeds sqrt(g max(H, 0));
  * land: mirror the normal discharge; ocean: ghost elevation from the
    tide, discharge copied; river: ghost normal discharge 2 q_river - q_n and
    the mass flux set to q_river exactly; outflow: ghost = interior state;
  * wet/dry edges (Sec. 2.4: flags drive the interaction; the suppressed
    text there mirrors the normal momentum when the condition is violated):
    wet-wet normal; otherwise the wet state (if any) meets the dry state with
    its discharge zeroed, and if that mass flux enters the dry element the
    flux is exchanged, else each side sees a land boundary (its own state
    mirrored), which keeps a dry cell at rest in hydrostatic balance;
    decided per Gauss point; boundary edges ignore the flags;
  * the limiter acts only where the element and its three neighbours have
    every vertex depth > H0 (no limiting across a wet/dry front), and for
    p >= 2 also a mean depth > H0 (a curved element can be wet at its
    vertices and dry on average; the positive-depth pass would then change
    the means the limiter of its neighbours reads);
  * decision margins: the positive-depth operator itself puts vertices at
    exactly H0, and at a front the mass flux between two such traces is pure
    round-off, so the tests that follow it are ties.  Every "is this vertex
    dry / wet" test uses H0 (1 + 1e-3), and a wet-dry edge exchanges water
    only when the mass flux into the dry element exceeds
    1e-3 H0 sqrt(g H0); both margins are far below anything physical and
    above the round-off of FP64 and FP32 arithmetic;
  * p = 2 wet/dry: if any vertex or edge-midpoint depth is <= H0 the element
    is truncated to its linear part before the p = 1 operator;
  * wind stress and atmospheric pressure (F_x, F_y of Eq. SWE, optional):
    nodal kinematic stress and pressure head at t^n (:mod:`oracle.met`),
    linear in each element, taken at the area points as
    tau - g H grad psi with H = zeta + h_b; held for every stage like rain;
  * p = 0 (only used to pin the scheme against a finite-volume code): no
    redistribution; a cell is dry when its mean depth is <= H0.
"""
from __future__ import annotations

import numpy as np

from . import basis, mesh as meshmod, physics, forcing, wetdry, limiter as limmod, met as metmod


def ssp_table(stages):
    """Shu-Osher coefficients (a_i, b_i, g_i, c_i) of the SSP schemes used.

    Stage i: w(i) = a_i w^n + b_i (w(i-1) + g_i dt L(w(i-1), t^n + c_i dt)).
      2 stages: SSP(2,2), the two-stage second-order scheme of Sec. 3;
      3 stages: SSP(3,3), used for p = 2 and p = 3 (a two-stage order-2
                scheme is linearly unstable with p >= 2 elements: its
                stability region holds no segment of the imaginary axis;
                SSP(3,3)'s does, so p = 3 runs at a reduced CFL, 0.1);
      5 stages: SSP(5,2), the optimal five-stage second-order scheme, a
                stand-in for the five-stage scheme used for Hurricane Harvey
                in Sec. 3 (whose optimised coefficients are not given).
    """
    if stages == 2:
        return [(0.0, 1.0, 1.0, 0.0), (0.5, 0.5, 1.0, 1.0)]
    if stages == 3:
        return [(0.0, 1.0, 1.0, 0.0), (0.75, 0.25, 1.0, 1.0), (1.0 / 3.0, 2.0 / 3.0, 1.0, 0.5)]
    if stages == 5:
        return [(0.0, 1.0, 0.25, 0.0), (0.0, 1.0, 0.25, 0.25), (0.0, 1.0, 0.25, 0.5),
                (0.0, 1.0, 0.25, 0.75), (0.2, 0.8, 0.25, 1.0)]
    raise ValueError("rk_stages must be 2, 3 or 5")


def ssp_flux_weights(table):
    """Weight of each stage's L(w(i-1)) in w^{n+1} (they sum to one)."""
    e = []
    for i, (a, b, g, c) in enumerate(table):
        e = [b * x for x in e] + [b * g]
    return e


def ssp_step(w, rhs, dt, table, post=lambda w: w):
    """One SSP step for a generic right-hand side ``rhs(w, stage_index)``."""
    wi = w
    for i, (a, b, g, c) in enumerate(table):
        wi = post(a * w + b * (wi + g * dt * rhs(wi, i)))
    return wi


def ssp_rk2_step(w, rhs, dt, post=lambda w: w):
    return ssp_step(w, rhs, dt, ssp_table(2), post)


class OracleSolver:
    def __init__(self, xy, tri, hb, fric, bedges=None, btype=None, bslot=None, *,
                 p=1, flux="roe", friction="manning", limiter=False, cfl=0.3,
                 dt_fixed=0.0, dt_max=1.0e30, H0=1.0e-3, g=9.81, rk_stages=2,
                 rain=None, tides=None, rivers=None, mms=None, met=None):
        self.rk = ssp_table(int(rk_stages))
        self.rk_weights = ssp_flux_weights(self.rk)
        self.xy = np.asarray(xy, dtype=np.float64)
        self.hb_nodes = np.asarray(hb, dtype=np.float64)
        self.G = meshmod.build(self.xy, tri, bedges, btype, bslot)
        G = self.G
        self.tri = G["tri"]
        self.E = self.tri.shape[0]
        self.p = int(p)
        self.T = basis.Tables(self.p)
        self.flux_kind = flux
        self.friction = friction
        self.use_limiter = bool(limiter)
        self.cfl, self.dt_fixed, self.dt_max = float(cfl), float(dt_fixed), float(dt_max)
        self.H0, self.g = float(H0), float(g)
        # decision margins (see the module docstring): a vertex is dry when
        # H <= H0 (1 + 1e-3); a wet-dry edge exchanges water only when its
        # mass flux into the dry element exceeds 1e-3 H0 sqrt(g H0)
        self.H_dry = self.H0 * (1.0 + 1e-3)
        self.F_eps = 1e-3 * self.H0 * np.sqrt(self.g * self.H0)
        self.hbv = self.hb_nodes[self.tri]                                  # (E, 3)
        fr = np.asarray(fric, dtype=np.float64)[self.tri]
        self.fric_e = (fr[:, 0] + fr[:, 1] + fr[:, 2]) / 3.0
        self.hbar = (self.hbv[:, 0] + self.hbv[:, 1] + self.hbv[:, 2]) / 3.0
        # constant bed gradient: J^{-T} (dhb/dr, dhb/ds)
        dr = 0.5 * (self.hbv[:, 1] - self.hbv[:, 0])
        ds = 0.5 * (self.hbv[:, 2] - self.hbv[:, 0])
        JT = G["JinvT"]
        self.dhb = np.stack([JT[:, 0, 0] * dr + JT[:, 0, 1] * ds,
                             JT[:, 1, 0] * dr + JT[:, 1, 1] * ds], axis=1)
        self.hb_q = self.hbv @ self.T.lam_q                                # (E, nq)
        self.hb_e = np.einsum("ei,kgi->ekg", self.hbv, self.T.lam_e)        # (E, 3, ng)
        self.hb_m = self.hbv @ self.T.lam_m.T                              # (E, 3 midpoints)
        dphx = (JT[:, 0, 0, None, None] * self.T.dphi_dr_q[None]
                + JT[:, 0, 1, None, None] * self.T.dphi_ds_q[None])
        dphy = (JT[:, 1, 0, None, None] * self.T.dphi_dr_q[None]
                + JT[:, 1, 1, None, None] * self.T.dphi_ds_q[None])
        self.dphx, self.dphy = dphx, dphy                                  # (E, Np, nq)
        self.stencil = limmod.stencil(G) if self.use_limiter else None
        self.rain = rain if rain is not None else {"kind": "none"}
        self.tides = dict(tides or {})
        self.rivers = dict(rivers or {})
        self.met = None if met is None else np.asarray(met, dtype=np.float64).reshape(-1, 9)
        self.mms = mms
        # interior edges, once each, canonical side = lower element id
        nbr = G["nbr"]
        e_idx, k_idx = np.nonzero((nbr >= 0) & (nbr > np.arange(self.E)[:, None]))
        self.ie_L, self.ie_kL = e_idx, k_idx
        self.ie_R, self.ie_kR = nbr[e_idx, k_idx], G["nbr_edge"][e_idx, k_idx]
        be, bk = np.nonzero(nbr < 0)
        self.be, self.bk = be, bk
        self.b_type = G["btype"][be, bk]
        self.b_slot = G["bslot"][be, bk]
        # state
        self.w = np.zeros((self.E, 3, self.T.np))
        self.flags = np.zeros(self.E, dtype=bool)
        self.t = 0.0
        self.steps = 0
        self.rain_in = 0.0
        self.bnd_in = 0.0
        self.bnd_out = 0.0
        self.dt = 0.0
        self.last_dt = 0.0

    # ------------------------------------------------------------------ state
    def set_initial_nodal(self, zeta, qx, qy):
        vals = np.stack([np.asarray(a, dtype=np.float64)[self.tri] for a in (zeta, qx, qy)], axis=1)  # (E,3,3)
        w = np.zeros((self.E, 3, self.T.np))
        if self.p == 0:
            w[:, :, 0] = (vals[:, :, 0] + vals[:, :, 1] + vals[:, :, 2]) / 3.0
        else:
            w[:, :, :3] = np.einsum("mi,evi->evm", self.T.V1inv, vals)
        self.set_state(w)

    def set_state(self, w, t=0.0, post=True):
        self.w = np.array(w, dtype=np.float64, copy=True)
        self.t = float(t)
        if post:
            self.w, self.flags = self.post(self.w)
        else:
            self.flags = self._flags_only(self.w)
        self.dt = self.compute_dt(self.w)

    def vertex_values(self, w=None):
        w = self.w if w is None else w
        return np.einsum("evm,im->evi", w, self.T.phi_v)                    # (E, 3 vars, 3 vertices)

    # ----------------------------------------------------------- boundary
    def _ghost(self, wl, types, slots, t, hb, nx, ny):
        """Ghost states for boundary points. wl: (3, nb, ng)."""
        z, qx, qy = wl
        qn = qx * nx + qy * ny
        gz, gx, gy = z.copy(), qx.copy(), qy.copy()
        land = types == meshmod.LAND
        gx = np.where(land[:, None], qx - 2.0 * qn * nx, gx)
        gy = np.where(land[:, None], qy - 2.0 * qn * ny, gy)
        ocean = types == meshmod.OCEAN
        if np.any(ocean):
            lev = np.zeros(len(types))
            for sl in np.unique(slots[ocean]):
                spec = self.tides.get(int(sl), (0.0, np.zeros((0, 3))))
                lev[ocean & (slots == sl)] = forcing.tide_level(spec, t)
            gz = np.where(ocean[:, None], lev[:, None], gz)
        river = types == meshmod.RIVER
        qr = np.zeros(len(types))
        if np.any(river):
            for sl in np.unique(slots[river]):
                qr[river & (slots == sl)] = forcing.river_flux(self.rivers[int(sl)], t)
            qn_g = 2.0 * qr[:, None] - qn
            gx = np.where(river[:, None], qx + (qn_g - qn) * nx, gx)
            gy = np.where(river[:, None], qy + (qn_g - qn) * ny, gy)
        return np.stack([gz, gx, gy]), qr

    # ----------------------------------------------------------------- RHS
    def rhs(self, w, t, R_e, flags, met=None):
        """L(w) and the boundary mass flux (out, in) of this evaluation.

        met: nodal (tau_x, tau_y, psi) of :mod:`oracle.met`, or None.
        """
        T, G = self.T, self.G
        g, H0 = self.g, self.H0
        ng = len(T.gt)
        # traces at every edge Gauss point: (E, 3 edges, ng, 3 vars)
        tr = np.einsum("evm,kgm->ekgv", w, T.phi_e)
        C = np.zeros((self.E, 3, 3, T.np))            # per (element, local edge) contribution
        wg_half = 0.5 * T.gw                           # (l/2) w_g  without l
        # (1) boundary edge integrals
        be, bk = self.be, self.bk
        out_sum = in_sum = 0.0
        if be.size:
            wl = np.moveaxis(tr[be, bk], 2, 0)                         # (3, nb, ng)
            nx = G["normal"][be, bk, 0][:, None] * np.ones(ng)
            ny = G["normal"][be, bk, 1][:, None] * np.ones(ng)
            hb = self.hb_e[be, bk]
            if self.mms is not None:
                gpts = self._edge_xy(be, bk)
                wr = self.mms.ghost(gpts[..., 0], gpts[..., 1], t)
                qr = np.zeros(be.size)
            else:
                wr, qr = self._ghost(wl, self.b_type, self.b_slot, t, hb, nx, ny)
            F = physics.numerical_flux(self.flux_kind, wl, wr, hb, nx, ny, g, H0)
            out_b = self.b_type == meshmod.OUTFLOW
            if np.any(out_b) and self.mms is None:
                Fo = physics.flux_n(wl[0], wl[1], wl[2], hb, nx, ny, g, H0)
                F = np.where(out_b[None, :, None], Fo, F)
            riv = self.b_type == meshmod.RIVER
            if np.any(riv) and self.mms is None:
                F[0] = np.where(riv[:, None], qr[:, None], F[0])
            ell = G["edge_len"][be, bk]
            C[be, bk] = self._edge_contrib(F, ell, bk)
            fmass = ell * (F[0] @ wg_half)
            out_sum = float(np.sum(np.maximum(fmass, 0.0)))
            in_sum = float(np.sum(np.maximum(-fmass, 0.0)))
        # (2) interior edge integrals, once per edge
        L, kL, R, kR = self.ie_L, self.ie_kL, self.ie_R, self.ie_kR
        if L.size:
            wl = np.moveaxis(tr[L, kL], 2, 0)                          # (3, ni, ng)
            wr = np.moveaxis(tr[R, kR][:, ::-1], 2, 0)                 # neighbour runs the edge backwards
            nx = G["normal"][L, kL, 0][:, None] * np.ones(ng)
            ny = G["normal"][L, kL, 1][:, None] * np.ones(ng)
            hb = self.hb_e[L, kL]
            fL, fR = self._interior_flux(wl, wr, flags[L], flags[R], hb, nx, ny)
            ell = G["edge_len"][L, kL]
            C[L, kL] = self._edge_contrib(fL, ell, kL)
            C[R, kR] = self._edge_contrib(fR[:, :, ::-1], ell, kR)
        edge = C[:, 0] + C[:, 1] + C[:, 2]
        # (3) forcing at the area points, (4) area integrals
        wq = np.einsum("evm,mq->veq", w, T.phi_q)                      # (3, E, nq)
        Fx, Fy = physics.flux_xy(wq[0], wq[1], wq[2], self.hb_q, g, H0)
        wdet = T.qw[None, :] * G["detJ"][:, None]                      # (E, nq)
        vol = (np.einsum("eq,emq,veq->evm", wdet, self.dphx, Fx)
               + np.einsum("eq,emq,veq->evm", wdet, self.dphy, Fy))
        tau = physics.friction_tau(self.friction, self.fric_e[:, None], wq[0], wq[1], wq[2],
                                   self.hb_q, g, H0)
        s0 = np.broadcast_to(R_e[:, None], wq[0].shape)
        s1 = g * wq[0] * self.dhb[:, 0:1] - tau * wq[1]
        s2 = g * wq[0] * self.dhb[:, 1:2] - tau * wq[2]
        if met is not None:
            # wind stress and pressure gradient (oracle.met): nodal values
            # linear in the element, H = zeta + h_b at the area points
            tx, ty, psi = (np.asarray(a, dtype=np.float64)[self.tri] for a in met)   # (E, 3) each
            pr = 0.5 * (psi[:, 1] - psi[:, 0])
            ps = 0.5 * (psi[:, 2] - psi[:, 0])
            JT = G["JinvT"]
            px = JT[:, 0, 0] * pr + JT[:, 0, 1] * ps
            py = JT[:, 1, 0] * pr + JT[:, 1, 1] * ps
            Hq = wq[0] + self.hb_q
            s1 = s1 + tx @ T.lam_q - g * Hq * px[:, None]
            s2 = s2 + ty @ T.lam_q - g * Hq * py[:, None]
        S = np.stack([s0, s1, s2])
        if self.mms is not None:
            xq, yq = self._area_xy()
            S = S + self.mms.source(xq, yq, t)
        src = np.einsum("eq,veq,mq->evm", wdet, S, T.phi_q)
        Lw = (vol + src - edge) / (G["detJ"][:, None, None] * T.mass[None, None, :])
        return Lw, (out_sum, in_sum)

    def _edge_contrib(self, F, ell, k):
        """sum_g (l/2) w_g F_g phi_m(edge k, g) for F (3, n, ng) -> (n, 3, Np)."""
        phi = self.T.phi_e[k]                                          # (n, ng, Np)
        return np.einsum("n,g,vng,ngm->nvm", 0.5 * ell, self.T.gw, F, phi)

    def _wall_flux(self, w, hb, nx, ny):
        """Flux of a state against its own mirror image (land boundary)."""
        qn = w[1] * nx + w[2] * ny
        refl = np.stack([w[0], w[1] - 2.0 * qn * nx, w[2] - 2.0 * qn * ny])
        return physics.numerical_flux(self.flux_kind, w, refl, hb, nx, ny, self.g, self.H0)

    def _interior_flux(self, wl, wr, dryL, dryR, hb, nx, ny):
        """Outward fluxes (for L, for R) at the Gauss points of interior edges.

        wet-wet: the numerical flux, opposite signs.  Otherwise the wet
        state (if any) meets the dry state with its discharge zeroed; if the
        resulting mass flux enters the dry element the flux is exchanged,
        else each side sees a land boundary (its own mirrored state).
        """
        g, H0, kind = self.g, self.H0, self.flux_kind
        F = physics.numerical_flux(kind, wl, wr, hb, nx, ny, g, H0)
        fL, fR = F.copy(), -F
        mixLw = (~dryL) & dryR
        mixRw = dryL & (~dryR)
        both = dryL & dryR
        if np.any(both):
            m = both
            fL[:, m] = self._wall_flux(wl[:, m], hb[m], nx[m], ny[m])
            fR[:, m] = self._wall_flux(wr[:, m], hb[m], -nx[m], -ny[m])
        if np.any(mixLw):
            m = mixLw
            a = wl[:, m]
            b = np.stack([wr[0, m], np.zeros_like(wr[0, m]), np.zeros_like(wr[0, m])])
            Fm = physics.numerical_flux(kind, a, b, hb[m], nx[m], ny[m], g, H0)
            into = Fm[0] > self.F_eps
            fL[:, m] = np.where(into, Fm, self._wall_flux(a, hb[m], nx[m], ny[m]))
            fR[:, m] = np.where(into, -Fm, self._wall_flux(wr[:, m], hb[m], -nx[m], -ny[m]))
        if np.any(mixRw):
            m = mixRw
            b = wr[:, m]
            a = np.stack([wl[0, m], np.zeros_like(wl[0, m]), np.zeros_like(wl[0, m])])
            Fm = physics.numerical_flux(kind, a, b, hb[m], nx[m], ny[m], g, H0)
            into = Fm[0] < -self.F_eps
            fL[:, m] = np.where(into, Fm, self._wall_flux(wl[:, m], hb[m], nx[m], ny[m]))
            fR[:, m] = np.where(into, -Fm, self._wall_flux(b, hb[m], -nx[m], -ny[m]))
        return fL, fR

    def _area_xy(self):
        v = self.G["verts"]
        lam = self.T.lam_q
        return (np.einsum("ei,iq->eq", v[..., 0], lam), np.einsum("ei,iq->eq", v[..., 1], lam))

    def _edge_xy(self, e, k):
        v = self.G["verts"]
        lam = self.T.lam_e[k]                                          # (n, ng, 3)
        return np.einsum("ngi,nid->ngd", lam, v[e])

    # --------------------------------------------------------------- post
    def _flags_only(self, w):
        if self.p == 0:
            return w[:, 0, 0] + self.hbar <= self.H0
        Hv = np.einsum("em,im->ei", w[:, 0, :], self.T.phi_v) + self.hbv
        return np.all(Hv <= self.H_dry, axis=1)

    def post(self, w):
        """Limiter (optional) -> depth operator -> discharge operator -> flags."""
        w = np.array(w, copy=True)
        T, H0 = self.T, self.H0
        if self.p == 0:
            return w, w[:, 0, 0] + self.hbar <= H0
        if self.use_limiter:
            Hv0 = np.einsum("em,im->ei", w[:, 0, :], T.phi_v) + self.hbv
            full = np.all(Hv0 > self.H_dry, axis=1)
            if self.p >= 2:
                # p >= 2: the vertex depths do not bound the mean depth, which
                # must be wet too (then the positive-depth pass that follows
                # keeps the element's means, the limiter's neighbour data)
                full &= (w[:, 0, 0] + self.hbar) > self.H_dry
            nb = self.G["nbr"]
            stencil_wet = full & np.all(np.where(nb >= 0, full[np.maximum(nb, 0)], False), axis=1)
            w = limmod.apply(w, self.G, self.stencil, T, stencil_wet)
        if self.p >= 2:
            Hv = np.einsum("em,im->ei", w[:, 0, :], T.phi_v) + self.hbv
            Hm = np.einsum("em,im->ei", w[:, 0, :], T.phi_m) + self.hb_m
            trunc = np.any(Hv <= self.H_dry, axis=1) | np.any(Hm <= self.H_dry, axis=1)
            w[trunc, :, 3:] = 0.0
        vals = np.einsum("evm,im->evi", w, T.phi_v)                    # vertex values
        Hv = vals[:, 0] + self.hbv
        Hn, dchg = wetdry.depth_operator(Hv, H0)
        dry = Hn <= self.H_dry
        zn = Hn - self.hbv
        if np.any(dchg):
            w[dchg, 0, :3] = zn[dchg] @ T.V1inv.T
        for v in (1, 2):
            qn, qchg = wetdry.discharge_operator(vals[:, v], dry)
            if np.any(qchg):
                w[qchg, v, :3] = qn[qchg] @ T.V1inv.T
        return w, np.all(dry, axis=1)

    # ------------------------------------------------------------ dt / mass
    def compute_dt(self, w):
        if self.dt_fixed > 0.0:
            return self.dt_fixed
        vals = np.einsum("evm,im->evi", w, self.T.phi_v)
        Hv = vals[:, 0] + self.hbv
        wet = Hv > self.H_dry
        Hs = np.where(wet, Hv, 1.0)
        lam = np.sqrt(vals[:, 1] ** 2 + vals[:, 2] ** 2) / Hs + np.sqrt(self.g * Hs)
        lam = np.where(wet, lam, 0.0).max(axis=1)
        with np.errstate(divide="ignore"):
            ratio = np.where(lam > 0.0, self.G["d_in"] / np.where(lam > 0, lam, 1.0), np.inf)
        m = ratio.min() if ratio.size else np.inf
        return float(min(self.dt_max, self.cfl * m))

    def volume(self, w=None):
        w = self.w if w is None else w
        return float(np.sum(self.G["area"] * (w[:, 0, 0] + self.hbar)))

    def element_rain(self, t):
        return forcing.element_rain(forcing.rain_nodes(self.rain, self.xy, t), self.tri)

    # --------------------------------------------------------------- step
    def step(self, n=1):
        for _ in range(int(n)):
            t, dt = self.t, self.dt
            R = self.element_rain(t)
            met = None if self.met is None else metmod.met_nodes(self.met, self.xy, t, self.g)
            w0, wi, fi = self.w, self.w, self.flags
            bout = bin_ = 0.0
            for (a, b, gm, c), ew in zip(self.rk, self.rk_weights):
                Li, bi = self.rhs(wi, t + c * dt, R, fi, met)
                wi, fi = self.post(a * w0 + b * (wi + gm * dt * Li))
                bout += ew * bi[0]
                bin_ += ew * bi[1]
            self.rain_in += dt * float(np.sum(self.G["area"] * R))
            self.bnd_out += dt * bout
            self.bnd_in += dt * bin_
            self.w, self.flags = wi, fi
            self.t = t + dt
            self.steps += 1
            self.last_dt = dt
            self.dt = self.compute_dt(self.w)
        return self

    def mass_totals(self):
        return dict(t=self.t, dt_last=self.last_dt, volume=self.volume(), rain_in=self.rain_in,
                    bnd_in=self.bnd_in, bnd_out=self.bnd_out, steps=self.steps,
                    n_dry=int(self.flags.sum()))


def from_scenario(sc, **over):
    """Build an oracle solver from a :mod:`meshgen` scenario."""
    prm = dict(sc.params)
    prm.update(over)
    m = sc.mesh
    s = OracleSolver(m.xy, m.tri, m.hb, m.fric, m.bedges, m.btype, m.bslot,
                     p=prm["p"], flux=prm["flux"], friction=prm["friction"],
                     limiter=prm["limiter"], cfl=prm["cfl"], dt_fixed=prm["dt_fixed"],
                     dt_max=prm["dt_max"], H0=prm["H0"], g=prm["g"],
                     rk_stages=prm.get("rk_stages", 2), rain=sc.rain, tides=sc.tides, rivers=sc.rivers,
                     met=getattr(sc, "met", None))
    s.set_initial_nodal(sc.zeta0, sc.qx0, sc.qy0)
    return s
