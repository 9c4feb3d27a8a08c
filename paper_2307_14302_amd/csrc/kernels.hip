// HIP kernels of the rain-augmented shallow water DG solver (gfx950).
//
// One thread owns one element; a workgroup owns a tile of TILE consecutive
// (Hilbert-ordered) elements of one member.  Per Runge-Kutta stage the
// stage kernel evaluates the element's whole right-hand side (Sec. 2.2, Eq.
// elem_weak_form): boundary and interior edge integrals with the numerical
// flux (Sec. 2.3), the rain source (Eq. rain), the area integrals of flux,
// bed slope and friction, the inverse of the diagonal Dubiner mass, and the
// SSP stage combination (Eq. RKSSP); with the limiter off it then applies
// the positive-depth operator and the wet/dry flag (Sec. 2.4) in the same
// pass.  Interior edge fluxes are computed by both neighbours in one
// canonical orientation (the lower element id is the left state), so both
// sides obtain the same bits without atomics or an edge buffer.
//
// FP32 members keep the state and fluxes in float; depth tests of the
// positive-depth operator, dt and all budgets are done in FP64.
#include "device_common.h"
#include "internal.h"

namespace dg {

// ------------------------------------------------------------ reductions
DG_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
DG_DEV double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Sums a per-thread value over the workgroup in a fixed order.
template <int NV>
DG_DEV void block_sums(double (&v)[NV], double* lds) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double s = wave_sum(v[i]);
    if (lane == 0) lds[wv * NV + i] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = (lds[i] + lds[NV + i]) + (lds[2 * NV + i] + lds[3 * NV + i]);
  __syncthreads();
}

// ------------------------------------------------------- element basics
template <int P> struct B {
  static constexpr int NP = Tab<P>::NP;
  // value of mode m at vertex i / edge midpoint i / area point q / edge point (k, g)
  DG_HD static double V(int i, int m) { return phi_(m, vr_(i), vs_(i)); }
  DG_HD static double M(int i, int m) { return phi_(m, mr_(i), ms_(i)); }
  DG_HD static double Q(int q, int m) { return phi_(m, Tab<P>::qr(q), Tab<P>::qs(q)); }
  DG_HD static double QR(int q, int m) { return dphi_dr_(m, Tab<P>::qr(q), Tab<P>::qs(q)); }
  DG_HD static double QS(int q, int m) { return dphi_ds_(m, Tab<P>::qr(q), Tab<P>::qs(q)); }
  DG_HD static double EG(int k, int g, int m) { return phi_(m, er_(k, gl_t(P, g)), es_(k, gl_t(P, g))); }
};

// point values at the three vertices and (p = 2) the three edge midpoints
template <typename Real, int P>
DG_DEV void edge_nodes(const Real (&w)[3][Tab<P>::NP], Real (&vv)[3][3], Real (&mv)[3][3]) {
  constexpr int NP = Tab<P>::NP;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real s = Real(0), t = Real(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        s += Real(B<P>::V(i, m)) * w[v][m];
        if (P == 2) t += Real(B<P>::M(i, m)) * w[v][m];
      }
      vv[v][i] = s;
      mv[v][i] = t;
    }
}

// trace along an edge from its start-vertex value a, midpoint value c
// (p = 2) and end-vertex value b, at the edge's Gauss point g
template <typename Real, int P>
DG_DEV Real trace(Real a, Real c, Real b, int g) {
  const double t = gl_t(P, g);
  if (P == 1) return Real(lag_(1, 0, t)) * a + Real(lag_(1, 1, t)) * b;
  return Real(lag_(2, 0, t)) * a + Real(lag_(2, 1, t)) * c + Real(lag_(2, 2, t)) * b;
}

// Positive-depth operator (Sec. 2.4) on one element, FP64 decisions.
// Returns the dry flag; hv/qxv/qyv receive the final vertex depths and
// discharges (for the CFL speed).
template <typename Real, int P>
DG_DEV bool positive_depth(Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], double H0, double (&hv)[3],
                           double (&qxv)[3], double (&qyv)[3]) {
  constexpr int NP = Tab<P>::NP;
  double z[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0, a = 0.0, c = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      s += B<P>::V(i, m) * double(w[0][m]);
      a += B<P>::V(i, m) * double(w[1][m]);
      c += B<P>::V(i, m) * double(w[2][m]);
    }
    z[i] = s;
    qxv[i] = a;
    qyv[i] = c;
    hv[i] = s + double(hb[i]);
  }
  if (P == 2) {
    // any vertex or edge-midpoint depth <= H0: keep only the linear part
    bool low = (hv[0] <= H0) | (hv[1] <= H0) | (hv[2] <= H0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += B<P>::M(i, m) * double(w[0][m]);
      low |= (s + 0.5 * (double(hb[i]) + double(hb[(i + 1) % 3]))) <= H0;
    }
    if (!low) return false;   // every vertex depth > H0: nothing to do
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int m = 3; m < NP; ++m) w[v][m] = Real(0);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0, a = 0.0, c = 0.0;
#pragma unroll
      for (int m = 0; m < 3; ++m) {
        s += B<P>::V(i, m) * double(w[0][m]);
        a += B<P>::V(i, m) * double(w[1][m]);
        c += B<P>::V(i, m) * double(w[2][m]);
      }
      z[i] = s;
      qxv[i] = a;
      qyv[i] = c;
      hv[i] = s + double(hb[i]);
    }
  }
  const double S = hv[0] + hv[1] + hv[2];
  const bool case1 = (hv[0] >= H0) & (hv[1] >= H0) & (hv[2] >= H0);
  if (!case1) {
    double hn[3];
    if (S / 3.0 <= H0) {
      hn[0] = hn[1] = hn[2] = S / 3.0;
    } else {
      // ascending order with ties by local index
      int i0 = 0, i1 = 1, i2 = 2, tmp;
      if (hv[i1] < hv[i0]) { tmp = i0; i0 = i1; i1 = tmp; }
      if (hv[i2] < hv[i1]) { tmp = i1; i1 = i2; i2 = tmp; }
      if (hv[i1] < hv[i0]) { tmp = i0; i0 = i1; i1 = tmp; }
      const double n0 = H0;
      const double n1 = fmax(H0, hv[i1] - (H0 - hv[i0]) / 2.0);
      const double n2 = S - n0 - n1;
      hn[0] = (i0 == 0) ? n0 : (i1 == 0) ? n1 : n2;
      hn[1] = (i0 == 1) ? n0 : (i1 == 1) ? n1 : n2;
      hn[2] = (i0 == 2) ? n0 : (i1 == 2) ? n1 : n2;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      hv[i] = hn[i];
      z[i] = hn[i] - double(hb[i]);
    }
    // linear modes from vertex values
    w[0][0] = Real((z[0] + z[1] + z[2]) / 3.0);
    w[0][1] = Real((z[1] - z[0]) / 2.0);
    w[0][2] = Real((2.0 * z[2] - z[0] - z[1]) / 6.0);
  }
  const bool d0 = hv[0] <= H0, d1 = hv[1] <= H0, d2 = hv[2] <= H0;
  const int nd = int(d0) + int(d1) + int(d2);
  if (nd > 0) {
    double* qs[2] = {qxv, qyv};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      double* q = qs[c];
      double r0, r1, r2;
      if (nd == 3) {
        r0 = r1 = r2 = 0.0;
      } else {
        const double delta = (d0 ? q[0] : 0.0) + (d1 ? q[1] : 0.0) + (d2 ? q[2] : 0.0);
        const double add = delta / double(3 - nd);
        r0 = d0 ? 0.0 : q[0] + add;
        r1 = d1 ? 0.0 : q[1] + add;
        r2 = d2 ? 0.0 : q[2] + add;
      }
      q[0] = r0; q[1] = r1; q[2] = r2;
      w[1 + c][0] = Real((r0 + r1 + r2) / 3.0);
      w[1 + c][1] = Real((r1 - r0) / 2.0);
      w[1 + c][2] = Real((2.0 * r2 - r0 - r1) / 6.0);
    }
  }
  return nd == 3;
}

// largest |u| + sqrt(g H) over wet vertices (0 if none)
DG_DEV double cfl_speed(const double (&hv)[3], const double (&qx)[3], const double (&qy)[3], double H0, double g) {
  double lam = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (hv[i] > H0) {
      const double s = sqrt(qx[i] * qx[i] + qy[i] * qy[i]) / hv[i] + sqrt(g * hv[i]);
      lam = fmax(lam, s);
    }
  }
  return lam;
}

// ----------------------------------------------------------- stage kernel
// LIM = 0: full stage + positive-depth operator; LIM = 1: unlimited stage
// output to Wt and the fully-wet byte (the post kernel limits afterwards).
template <typename Real, int P, int FLUX, int LIM>
__global__ __launch_bounds__(TILE) void stage_kernel(const Member<Real>* __restrict__ mem,
                                                     const Tile* __restrict__ tiles, StageArgs A) {
  constexpr int NP = Tab<P>::NP, NG = Tab<P>::NG, NQ = Tab<P>::NQ;
  __shared__ double lds[4 * 6];
  const Tile tl = tiles[blockIdx.x];
  const Member<Real>& M = mem[tl.member];
  Scalars* __restrict__ sc = M.sc;
  if (!sc->active) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const Real g = Real(M.g), H0 = Real(M.H0);
  const double dt = sc->dt;
  const Real* __restrict__ Win = M.W[A.in_buf];
  const uint8_t* __restrict__ Fin = M.F[A.fin];

  Real w[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) w[v][m] = Win[(v * NP + m) * E + ec];
  Real ex[3], ey[3], hb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ex[k] = M.ev[(2 * k) * E + ec];
    ey[k] = M.ev[(2 * k + 1) * E + ec];
    hb[k] = M.hbv[k * E + ec];
  }
  const Real detJ = Real(0.25) * (ex[2] * ey[0] - ex[0] * ey[2]);
  const Real idet = rcp(detJ);
  // det J * J^{-T} = [[-e2y, -e0y], [e2x, e0x]] / 2
  const Real cx0 = Real(-0.5) * ey[2], cx1 = Real(-0.5) * ey[0];
  const Real cy0 = Real(0.5) * ex[2], cy1 = Real(0.5) * ex[0];
  const uint8_t myflag = Fin[ec] & 1;
  const uint8_t nkp = M.nk[ec];

  Real acc[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) acc[v][m] = Real(0);

  Real vv[3][3], mv[3][3];
  edge_nodes<Real, P>(w, vv, mv);
  double bout = 0.0, bin = 0.0;

  // ---- edge integrals: sum_g (l/2) w_g Fhat_g phi_m(g)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int k1 = (k + 1) % 3;
    const Real ell = dsqrt(ex[k] * ex[k] + ey[k] * ey[k]);
    const Real il = rcp(ell);
    const Real nx = ey[k] * il, ny = -ex[k] * il;
    const Real half = Real(0.5) * ell;
    const int nb = M.nbr[k * E + ec];
    if (nb >= 0) {
      const int kn = (nkp >> (2 * k)) & 3;
      Real wn[3][NP];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) wn[v][m] = Win[(v * NP + m) * E + nb];
      const uint8_t nflag = Fin[nb] & 1;
      Real nvv[3][3], nmv[3][3];
      edge_nodes<Real, P>(wn, nvv, nmv);
      const int kn1 = kn == 2 ? 0 : kn + 1;
      const bool meL = e < nb;
      // edge node values of the left (L) and right (R) sides along their own edges
      Real La[3], Lc[3], Lb[3], Ra[3], Rc[3], Rb[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const Real oa = vv[v][k], oc = mv[v][k], ob = vv[v][k1];
        const Real na = kn == 0 ? nvv[v][0] : kn == 1 ? nvv[v][1] : nvv[v][2];
        const Real nc = kn == 0 ? nmv[v][0] : kn == 1 ? nmv[v][1] : nmv[v][2];
        const Real nbv = kn1 == 0 ? nvv[v][0] : kn1 == 1 ? nvv[v][1] : nvv[v][2];
        La[v] = meL ? oa : na; Lc[v] = meL ? oc : nc; Lb[v] = meL ? ob : nbv;
        Ra[v] = meL ? na : oa; Rc[v] = meL ? nc : oc; Rb[v] = meL ? nbv : ob;
      }
      const Real hLa = meL ? hb[k] : hb[k1], hLb = meL ? hb[k1] : hb[k];
      const Real lnx = meL ? nx : -nx, lny = meL ? ny : -ny;
      const bool dryL = meL ? myflag : nflag, dryR = meL ? nflag : myflag;
#pragma unroll
      for (int gL = 0; gL < NG; ++gL) {
        const int gR = NG - 1 - gL;
        W3<Real> a{trace<Real, P>(La[0], Lc[0], Lb[0], gL), trace<Real, P>(La[1], Lc[1], Lb[1], gL),
                   trace<Real, P>(La[2], Lc[2], Lb[2], gL)};
        W3<Real> b{trace<Real, P>(Ra[0], Rc[0], Rb[0], gR), trace<Real, P>(Ra[1], Rc[1], Rb[1], gR),
                   trace<Real, P>(Ra[2], Rc[2], Rb[2], gR)};
        const Real hg = Real(lag_(1, 0, gl_t(P, gL))) * hLa + Real(lag_(1, 1, gl_t(P, gL))) * hLb;
        Real Fc[3] = {Real(0), Real(0), Real(0)};
        bool exch;
        if (!dryL && !dryR) {
          num_flux<FLUX>(a, b, hg, lnx, lny, g, H0, Fc);
          exch = true;
        } else if (dryL && dryR) {
          exch = false;
        } else {
          if (dryR) { b.x = Real(0); b.y = Real(0); } else { a.x = Real(0); a.y = Real(0); }
          num_flux<FLUX>(a, b, hg, lnx, lny, g, H0, Fc);
          exch = dryR ? (Fc[0] > Real(0)) : (Fc[0] < Real(0));
        }
        Real F[3];
        if (exch) {
          const Real sgn = meL ? Real(1) : Real(-1);
          F[0] = sgn * Fc[0]; F[1] = sgn * Fc[1]; F[2] = sgn * Fc[2];
        } else {
          const int gm = meL ? gL : gR;
          W3<Real> own{trace<Real, P>(vv[0][k], mv[0][k], vv[0][k1], gm),
                       trace<Real, P>(vv[1][k], mv[1][k], vv[1][k1], gm),
                       trace<Real, P>(vv[2][k], mv[2][k], vv[2][k1], gm)};
          wall_flux<FLUX>(own, hg, nx, ny, g, H0, F);
        }
        const Real wg = half * Real(gl_w(P, gL));
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const Real ph = meL ? Real(B<P>::EG(k, gL, m)) : Real(B<P>::EG(k, gR, m));
          const Real c = wg * ph;
          acc[0][m] -= c * F[0];
          acc[1][m] -= c * F[1];
          acc[2][m] -= c * F[2];
        }
      }
    } else {
      const int code = -1 - nb;
      const int type = code & 3, slot = code >> 2;
      double fm = 0.0;
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        W3<Real> a{trace<Real, P>(vv[0][k], mv[0][k], vv[0][k1], gi),
                   trace<Real, P>(vv[1][k], mv[1][k], vv[1][k1], gi),
                   trace<Real, P>(vv[2][k], mv[2][k], vv[2][k1], gi)};
        const Real hg = Real(lag_(1, 0, gl_t(P, gi))) * hb[k] + Real(lag_(1, 1, gl_t(P, gi))) * hb[k1];
        Real F[3];
        if (type == 0) {
          wall_flux<FLUX>(a, hg, nx, ny, g, H0, F);
        } else if (type == 3) {
          flux_normal(a, hg, nx, ny, g, H0, F[0], F[1], F[2]);
        } else if (type == 1) {
          W3<Real> gh{Real(sc->tide[A.stage][slot]), a.x, a.y};
          num_flux<FLUX>(a, gh, hg, nx, ny, g, H0, F);
        } else {
          const Real qr = Real(sc->river[A.stage][slot]);
          const Real qn = a.x * nx + a.y * ny;
          const Real dq = (Real(2) * qr - qn) - qn;
          W3<Real> gh{a.z, a.x + dq * nx, a.y + dq * ny};
          num_flux<FLUX>(a, gh, hg, nx, ny, g, H0, F);
          F[0] = qr;
        }
        const Real wg = half * Real(gl_w(P, gi));
        fm += double(wg * F[0]);
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const Real c = wg * Real(B<P>::EG(k, gi, m));
          acc[0][m] -= c * F[0];
          acc[1][m] -= c * F[1];
          acc[2][m] -= c * F[2];
        }
      }
      if (fm > 0.0) bout += fm; else bin -= fm;
    }
  }

  // ---- rain (Eq. rain): only the mean mode sees a constant source
  acc[0][0] += Real(2) * detJ * M.R[ec];

  // ---- area integrals: volume flux, bed slope, friction
  const Real dhr = Real(0.5) * (hb[1] - hb[0]), dhs = Real(0.5) * (hb[2] - hb[0]);
  const Real dhx = (cx0 * dhr + cx1 * dhs) * idet, dhy = (cy0 * dhr + cy1 * dhs) * idet;
  const Real fc = M.fric[ec];
  const Real gn2 = g * fc * fc;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    Real wq[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Real s = Real(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) s += Real(B<P>::Q(q, m)) * w[v][m];
      wq[v] = s;
    }
    const double qr = Tab<P>::qr(q), qs = Tab<P>::qs(q);
    const Real hq = Real(lam_(0, qr, qs)) * hb[0] + Real(lam_(1, qr, qs)) * hb[1] + Real(lam_(2, qr, qs)) * hb[2];
    const Real Hs = dmax(wq[0] + hq, H0);
    const Real iH = rcp(Hs);
    const Real u = wq[1] * iH, vv_ = wq[2] * iH;
    const Real Pq = Real(0.5) * g * wq[0] * (wq[0] + Real(2) * hq);
    const Real spd = dsqrt(wq[1] * wq[1] + wq[2] * wq[2]) * iH;
    const Real tau = (M.friction == 0) ? gn2 * spd * rcp(pow43(Hs)) : fc * spd * iH;
    const Real Fx[3] = {wq[1], wq[1] * u + Pq, wq[2] * u};
    const Real Fy[3] = {wq[2], wq[1] * vv_, wq[2] * vv_ + Pq};
    const Real s1 = g * wq[0] * dhx - tau * wq[1];
    const Real s2 = g * wq[0] * dhy - tau * wq[2];
    const Real Wq = Real(Tab<P>::qw(q));
    const Real wdet = Wq * detJ;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      if (m > 0) {
        const Real dr = Real(B<P>::QR(q, m)), ds = Real(B<P>::QS(q, m));
        const Real gx = Wq * (cx0 * dr + cx1 * ds), gy = Wq * (cy0 * dr + cy1 * ds);
        acc[0][m] += gx * Fx[0] + gy * Fy[0];
        acc[1][m] += gx * Fx[1] + gy * Fy[1];
        acc[2][m] += gx * Fx[2] + gy * Fy[2];
      }
      const Real ps = wdet * Real(B<P>::Q(q, m));
      acc[1][m] += ps * s1;
      acc[2][m] += ps * s2;
    }
  }

  // ---- inverse mass and SSP combination
  const Real cdt = Real(A.gam * dt);
  const Real ca = Real(A.a), cb = Real(A.b);
  const Real* __restrict__ W0 = M.W[0];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const Real L = acc[v][m] * idet * Real(1.0 / mass_(m));
      Real nw = cb * (w[v][m] + cdt * L);
      if (A.a != 0.0) nw += ca * W0[(v * NP + m) * E + ec];
      w[v][m] = nw;
    }

  double part[6] = {bout, bin, 0.0, 0.0, 0.0, 0.0};
  if (LIM == 0) {
    double hv[3], qxv[3], qyv[3];
    const bool dry = positive_depth<Real, P>(w, hb, M.H0, hv, qxv, qyv);
    if (valid) {
      Real* __restrict__ Wout = M.W[A.out_buf];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) Wout[(v * NP + m) * E + e] = w[v][m];
      M.F[A.fout][e] = dry ? 1 : 0;
    }
    if (A.last) {
      const double lam = cfl_speed(hv, qxv, qyv, M.H0, M.g);
      const double area = 0.5 * (double(ex[2]) * double(ey[0]) - double(ex[0]) * double(ey[2]));
      part[2] = valid ? area * (double(w[0][0]) + (double(hb[0]) + double(hb[1]) + double(hb[2])) / 3.0) : 0.0;
      part[3] = (valid && lam > 0.0) ? double(M.din[ec]) / lam : __builtin_inf();
      part[4] = (valid && dry) ? 1.0 : 0.0;
    }
  } else {
    if (valid) {
      Real* __restrict__ Wt = M.Wt;
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) Wt[(v * NP + m) * E + e] = w[v][m];
      bool full = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) s += B<P>::V(i, m) * double(w[0][m]);
        full &= (s + double(hb[i])) > M.H0;
      }
      M.fullwet[e] = full ? 1 : 0;
    }
  }
  // ---- tile partials (fixed-order reductions)
  {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double s0 = wave_sum(valid ? part[0] : 0.0), s1 = wave_sum(valid ? part[1] : 0.0);
    double s2 = 0.0, s4 = 0.0, mn = __builtin_inf();
    if (LIM == 0 && A.last) {
      s2 = wave_sum(part[2]);
      s4 = wave_sum(part[4]);
      mn = wave_min(part[3]);
    }
    if (lane == 0) {
      lds[wv * 5 + 0] = s0; lds[wv * 5 + 1] = s1; lds[wv * 5 + 2] = s2; lds[wv * 5 + 3] = mn; lds[wv * 5 + 4] = s4;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double* __restrict__ pt = M.part;
      const int nt = M.n_tiles, t = tl.tile;
      pt[(P_OUT0 + A.stage) * nt + t] = (lds[0] + lds[5]) + (lds[10] + lds[15]);
      pt[(P_IN0 + A.stage) * nt + t] = (lds[1] + lds[6]) + (lds[11] + lds[16]);
      if (LIM == 0 && A.last) {
        pt[P_VOL * nt + t] = (lds[2] + lds[7]) + (lds[12] + lds[17]);
        pt[P_MINR * nt + t] = fmin(fmin(lds[3], lds[8]), fmin(lds[13], lds[18]));
        pt[P_NDRY * nt + t] = (lds[4] + lds[9]) + (lds[14] + lds[19]);
      }
    }
  }
}

// ------------------------------------------------------------ post kernel
// Slope limiter (Cockburn-Shu, componentwise on zeta, qx, qy; nu = 1.5; only
// where the element and its three neighbours are fully wet), then the
// positive-depth operator, flags, CFL speed and tile partials.
// init: 0 = after a stage (reads Wt); 1 = initial state in Wt (limiter if
// the member has it, positive depth); 2 = flags and partials of W[0] only.
template <typename Real, int P>
__global__ __launch_bounds__(TILE) void post_kernel(const Member<Real>* __restrict__ mem,
                                                    const Tile* __restrict__ tiles, StageArgs A, int init,
                                                    int use_lim) {
  constexpr int NP = Tab<P>::NP;
  __shared__ double lds[4 * 5];
  const Tile tl = tiles[blockIdx.x];
  const Member<Real>& M = mem[tl.member];
  Scalars* __restrict__ sc = M.sc;
  if (!sc->active && init == 0) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const Real* __restrict__ Wsrc = (init == 2) ? M.W[0] : M.Wt;
  Real w[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) w[v][m] = Wsrc[(v * NP + m) * E + ec];
  Real hb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) hb[k] = M.hbv[k * E + ec];

  if (init != 2 && use_lim) {
    const uint8_t lc = M.limc[ec];
    int nb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) nb[k] = M.nbr[k * E + ec];
    bool ok = (lc & 1) && M.fullwet[ec];
    if (ok) {
#pragma unroll
      for (int k = 0; k < 3; ++k) ok = ok && M.fullwet[nb[k]];
    }
    if (ok) {
      Real al[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) al[j] = M.lima[j * E + ec];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const Real wb = w[v][0];
        Real nbm[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) nbm[k] = Wsrc[(v * NP) * E + nb[k]] - wb;
        Real d[3], D[3];
        bool same = true;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          d[i] = Real(B<1>::M(i, 1)) * w[v][1] + Real(B<1>::M(i, 2)) * w[v][2];
          const int kk = ((lc >> (1 + i)) & 1) ? (i + 2) % 3 : (i + 1) % 3;
          const Real nbk = kk == 0 ? nbm[0] : kk == 1 ? nbm[1] : nbm[2];
          const Real nbj = i == 0 ? nbm[0] : i == 1 ? nbm[1] : nbm[2];
          const Real db = Real(1.5) * (al[2 * i] * nbj + al[2 * i + 1] * nbk);
          const bool sgn = (d[i] > Real(0) && db > Real(0)) || (d[i] < Real(0) && db < Real(0));
          D[i] = sgn ? (d[i] > Real(0) ? dmin(d[i], db) : dmax(d[i], db)) : Real(0);
          same = same && (D[i] == d[i]);
        }
        if (!same) {
          const Real s = D[0] + D[1] + D[2];
          if (s != Real(0)) {
            const Real Pp = dmax(D[0], Real(0)) + dmax(D[1], Real(0)) + dmax(D[2], Real(0));
            const Real Nn = dmax(-D[0], Real(0)) + dmax(-D[1], Real(0)) + dmax(-D[2], Real(0));
            const Real tp = Pp == Real(0) ? Real(1) : dmin(Real(1), Nn / Pp);
            const Real tn = Nn == Real(0) ? Real(1) : dmin(Real(1), Pp / Nn);
#pragma unroll
            for (int i = 0; i < 3; ++i) D[i] = tp * dmax(D[i], Real(0)) - tn * dmax(-D[i], Real(0));
          }
          // least-squares linear part from the three midpoint deviations
          w[v][1] = D[1] - D[2];
          w[v][2] = (D[1] + D[2] - Real(2) * D[0]) / Real(3);
#pragma unroll
          for (int m = 3; m < NP; ++m) w[v][m] = Real(0);
        }
      }
    }
  }
  bool dry;
  double hv[3], qxv[3], qyv[3];
  if (init == 2) {
    // flags of the state as given
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0, a = 0.0, c = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        s += B<P>::V(i, m) * double(w[0][m]);
        a += B<P>::V(i, m) * double(w[1][m]);
        c += B<P>::V(i, m) * double(w[2][m]);
      }
      hv[i] = s + double(hb[i]);
      qxv[i] = a;
      qyv[i] = c;
    }
    dry = (hv[0] <= M.H0) & (hv[1] <= M.H0) & (hv[2] <= M.H0);
  } else {
    dry = positive_depth<Real, P>(w, hb, M.H0, hv, qxv, qyv);
  }
  const int ob = init ? 0 : A.out_buf;
  const int fo = init ? 0 : A.fout;
  if (valid) {
    if (init != 2) {
      Real* __restrict__ Wout = M.W[ob];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) Wout[(v * NP + m) * E + e] = w[v][m];
    }
    M.F[fo][e] = dry ? 1 : 0;
  }
  if (init || A.last) {
    Real ex[3], ey[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ex[k] = M.ev[(2 * k) * E + ec];
      ey[k] = M.ev[(2 * k + 1) * E + ec];
    }
    const double area = 0.5 * (double(ex[2]) * double(ey[0]) - double(ex[0]) * double(ey[2]));
    const double lam = cfl_speed(hv, qxv, qyv, M.H0, M.g);
    double vals[2] = {valid ? area * (double(w[0][0]) + (double(hb[0]) + double(hb[1]) + double(hb[2])) / 3.0) : 0.0,
                      (valid && dry) ? 1.0 : 0.0};
    const double mr = (valid && lam > 0.0) ? double(M.din[ec]) / lam : __builtin_inf();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double s0 = wave_sum(vals[0]), s1 = wave_sum(vals[1]), mn = wave_min(mr);
    if (lane == 0) { lds[wv * 3 + 0] = s0; lds[wv * 3 + 1] = s1; lds[wv * 3 + 2] = mn; }
    __syncthreads();
    if (threadIdx.x == 0) {
      double* __restrict__ pt = M.part;
      const int nt = M.n_tiles, t = tl.tile;
      pt[P_VOL * nt + t] = (lds[0] + lds[3]) + (lds[6] + lds[9]);
      pt[P_NDRY * nt + t] = (lds[1] + lds[4]) + (lds[7] + lds[10]);
      pt[P_MINR * nt + t] = fmin(fmin(lds[2], lds[5]), fmin(lds[8], lds[11]));
    }
  }
}

// fully-wet bytes of the state in Wt (initial limiting)
template <typename Real, int P>
__global__ __launch_bounds__(TILE) void classify_kernel(const Member<Real>* __restrict__ mem,
                                                        const Tile* __restrict__ tiles) {
  constexpr int NP = Tab<P>::NP;
  const Tile tl = tiles[blockIdx.x];
  const Member<Real>& M = mem[tl.member];
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  if (e >= E) return;
  bool full = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < NP; ++m) s += B<P>::V(i, m) * double(M.Wt[(0 * NP + m) * E + e]);
    full &= (s + double(M.hbv[i * E + e])) > M.H0;
  }
  M.fullwet[e] = full ? 1 : 0;
}

// -------------------------------------------------------------- rain
DG_DEV double lattice(const float* __restrict__ v, int nx, int ny, double x0, double y0, double dx, double dy,
                      double x, double y) {
  const double fx = (x - x0) / dx, fy = (y - y0) / dy;
  if (!(fx >= 0.0 && fx <= double(nx - 1) && fy >= 0.0 && fy <= double(ny - 1))) return 0.0;
  int i = int(floor(fx)), j = int(floor(fy));
  i = i > nx - 2 ? nx - 2 : i;
  j = j > ny - 2 ? ny - 2 : j;
  i = i < 0 ? 0 : i;
  j = j < 0 ? 0 : j;
  const double ax = fx - i, ay = fy - j;
  const int i1 = i + 1 < nx ? i + 1 : nx - 1, j1 = j + 1 < ny ? j + 1 : ny - 1;
  const double v00 = v[j * nx + i], v01 = v[j * nx + i1], v10 = v[j1 * nx + i], v11 = v[j1 * nx + i1];
  return (1.0 - ay) * ((1.0 - ax) * v00 + ax * v01) + ay * ((1.0 - ax) * v10 + ax * v11);
}

template <typename Real>
__global__ __launch_bounds__(TILE) void rain_kernel(const Member<Real>* __restrict__ mem,
                                                    const Tile* __restrict__ tiles, int nodal,
                                                    const double* __restrict__ rnode) {
  __shared__ double lds[4];
  const Tile tl = tiles[blockIdx.x];
  const Member<Real>& M = mem[tl.member];
  const Scalars* __restrict__ sc = M.sc;
  if (!nodal && (!sc->active || M.fo.rain_kind == RAIN_CONST)) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  double r[3];
  const int kind = M.fo.rain_kind;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int n = M.tri[i * E + ec];
    if (nodal) {
      r[i] = rnode[n];
    } else {
      const double x = M.nxy[n], y = M.nxy[M.n_nodes + n];
      if (kind == RAIN_PARAM) {
        const double xc = sc->storm[0], yc = sc->storm[1], pk = sc->storm[2], T0 = sc->storm[3];
        const double rm = sc->storm[4], re = sc->storm[5];
        const double d = hypot(x - xc, y - yc);
        r[i] = d < rm ? T0 + (pk - T0) * d / rm : pk * exp(-(d - rm) / re);
      } else {
        const Forcing& f = M.fo;
        const size_t rs = size_t(f.gnx) * f.gny;
        const double th = sc->gth;
        const double a = lattice(f.gvals + rs * sc->gk0, f.gnx, f.gny, f.gx0, f.gy0, f.gdx, f.gdy, x, y);
        const double b = lattice(f.gvals + rs * sc->gk1, f.gnx, f.gny, f.gx0, f.gy0, f.gdx, f.gdy, x, y);
        r[i] = (1.0 - th) * a + th * b;
      }
    }
  }
  const Real Re = Real((r[0] + r[1] + r[2]) / 3.0);
  if (valid) M.R[e] = Re;
  const double area = 0.5 * (double(M.ev[4 * E + ec]) * double(M.ev[1 * E + ec]) -
                             double(M.ev[0 * E + ec]) * double(M.ev[5 * E + ec]));
  double v = valid ? area * double(Re) : 0.0;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) lds[wv] = v;
  __syncthreads();
  if (threadIdx.x == 0) M.part[P_RAIN * M.n_tiles + tl.tile] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

// ------------------------------------------------------------ reduce

DG_DEV double interp_series(const double* __restrict__ tq, int n, double t) {
  // (t, q) pairs; linear between samples, held outside
  if (n <= 0) return 0.0;
  if (n == 1 || t <= tq[0]) return tq[1];
  if (t >= tq[2 * (n - 1)]) return tq[2 * (n - 1) + 1];
  int k = 0;
  while (k + 1 < n && tq[2 * (k + 1)] <= t) ++k;
  const double th = (t - tq[2 * k]) / (tq[2 * (k + 1)] - tq[2 * k]);
  return (1.0 - th) * tq[2 * k + 1] + th * tq[2 * k + 3];
}

template <typename Real>
__global__ __launch_bounds__(256) void reduce_kernel(const Member<Real>* __restrict__ mem,
                                                     const int* __restrict__ ids, int init, RKInfo rk) {
  __shared__ double lds[4 * (3 + 2 * MAX_STAGES)];
  __shared__ double shared_t, shared_dt;
  const Member<Real>& M = mem[ids[blockIdx.x]];
  Scalars* __restrict__ sc = M.sc;
  if (!init && !sc->active) return;
  const int nt = M.n_tiles;
  const double* __restrict__ pt = M.part;
  constexpr int NV = 3 + 2 * MAX_STAGES;
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  double mn = __builtin_inf();
  for (int t = threadIdx.x; t < nt; t += 256) {
    v[0] += pt[P_VOL * nt + t];
    v[1] += pt[P_RAIN * nt + t];
    v[2] += pt[P_NDRY * nt + t];
    mn = fmin(mn, pt[P_MINR * nt + t]);
    if (!init) {
#pragma unroll
      for (int s = 0; s < MAX_STAGES; ++s) {
        if (s < rk.n) {
          v[3 + s] += pt[(P_OUT0 + s) * nt + t];
          v[3 + MAX_STAGES + s] += pt[(P_IN0 + s) * nt + t];
        }
      }
    }
  }
  block_sums<NV>(v, lds);
  mn = wave_min(mn);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) lds[wv] = mn;
  __syncthreads();
  mn = fmin(fmin(lds[0], lds[1]), fmin(lds[2], lds[3]));
  if (threadIdx.x == 0) {
    double t = sc->t;
    if (!init) {
      const double dt = sc->dt;
      double bo = 0.0, bi = 0.0;
      for (int s = 0; s < rk.n; ++s) {
        bo += rk.w[s] * v[3 + s];
        bi += rk.w[s] * v[3 + MAX_STAGES + s];
      }
      sc->rain_in += dt * v[1];
      sc->bnd_out += dt * bo;
      sc->bnd_in += dt * bi;
      t = t + dt;
      sc->t = t;
      sc->steps += 1;
      sc->dt_last = dt;
    }
    sc->volume = v[0];
    sc->n_dry = (long long)(v[2]);
    double dtn = M.dt_fixed > 0.0 ? M.dt_fixed : fmin(M.dt_max, M.cfl * mn);
    if (!(v[0] == v[0]) || v[0] == __builtin_inf() || v[0] == -__builtin_inf() || !(dtn > 0.0)) {
      sc->error = 1;
      sc->active = 0;
    }
    if (sc->steps >= sc->target) sc->active = 0;
    sc->dt = dtn;
    shared_t = t;
    shared_dt = dtn;
  }
  __syncthreads();
  // forcing for the coming step
  const double t = shared_t, dt = shared_dt;
  const Forcing& f = M.fo;
  const int tid = threadIdx.x;
  if (tid < MAX_SLOTS) {
    const int s = tid;
    for (int st = 0; st < rk.n; ++st) {
      const double ts = t + rk.c[st] * dt;
      double lev = 0.0, q = 0.0;
      if (f.ocean_mask & (1u << s)) {
        lev = f.tide_mean[s];
        const double* c = f.tide_c + 3 * f.tide_off[s];
        for (int k = 0; k < f.tide_cnt[s]; ++k)
          lev += c[3 * k] * sin(2.0 * 3.14159265358979323846 * ts / c[3 * k + 1] + c[3 * k + 2]);
      }
      if (f.river_mask & (1u << s)) q = interp_series(f.riv_tq + 2 * f.riv_off[s], f.riv_cnt[s], t + rk.c[st] * dt);
      sc->tide[st][s] = lev;
      sc->river[st][s] = q;
    }
  } else if (tid == MAX_SLOTS && f.rain_kind == RAIN_PARAM && f.n_storm > 0) {
    const double* r = f.storm;
    const int n = f.n_storm;
    if (n == 1 || t <= r[0]) {
      for (int i = 0; i < 6; ++i) sc->storm[i] = r[1 + i];
    } else if (t >= r[7 * (n - 1)]) {
      for (int i = 0; i < 6; ++i) sc->storm[i] = r[7 * (n - 1) + 1 + i];
    } else {
      int k = 0;
      while (k + 1 < n && r[7 * (k + 1)] <= t) ++k;
      const double th = (t - r[7 * k]) / (r[7 * (k + 1)] - r[7 * k]);
      for (int i = 0; i < 6; ++i) sc->storm[i] = (1.0 - th) * r[7 * k + 1 + i] + th * r[7 * (k + 1) + 1 + i];
    }
  } else if (tid == MAX_SLOTS + 1 && f.rain_kind == RAIN_GRID && f.gnrec > 0) {
    const double* tr = f.gt;
    const int n = f.gnrec;
    if (n == 1 || t <= tr[0]) {
      sc->gk0 = 0; sc->gk1 = 0; sc->gth = 0.0;
    } else if (t >= tr[n - 1]) {
      sc->gk0 = n - 1; sc->gk1 = n - 1; sc->gth = 0.0;
    } else {
      int k = 0;
      while (k + 1 < n && tr[k + 1] <= t) ++k;
      sc->gk0 = k; sc->gk1 = k + 1; sc->gth = (t - tr[k]) / (tr[k + 1] - tr[k]);
    }
  }
}

// ------------------------------------------------------------ launchers
template <typename Real>
hipError_t launch_stage(int P, int flux, int limiter, const Member<Real>* m, const Tile* t, int n, StageArgs a,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(n), block(TILE);
#define DG_STAGE(PP, FF, LL) \
  if (P == PP && flux == FF && limiter == LL) { \
    hipLaunchKernelGGL((stage_kernel<Real, PP, FF, LL>), grid, block, 0, s, m, t, a); \
    return hipGetLastError(); \
  }
  DG_STAGE(1, 0, 0) DG_STAGE(1, 1, 0) DG_STAGE(1, 0, 1) DG_STAGE(1, 1, 1)
  DG_STAGE(2, 0, 0) DG_STAGE(2, 1, 0) DG_STAGE(2, 0, 1) DG_STAGE(2, 1, 1)
#undef DG_STAGE
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t launch_post(int P, int use_lim, const Member<Real>* m, const Tile* t, int n, StageArgs a, int init,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (P == 1) hipLaunchKernelGGL((post_kernel<Real, 1>), dim3(n), dim3(TILE), 0, s, m, t, a, init, use_lim);
  else if (P == 2) hipLaunchKernelGGL((post_kernel<Real, 2>), dim3(n), dim3(TILE), 0, s, m, t, a, init, use_lim);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_classify(int P, const Member<Real>* m, const Tile* t, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (P == 1) hipLaunchKernelGGL((classify_kernel<Real, 1>), dim3(n), dim3(TILE), 0, s, m, t);
  else hipLaunchKernelGGL((classify_kernel<Real, 2>), dim3(n), dim3(TILE), 0, s, m, t);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_rain(const Member<Real>* m, const Tile* t, int n, int nodal, const double* rnode, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((rain_kernel<Real>), dim3(n), dim3(TILE), 0, s, m, t, nodal, rnode);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_reduce(const Member<Real>* m, const int* ids, int n_members, int init, const RKInfo& rk,
                         hipStream_t s) {
  if (n_members <= 0) return hipSuccess;
  hipLaunchKernelGGL((reduce_kernel<Real>), dim3(n_members), dim3(256), 0, s, m, ids, init, rk);
  return hipGetLastError();
}

#define DG_INST(R)                                                                                              \
  template hipError_t launch_stage<R>(int, int, int, const Member<R>*, const Tile*, int, StageArgs, hipStream_t); \
  template hipError_t launch_post<R>(int, int, const Member<R>*, const Tile*, int, StageArgs, int, hipStream_t);  \
  template hipError_t launch_classify<R>(int, const Member<R>*, const Tile*, int, hipStream_t);                   \
  template hipError_t launch_rain<R>(const Member<R>*, const Tile*, int, int, const double*, hipStream_t);        \
  template hipError_t launch_reduce<R>(const Member<R>*, const int*, int, int, const RKInfo&, hipStream_t);
DG_INST(float)
DG_INST(double)

}  // namespace dg
