// Device-side building blocks shared by the HIP kernels of the DG solver:
// Dubiner basis tables, quadrature rules, numerical fluxes and friction.
//
// Reference triangle v0 = (-1,-1), v1 = (1,-1), v2 = (-1,1); local edge k
// runs v_k -> v_{k+1}.  Dubiner modes (Sec. 2.2, Eq. dubiner) in the order
// (0,0),(1,0),(0,1),(2,0),(1,1),(0,2),(3,0),(2,1),(1,2),(0,3), written as
// explicit polynomials with x = r + (1+s)/2 and b = (1-s)/2 (the collapsed
// Legendre factor P_i(a) b^i is a polynomial in x and b; the second factor
// is the Jacobi polynomial P_j^(2i+1,0)(s)):
//   phi00 = 1                  phi10 = x              phi01 = (1 + 3s)/2
//   phi20 = (3x^2 - b^2)/2     phi11 = x (5s + 3)/2   phi02 = (5s^2 + 2s - 1)/2
//   phi30 = (5x^3 - 3x b^2)/2  phi21 = phi20 (7s + 5)/2
//   phi12 = x (21s^2 + 18s + 1)/4                     phi03 = (35s^3 + 15s^2 - 15s - 3)/8
// Diagonal mass int phi^2 = 2/((2i+1)(i+j+1)) = 2, 1/3, 1, 2/15, 2/9, 2/3,
// 1/14, 1/10, 1/6, 1/2.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define DG_DEV __device__ __forceinline__
#define DG_HD __host__ __device__ constexpr

namespace dg {

// ------------------------------------------------------------------ basis
DG_HD double phi_(int m, double r, double s) {
  const double x = r + 0.5 * (1.0 + s), b = 0.5 * (1.0 - s);
  switch (m) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return 0.5 * (1.0 + 3.0 * s);
    case 3: return 0.5 * (3.0 * x * x - b * b);
    case 4: return 0.5 * x * (5.0 * s + 3.0);
    case 5: return 0.5 * (5.0 * s * s + 2.0 * s - 1.0);
    case 6: return 0.5 * x * (5.0 * x * x - 3.0 * b * b);
    case 7: return 0.25 * (3.0 * x * x - b * b) * (7.0 * s + 5.0);
    case 8: return 0.25 * x * (21.0 * s * s + 18.0 * s + 1.0);
    default: return 0.125 * (((35.0 * s + 15.0) * s - 15.0) * s - 3.0);
  }
}
// d/dr acts on x only (dx/dr = 1); d/ds on x (dx/ds = 1/2), b (db/ds = -1/2)
// and s itself
DG_HD double dphi_dr_(int m, double r, double s) {
  const double x = r + 0.5 * (1.0 + s), b = 0.5 * (1.0 - s);
  switch (m) {
    case 0: return 0.0;
    case 1: return 1.0;
    case 2: return 0.0;
    case 3: return 3.0 * x;
    case 4: return 0.5 * (5.0 * s + 3.0);
    case 5: return 0.0;
    case 6: return 0.5 * (15.0 * x * x - 3.0 * b * b);
    case 7: return 1.5 * x * (7.0 * s + 5.0);
    case 8: return 0.25 * (21.0 * s * s + 18.0 * s + 1.0);
    default: return 0.0;
  }
}
DG_HD double dphi_ds_(int m, double r, double s) {
  const double x = r + 0.5 * (1.0 + s), b = 0.5 * (1.0 - s);
  switch (m) {
    case 0: return 0.0;
    case 1: return 0.5;
    case 2: return 1.5;
    case 3: return 0.5 * (3.0 * x + b);
    case 4: return 0.25 * (5.0 * s + 3.0) + 2.5 * x;
    case 5: return 5.0 * s + 1.0;
    case 6: return 0.25 * (15.0 * x * x - 3.0 * b * b) + 1.5 * x * b;
    case 7: return 0.25 * (3.0 * x + b) * (7.0 * s + 5.0) + 1.75 * (3.0 * x * x - b * b);
    case 8: return 0.125 * (21.0 * s * s + 18.0 * s + 1.0) + 0.5 * x * (21.0 * s + 9.0);
    default: return 0.125 * (105.0 * s * s + 30.0 * s - 15.0);
  }
}
DG_HD double mass_(int m) {
  return m == 0 ? 2.0 : m == 1 ? 1.0 / 3.0 : m == 2 ? 1.0 : m == 3 ? 2.0 / 15.0 : m == 4 ? 2.0 / 9.0
       : m == 5 ? 2.0 / 3.0 : m == 6 ? 1.0 / 14.0 : m == 7 ? 0.1 : m == 8 ? 1.0 / 6.0 : 0.5;
}
DG_HD double vr_(int i) { return i == 1 ? 1.0 : -1.0; }
DG_HD double vs_(int i) { return i == 2 ? 1.0 : -1.0; }

// Gauss-Legendre nodes/weights on [-1,1] (p+1 points, ascending); the
// 4-point rule is sqrt(3/7 -+ (2/7) sqrt(6/5)) with weights (18 +- sqrt(30))/36.
DG_HD double gl_t(int P, int g) {
  if (P == 1) return g == 0 ? -0.57735026918962576451 : 0.57735026918962576451;
  if (P == 2) return g == 0 ? -0.77459666924148337704 : g == 1 ? 0.0 : 0.77459666924148337704;
  return g == 0 ? -0.86113631159405257522 : g == 1 ? -0.33998104358485626480
       : g == 2 ? 0.33998104358485626480 : 0.86113631159405257522;
}
DG_HD double gl_w(int P, int g) {
  if (P == 1) return 1.0;
  if (P == 2) return g == 1 ? 8.0 / 9.0 : 5.0 / 9.0;
  return (g == 1 || g == 2) ? 0.65214515486254614263 : 0.34785484513745385737;
}

template <int P> struct Tab;

// p = 1: 3-point interior area rule (barycentric 2/3, 1/6, 1/6; weight 2/3)
template <> struct Tab<1> {
  static constexpr int NP = 3, NQ = 3, NG = 2;
  DG_HD static double qr(int q) { return q == 1 ? 1.0 / 3.0 : -2.0 / 3.0; }
  DG_HD static double qs(int q) { return q == 2 ? 1.0 / 3.0 : -2.0 / 3.0; }
  DG_HD static double qw(int) { return 2.0 / 3.0; }
};
// p = 2: collapsed 3 x 3 Gauss-Legendre (b outer, a inner)
template <> struct Tab<2> {
  static constexpr int NP = 6, NQ = 9, NG = 3;
  DG_HD static double qa(int q) { return gl_t(2, q % 3); }
  DG_HD static double qb(int q) { return gl_t(2, q / 3); }
  DG_HD static double qr(int q) { return 0.5 * (1.0 + qa(q)) * (1.0 - qb(q)) - 1.0; }
  DG_HD static double qs(int q) { return qb(q); }
  DG_HD static double qw(int q) { return gl_w(2, q % 3) * gl_w(2, q / 3) * 0.5 * (1.0 - qb(q)); }
};

// p = 3: collapsed 4 x 4 Gauss-Legendre (b outer, a inner)
template <> struct Tab<3> {
  static constexpr int NP = 10, NQ = 16, NG = 4;
  DG_HD static double qa(int q) { return gl_t(3, q % 4); }
  DG_HD static double qb(int q) { return gl_t(3, q / 4); }
  DG_HD static double qr(int q) { return 0.5 * (1.0 + qa(q)) * (1.0 - qb(q)) - 1.0; }
  DG_HD static double qs(int q) { return qb(q); }
  DG_HD static double qw(int q) { return gl_w(3, q % 4) * gl_w(3, q / 4) * 0.5 * (1.0 - qb(q)); }
};

// barycentric weights of a reference point
DG_HD double lam_(int i, double r, double s) {
  return i == 0 ? -0.5 * (r + s) : i == 1 ? 0.5 * (1.0 + r) : 0.5 * (1.0 + s);
}
// reference point on local edge k at parameter t
DG_HD double er_(int k, double t) { return 0.5 * (1.0 - t) * vr_(k) + 0.5 * (1.0 + t) * vr_((k + 1) % 3); }
DG_HD double es_(int k, double t) { return 0.5 * (1.0 - t) * vs_(k) + 0.5 * (1.0 + t) * vs_((k + 1) % 3); }
// edge-midpoint reference coordinates
DG_HD double mr_(int k) { return 0.5 * (vr_(k) + vr_((k + 1) % 3)); }
DG_HD double ms_(int k) { return 0.5 * (vs_(k) + vs_((k + 1) % 3)); }

// 1D Lagrange weights at parameter t for edge nodes at t = -1, (0,) +1.
DG_HD double lag_(int P, int j, double t) {
  if (P == 1) return j == 0 ? 0.5 * (1.0 - t) : 0.5 * (1.0 + t);
  return j == 0 ? 0.5 * t * (t - 1.0) : j == 1 ? 1.0 - t * t : 0.5 * t * (t + 1.0);
}

// ------------------------------------------------------------- arithmetic
// FP32: the hardware reciprocal / square root / reciprocal square root
// (about 1 ulp).  FP64: the hardware approximation refined by two
// Newton-Raphson steps, y <- y + y (1 - x y) for 1/x and
// y <- y + y (1 - x y^2) / 2 for 1/sqrt(x); each step squares the relative
// error, so two steps reach double precision (to about 1 ulp, not
// correctly rounded).  Arguments are positive and finite except where a
// caller says otherwise.
template <typename R> DG_DEV R rcp(R x);
template <> DG_DEV double rcp<double>(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  return y;
}
template <> DG_DEV float rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename R> DG_DEV R rsq(R x);
template <> DG_DEV double rsq<double>(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  y = __builtin_fma(0.5 * y, __builtin_fma(-x * y, y, 1.0), y);
  return y;
}
template <> DG_DEV float rsq<float>(float x) { return __builtin_amdgcn_rsqf(x); }
// square root of x >= 0 (0 at 0)
template <typename R> DG_DEV R dsqrt(R x);
template <> DG_DEV double dsqrt<double>(double x) { return x > 0.0 ? x * rsq<double>(x) : 0.0; }
template <> DG_DEV float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
// x^(-4/3) for x > 0 (Manning): FP32 through exp2/log2; FP64 refines a
// single-precision guess of y = x^(-1/3) by two Newton steps of
// y^-3 = x, y <- y (4 - x y^3) / 3, then returns y^4
template <typename R> DG_DEV R rpow43(R x);
template <> DG_DEV double rpow43<double>(double x) {
  double y = double(__builtin_amdgcn_exp2f(-0.33333333333333333f * __builtin_amdgcn_logf(float(x))));
  y = y * (4.0 - x * (y * y * y)) * (1.0 / 3.0);
  y = y * (4.0 - x * (y * y * y)) * (1.0 / 3.0);
  const double y2 = y * y;
  return y2 * y2;
}
template <> DG_DEV float rpow43<float>(float x) {
  return __builtin_amdgcn_exp2f(-1.3333333333333333f * __builtin_amdgcn_logf(x));
}
template <typename R> DG_DEV R dmax(R a, R b) { return a > b ? a : b; }
template <typename R> DG_DEV R dmin(R a, R b) { return a < b ? a : b; }
template <typename R> DG_DEV R dabs(R a) { return a < R(0) ? -a : a; }

// -------------------------------------------------------------- fluxes
// State w = (zeta, qx, qy); H = zeta + hb; velocities q / max(H, H0);
// pressure g/2 (H^2 - hb^2) = g/2 zeta (zeta + 2 hb) (Eq. SWE).
template <typename R> struct W3 { R z, x, y; };

// Inverse depth and gravity-wave speed of one side: ih = 1 / max(H, H0),
// c = sqrt(g max(H, 0)).  FP32 takes both from one reciprocal square root
// (sqrt(x) = x / sqrt(x), 1/x = (1/sqrt(x))^2; below H0 the clamped inverse
// is the constant 1/H0); FP64 divides and takes the square root.
template <typename R>
DG_DEV void depth_inv_speed(R H, R g, R H0, R& ih, R& c) {
  if constexpr (sizeof(R) == 4) {
    const float r = __builtin_amdgcn_rsqf(dmax(H, 1e-30f));
    ih = H >= H0 ? r * r : __builtin_amdgcn_rcpf(H0);
    c = __builtin_amdgcn_sqrtf(g) * (dmax(H, 0.0f) * r);
  } else {
    ih = rcp(dmax(H, H0));
    c = dsqrt(g * dmax(H, R(0)));
  }
}

template <typename R>
DG_DEV void flux_normal(const W3<R>& w, R hb, R nx, R ny, R g, R H0, R& f0, R& f1, R& f2) {
  const R Hs = dmax(w.z + hb, H0);
  const R qn = w.x * nx + w.y * ny;
  const R un = qn * rcp(Hs);
  const R P = R(0.5) * g * w.z * (w.z + R(2) * hb);
  f0 = qn;
  f1 = w.x * un + P * nx;
  f2 = w.y * un + P * ny;
}

// Local Lax-Friedrichs: (F(a)+F(b))/2 - lam/2 (b - a), lam the larger of
// |u.n| + sqrt(g H) on the two sides.
template <typename R>
DG_DEV void flux_llf(const W3<R>& a, const W3<R>& b, R hb, R nx, R ny, R g, R H0, R* F) {
  R ia, ib, ca, cb;
  depth_inv_speed(a.z + hb, g, H0, ia, ca);
  depth_inv_speed(b.z + hb, g, H0, ib, cb);
  const R qna = a.x * nx + a.y * ny, qnb = b.x * nx + b.y * ny;
  const R ua = qna * ia, ub = qnb * ib;
  const R Pa = R(0.5) * g * a.z * (a.z + R(2) * hb), Pb = R(0.5) * g * b.z * (b.z + R(2) * hb);
  const R lam = dmax(dabs(ua) + ca, dabs(ub) + cb);
  F[0] = R(0.5) * (qna + qnb) - R(0.5) * lam * (b.z - a.z);
  F[1] = R(0.5) * ((a.x * ua + Pa * nx) + (b.x * ub + Pb * nx)) - R(0.5) * lam * (b.x - a.x);
  F[2] = R(0.5) * ((a.y * ua + Pa * ny) + (b.y * ub + Pb * ny)) - R(0.5) * lam * (b.y - a.y);
}

// Roe: linearisation about the Roe average in the frame (n, t):
// waves u~n - c~, u~n, u~n + c~ with c~ = sqrt(g (Ha + Hb)/2); right
// eigenvectors (1, u~n - c~, u~t), (0, 0, 1), (1, u~n + c~, u~t); with a
// continuous bed the depth jump equals the elevation jump.  No entropy fix.
// The Roe average of a velocity is (q_a/sqrt(Ha) + q_b/sqrt(Hb)) / (sqrt(Ha)
// + sqrt(Hb)).
template <typename R>
DG_DEV void flux_roe(const W3<R>& a, const W3<R>& b, R hb, R nx, R ny, R g, R H0, R* F) {
  const R Ha = dmax(a.z + hb, H0), Hb = dmax(b.z + hb, H0);
  const R qna = a.x * nx + a.y * ny, qta = -a.x * ny + a.y * nx;
  const R qnb = b.x * nx + b.y * ny, qtb = -b.x * ny + b.y * nx;
  R sa, sb, ia, ib, ra, rb, c, i2c;
  if constexpr (sizeof(R) == 4) {
    ra = __builtin_amdgcn_rsqf(Ha);
    rb = __builtin_amdgcn_rsqf(Hb);
    sa = Ha * ra; sb = Hb * rb;
    ia = ra * ra; ib = rb * rb;
    const R c2 = R(0.5) * g * (Ha + Hb);
    const R rc = __builtin_amdgcn_rsqf(c2);
    c = c2 * rc;
    i2c = R(0.5) * rc;
  } else {
    ra = rsq(Ha); rb = rsq(Hb);
    sa = Ha * ra; sb = Hb * rb;
    ia = ra * ra; ib = rb * rb;
    const R c2 = R(0.5) * g * (Ha + Hb);
    const R rc = rsq(c2);
    c = c2 * rc;
    i2c = R(0.5) * rc;
  }
  const R isum = rcp(sa + sb);
  const R un = (qna * ra + qnb * rb) * isum;
  const R ut = (qta * ra + qtb * rb) * isum;
  const R Pa = R(0.5) * g * a.z * (a.z + R(2) * hb), Pb = R(0.5) * g * b.z * (b.z + R(2) * hb);
  const R ua = qna * ia, ub = qnb * ib;
  const R dH = b.z - a.z, dqn = qnb - qna, dqt = qtb - qta;
  const R a1 = ((un + c) * dH - dqn) * i2c;
  const R a3 = (dqn - (un - c) * dH) * i2c;
  const R a2 = dqt - ut * dH;
  const R l1 = dabs(un - c) * a1, l2 = dabs(un) * a2, l3 = dabs(un + c) * a3;
  const R d0 = l1 + l3;
  const R dn = l1 * (un - c) + l3 * (un + c);
  const R dt = (l1 + l3) * ut + l2;
  F[0] = R(0.5) * (qna + qnb) - R(0.5) * d0;
  F[1] = R(0.5) * ((a.x * ua + Pa * nx) + (b.x * ub + Pb * nx)) - R(0.5) * (dn * nx - dt * ny);
  F[2] = R(0.5) * ((a.y * ua + Pa * ny) + (b.y * ub + Pb * ny)) - R(0.5) * (dn * ny + dt * nx);
}

template <int FLUX, typename R>
DG_DEV void num_flux(const W3<R>& a, const W3<R>& b, R hb, R nx, R ny, R g, R H0, R* F) {
  if (FLUX == 0) flux_roe(a, b, hb, nx, ny, g, H0, F);
  else flux_llf(a, b, hb, nx, ny, g, H0, F);
}

// Land boundary: the numerical flux between the state and its mirror image
// (normal discharge reversed).  Written out, both solvers give a zero mass
// flux and a normal momentum flux Phi n with
//   LLF: Phi = P + q_n (u_n + |u_n| + c),   c = sqrt(g max(H, 0)),
//   Roe: Phi = P + q_n (u_n + c~),          c~ = sqrt(g max(H, H0))
// (the Roe average of the pair has zero normal velocity, so the two
// acoustic waves carry the reflected discharge), u_n = q_n / max(H, H0).
template <int FLUX, typename R>
DG_DEV void wall_flux(const W3<R>& a, R hb, R nx, R ny, R g, R H0, R* F) {
  const R H = a.z + hb;
  const R qn = a.x * nx + a.y * ny;
  const R P = R(0.5) * g * a.z * (a.z + R(2) * hb);
  R Phi;
  if (FLUX == 0) {
    const R Hs = dmax(H, H0);
    R ih, c;
    if constexpr (sizeof(R) == 4) {
      const float r = __builtin_amdgcn_rsqf(Hs);
      ih = r * r;
      c = __builtin_amdgcn_sqrtf(g) * (Hs * r);
    } else {
      const R r = rsq(Hs);
      ih = r * r;
      c = dsqrt(g) * (Hs * r);
    }
    Phi = P + qn * (qn * ih + c);
  } else {
    R ih, c;
    depth_inv_speed(H, g, H0, ih, c);
    const R un = qn * ih;
    Phi = P + qn * (un + dabs(un) + c);
  }
  F[0] = R(0);
  F[1] = Phi * nx;
  F[2] = Phi * ny;
}

}  // namespace dg
