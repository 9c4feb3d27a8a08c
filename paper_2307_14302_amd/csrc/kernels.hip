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
#include <hip/hip_ext.h>

#include <type_traits>
#include <utility>

#include "device_common.h"
#include "internal.h"

namespace dg {

#ifndef DG_STAGE_WAVES
#define DG_STAGE_WAVES 1
#endif
#define DG_STAGE_ATTR __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(DG_STAGE_WAVES)))
// the FP64 p = 3 per-edge kernel on 64-element tiles is built for two
// wavefronts per SIMD (its LDS allows six workgroups per CU) and the FP32
// one with matrix-core area integrals (MF) for three, the others for one
// (their occupancy is set by LDS or by registers the compiler keeps)
#define DG_STAGE_ATTR_T(T)                                                                        \
  __launch_bounds__(T) __attribute__((amdgpu_waves_per_eu(                                        \
      MF ? 3 : (P == 3 && sizeof(Real) == 8 && T == 64) ? 2 : DG_STAGE_WAVES)))

// f(std::integral_constant<int, i>) for i = 0 .. N-1, expanded at compile time
template <typename F, int... I>
DG_DEV void static_for_(F& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
DG_DEV void static_for(F&& f) {
  static_for_(f, std::make_integer_sequence<int, N>{});
}

// Pointers read from the member descriptor are generic to the compiler; all
// device arrays live in global memory, so they are re-typed to the global
// address space (global_load/store with a scalar base instead of flat).
#define DG_G __attribute__((address_space(1)))
template <typename T> DG_DEV DG_G T* gp(T* p) { return (DG_G T*)p; }
template <typename T> DG_DEV const DG_G T* gp(const T* p) { return (const DG_G T*)p; }

// Element- and node-indexed access through buffer instructions: the array's
// base goes into a scalar resource descriptor, the column's offset into a
// scalar offset and the lane's index into a 32-bit byte offset, so an access
// costs no vector address arithmetic (global addressing forms a 64-bit
// address per access) and a kernel keeps one descriptor per array.  The
// element index must be valid (the descriptor's record count is the
// maximum, so there is no range check) and every byte offset within an
// array below 2^32; the library refuses meshes whose arrays would exceed it.
// ldc(base, col, i) reads base[col + i] with col uniform over the wavefront.
DG_DEV __amdgpu_buffer_rsrc_t rsrc(const void* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, -1, 0x00020000);
}
typedef unsigned int dg_u2 __attribute__((ext_vector_type(2)));
template <typename T> DG_DEV T ldc(const DG_G T* base, int col, int i) {
  static_assert(sizeof(T) == 1 || sizeof(T) == 4 || sizeof(T) == 8, "1, 4 or 8 byte elements");
  const uint32_t off = uint32_t(i) * uint32_t(sizeof(T)), so = uint32_t(col) * uint32_t(sizeof(T));
  const __amdgpu_buffer_rsrc_t r = rsrc((const void*)base);
  if constexpr (sizeof(T) == 1) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b8(r, off, so, 0));
  else if constexpr (sizeof(T) == 4) return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, so, 0));
  else return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, so, 0));
}
template <typename T> DG_DEV T ldx(const DG_G T* base, int i) { return ldc(base, 0, i); }
template <typename T> DG_DEV void stc(DG_G T* base, int col, int i, T v) {
  static_assert(sizeof(T) == 1 || sizeof(T) == 4 || sizeof(T) == 8, "1, 4 or 8 byte elements");
  const uint32_t off = uint32_t(i) * uint32_t(sizeof(T)), so = uint32_t(col) * uint32_t(sizeof(T));
  const __amdgpu_buffer_rsrc_t r = rsrc((const void*)base);
  if constexpr (sizeof(T) == 1) __builtin_amdgcn_raw_buffer_store_b8(__builtin_bit_cast(unsigned char, v), r, off, so, 0);
  else if constexpr (sizeof(T) == 4) __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned int, v), r, off, so, 0);
  else __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(dg_u2, v), r, off, so, 0);
}
template <typename T> DG_DEV void stx(DG_G T* base, int i, T v) { stc(base, 0, i, v); }

// ------------------------------------------------------------ reductions
// Wavefront reductions in a fixed order with DPP lane moves (VALU only; no
// LDS traffic): within each 16-lane row, swap neighbours, swap pairs, rotate
// by 4 and by 8, which leaves the row total in every lane of the row; then
// the four row totals are combined in order 0, 1, 2, 3 through readlane.
// Doubles move as two 32-bit halves.
DG_DEV double dpp_f64(double x, int ctrl_sel) {
  const long long b = __double_as_longlong(x);
  int lo = int(b & 0xffffffffll), hi = int(b >> 32);
  switch (ctrl_sel) {
    case 0: lo = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: lo = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: lo = __builtin_amdgcn_update_dpp(0, lo, 0x124, 0xF, 0xF, false);
            hi = __builtin_amdgcn_update_dpp(0, hi, 0x124, 0xF, 0xF, false); break;  // row_ror:4
    default: lo = __builtin_amdgcn_update_dpp(0, lo, 0x128, 0xF, 0xF, false);
             hi = __builtin_amdgcn_update_dpp(0, hi, 0x128, 0xF, 0xF, false); break; // row_ror:8
  }
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
DG_DEV double lane_f64(double x, int lane) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
// Inclusive prefix sum of an int over the wavefront with DPP: shifts by 1,
// 2, 4 and 8 lanes within each 16-lane row (zero fill), then the last lane
// of row 0 and 2 is added to rows 1 and 3 and the last lane of row 1 to
// rows 2 and 3.
DG_DEV int wave_incl_scan(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);   // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xA, 0xF, false);   // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xC, 0xF, false);   // row_bcast:31
  return x;
}

DG_DEV double wave_sum(double v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v += dpp_f64(v, c);
  return ((lane_f64(v, 0) + lane_f64(v, 16)) + lane_f64(v, 32)) + lane_f64(v, 48);
}
DG_DEV double wave_min(double v) {
#pragma unroll
  for (int c = 0; c < 4; ++c) v = fmin(v, dpp_f64(v, c));
  return fmin(fmin(lane_f64(v, 0), lane_f64(v, 16)), fmin(lane_f64(v, 32), lane_f64(v, 48)));
}

// Element id of the lowest set lane of a ballot (base = id of lane 0), or
// infinity when no lane is set.
DG_DEV double first_lane_id(unsigned long long mask, int base) {
  return mask ? double(base + __builtin_ctzll(mask)) : __builtin_inf();
}

// Decision margins: the positive-depth operator puts vertices at exactly H0,
// so the tests that follow use H0 (1 + 1e-3) for "dry", and a wet-dry edge
// exchanges water only above a mass flux of 1e-3 H0 sqrt(g H0) (Member::feps,
// formed on the host).
DG_DEV double dry_depth(double H0) { return H0 * (1.0 + 1e-3); }

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  The grid is padded to a multiple of 8 and block b takes tile
// (b mod 8) * chunk + b / 8, so every XCD walks one contiguous run of
// (Hilbert-ordered) tiles and the halos of neighbouring tiles share its L2.
DG_DEV int xcd_tile() {
  const int chunk = int(gridDim.x) >> 3;
  return int(blockIdx.x & 7u) * chunk + int(blockIdx.x >> 3);
}
inline int xcd_grid(int n) { return ((n + 7) / 8) * 8; }

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

// a b + c rounded once
template <typename Real>
DG_DEV Real fmac(Real a, Real b, Real c) {
  if constexpr (sizeof(Real) == 4) return __builtin_fmaf(a, b, c);
  else return __builtin_fma(a, b, c);
}

// point values at the three vertices and (p = 2) the three edge midpoints
// (fused multiply-adds written out, so that every call site rounds alike)
template <typename Real, int P>
DG_DEV void edge_nodes(const Real (&w)[3][Tab<P>::NP], Real (&vv)[3][3], Real (&mv)[3][3]) {
  constexpr int NP = Tab<P>::NP;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      Real s = Real(B<P>::V(i, 0)) * w[v][0], t = Real(B<P>::M(i, 0)) * w[v][0];
#pragma unroll
      for (int m = 1; m < NP; ++m) {
        s = fmac(Real(B<P>::V(i, m)), w[v][m], s);
        if (P >= 2) t = fmac(Real(B<P>::M(i, m)), w[v][m], t);
      }
      vv[v][i] = s;
      mv[v][i] = P >= 2 ? t : Real(0);
    }
}

// Basis values at the edge Gauss points, evaluated at compile time (a
// constexpr table: a select between entries stays a select of literals).
template <int P> struct EdgeTable {
  double v[3][Tab<P>::NG][Tab<P>::NP];
};
template <int P>
constexpr EdgeTable<P> make_edge_table() {
  EdgeTable<P> t{};
  for (int k = 0; k < 3; ++k)
    for (int g = 0; g < Tab<P>::NG; ++g)
      for (int m = 0; m < Tab<P>::NP; ++m) t.v[k][g][m] = B<P>::EG(k, g, m);
  return t;
}

// trace of the modes w at Gauss point G of local edge k.  k may be a
// runtime value: then the three edges' traces are formed with constant
// coefficients and one is selected (selecting the coefficients instead
// turns them into a table in memory read per lane).
template <typename Real, int P, int G>
DG_DEV Real trace_modal(const Real (&w)[Tab<P>::NP], int k) {
  constexpr EdgeTable<P> T = make_edge_table<P>();
  Real s0 = Real(0), s1 = Real(0), s2 = Real(0);
#pragma unroll
  for (int m = 0; m < Tab<P>::NP; ++m) {
    s0 += Real(T.v[0][G][m]) * w[m];
    s1 += Real(T.v[1][G][m]) * w[m];
    s2 += Real(T.v[2][G][m]) * w[m];
  }
  return k == 0 ? s0 : k == 1 ? s1 : s2;
}

// trace along an edge from its start-vertex value a, midpoint value c
// (p = 2) and end-vertex value b, at the edge's Gauss point g (p <= 2: the
// trace is the 1-D interpolant of those point values).  The fused
// multiply-adds are written out so that every call site rounds alike: the
// traces of an element's own edges and those of a neighbour in another
// tile are formed in different places, and must agree to the bit.
template <typename Real, int P>
DG_DEV Real trace(Real a, Real c, Real b, int g) {
  static_assert(P <= 2, "point-value traces are exact for p <= 2 only");
  const double t = gl_t(P, g);
  if (P == 1) return fmac(Real(lag_(1, 1, t)), b, Real(lag_(1, 0, t)) * a);
  return fmac(Real(lag_(2, 2, t)), b, fmac(Real(lag_(2, 1, t)), c, Real(lag_(2, 0, t)) * a));
}

// Positive-depth operator (Sec. 2.4) on one element, FP64 decisions.
// Returns the dry flag; hv/qxv/qyv receive the final vertex depths and
// discharges (for the CFL speed).
// True when every vertex (and, for p >= 2, edge-midpoint) depth is above the
// dry margin by more than the rounding error of evaluating it in Real: then
// the exact FP64 tests below would find the element fully wet and leave it
// unchanged, so they can be skipped.
template <typename Real, int P>
DG_DEV bool surely_wet(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], double Hd) {
  constexpr int NP = Tab<P>::NP;
  const Real rel = Real(sizeof(Real) == 4 ? 4e-6 : 1e-12);
  bool ok = true;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Real s = Real(0), t = Real(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      s += Real(B<P>::V(i, m)) * w[0][m];
      if (P >= 2) t += Real(B<P>::M(i, m)) * w[0][m];
    }
    ok &= (s + hb[i]) > Real(Hd) + rel * (dabs(s) + dabs(hb[i]) + Real(1));
    if (P >= 2) {
      const Real hm = Real(0.5) * (hb[i] + hb[(i + 1) % 3]);
      ok &= (t + hm) > Real(Hd) + rel * (dabs(t) + dabs(hm) + Real(1));
    }
  }
  return ok;
}

// The limiter's condition on an element (Sec. 2.3 limiter, Sec. 2.4 fronts):
// every vertex depth above the dry margin and, for p >= 2, the mean depth
// too (the vertices do not bound the mean of a curved element).  Decided in
// FP64 as the positive-depth tests are.  A fully-wet element keeps its means
// through the positive-depth pass that follows the limiter: its mean depth
// stays above the margin, so at least one vertex stays wet and the discharge
// means are not zeroed.
template <typename Real, int P>
DG_DEV bool fully_wet(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], double H0) {
  constexpr int NP = Tab<P>::NP;
  const double Hd = dry_depth(H0);
  // the exact vertex tests are skipped where the element is surely wet
  bool full = surely_wet<Real, P>(w, hb, Hd);
  if (!full) {
    full = true;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += B<P>::V(i, m) * double(w[0][m]);
      full &= (s + double(hb[i])) > Hd;
    }
  }
  if (P >= 2) full &= (double(w[0][0]) + (double(hb[0]) + double(hb[1]) + double(hb[2])) / 3.0) > Hd;
  return full;
}

// need_v: the caller needs hv/qxv/qyv (the CFL speed); otherwise a surely
// wet element returns at once.  *changed is set when w was modified.  Both
// operators keep the element means of depth and momentum (redistribution
// between vertices), so mode 0 is left as it is, except for the momentum
// of an element dry at every vertex, which is set to zero.
template <typename Real, int P>
DG_DEV bool positive_depth(Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], double H0, double (&hv)[3],
                           double (&qxv)[3], double (&qyv)[3], bool need_v, bool& filled,
                           bool* changed = nullptr) {
  constexpr int NP = Tab<P>::NP;
  const double Hd = dry_depth(H0);
  filled = false;
  if (!need_v && surely_wet<Real, P>(w, hb, Hd)) return false;
  filled = true;
  bool mod = false;
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
  if (P >= 2) {
    // any vertex or edge-midpoint depth <= H0: keep only the linear part
    bool low = (hv[0] <= Hd) | (hv[1] <= Hd) | (hv[2] <= Hd);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double s = 0.0;
#pragma unroll
      for (int m = 0; m < NP; ++m) s += B<P>::M(i, m) * double(w[0][m]);
      low |= (s + 0.5 * (double(hb[i]) + double(hb[(i + 1) % 3]))) <= Hd;
    }
    if (!low) return false;   // every vertex depth above the dry margin: nothing to do
    mod = true;
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
    // slopes from the new vertex values (their mean is the old one)
    w[0][1] = Real((z[1] - z[0]) / 2.0);
    w[0][2] = Real((2.0 * z[2] - z[0] - z[1]) / 6.0);
    mod = true;
  }
  const bool d0 = hv[0] <= Hd, d1 = hv[1] <= Hd, d2 = hv[2] <= Hd;
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
      if (nd == 3) w[1 + c][0] = Real(0);
      w[1 + c][1] = Real((r1 - r0) / 2.0);
      w[1 + c][2] = Real((2.0 * r2 - r0 - r1) / 6.0);
    }
    mod = true;
  }
  if (changed) *changed = mod;
  return nd == 3;
}

// largest |u| + sqrt(g H) over wet vertices (0 if none; NaN if a speed is
// NaN, e.g. from an overflowing discharge)
DG_DEV double cfl_speed(const double (&hv)[3], const double (&qx)[3], const double (&qy)[3], double H0, double g) {
  double lam = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    if (hv[i] > dry_depth(H0)) {
      const double s = dsqrt(qx[i] * qx[i] + qy[i] * qy[i]) * rcp(hv[i]) + dsqrt(g * hv[i]);
      lam = (s > lam || s != s) ? s : lam;      // a NaN speed is kept (flagged by the caller)
    }
  }
  return lam;
}

// The same speed for an element known to be wet at every vertex, in the
// state's precision (FP32 members; the wet test that selects vertices is not
// needed).
template <typename Real, int P>
DG_DEV double element_speed(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], Real g) {
  constexpr int NP = Tab<P>::NP;
  Real lam = Real(0);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    Real h = hb[i], a = Real(0), c = Real(0);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      h += Real(B<P>::V(i, m)) * w[0][m];
      a += Real(B<P>::V(i, m)) * w[1][m];
      c += Real(B<P>::V(i, m)) * w[2][m];
    }
    const Real s = dsqrt(a * a + c * c) * rcp(h) + dsqrt(g * h);
    lam = dmax(lam, s);
  }
  return double(lam);
}

// CFL speed after the positive-depth operator: from its FP64 vertex values
// when it computed them, else (FP32 member, surely wet element) in FP32.
template <typename Real, int P>
DG_DEV double post_speed(bool filled, const double (&hv)[3], const double (&qxv)[3], const double (&qyv)[3],
                         const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], double H0, double g) {
  if (filled) return cfl_speed(hv, qxv, qyv, H0, g);
  return element_speed<Real, P>(w, hb, Real(g));
}

// Slope limiter on one element whose stencil is fully wet (Sec. 2.3,
// Cockburn-Shu, componentwise on zeta, qx, qy, nu = 1.5): nmean[v][k] is the
// mean of variable v in the neighbour across local edge k, al and lc the
// element's decomposition weights and code.  Returns true when any
// component changed (its linear part is rebuilt from the limited midpoint
// deviations and its higher modes are dropped).
template <typename Real, int P>
DG_DEV bool limit_element(Real (&w)[3][Tab<P>::NP], uint8_t lc, const Real (&al)[6], const Real (&nmean)[3][3]) {
  constexpr int NP = Tab<P>::NP;
  bool changed = false;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    const Real wb = w[v][0];
    Real nbm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) nbm[k] = nmean[v][k] - wb;
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
      changed = true;
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
  return changed;
}

// The post-processing of one element of a raw stage output (Sec. 2.3
// limiter where its stencil is fully wet, then the positive-depth operator
// of Sec. 2.4): the post kernel's arithmetic with the neighbours' raw means
// and fully-wet bytes taken from LDS slots (s_mean[v * SM + slot],
// s_fw[slot]; ns = the element's neighbour slots, 10 bits each, self = its
// own slot; lc and al its limiter code and weights, loaded by the caller
// ahead of the barrier that publishes the slots).  Returns the dry flag.
template <typename Real, int P>
DG_DEV bool post_from_slots(const Member<Real>& M, Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], uint8_t lc,
                            const Real (&al)[6], uint32_t ns, int self, const Real* s_mean, const uint8_t* s_fw,
                            int SM) {
  bool ok = ((lc & 1) != 0) & (s_fw[self] != 0);
  Real nmean[3][3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int sl = int((ns >> (10 * k)) & HALO_SLOT_MASK);
    const bool in = sl != int(HALO_SLOT_MASK);
    const int at = in ? sl : self;
    ok = ok & in & (s_fw[at] != 0);
#pragma unroll
    for (int v = 0; v < 3; ++v) nmean[v][k] = s_mean[v * SM + at];
  }
  if (ok) (void)limit_element<Real, P>(w, lc, al, nmean);
  double hv[3], qxv[3], qyv[3];
  bool filled;
  return positive_depth<Real, P>(w, hb, M.H0, hv, qxv, qyv, false, filled);
}

// ------------------------------------------------------ stage building blocks
// Outward fluxes at one Gauss point of an interior edge, in the canonical
// orientation (L = lower element id, n = L's outward normal, a/b = traces of
// L and R at this point).  wet-wet: the numerical flux.  Otherwise the wet
// trace meets the dry one with its discharge zeroed; if that mass flux enters
// the dry element the flux is exchanged, else each side gets the flux of its
// own mirrored state (land boundary).  FL / FR are the outward fluxes of L
// and R; needL / needR say which the caller uses.
template <int FLUX, typename Real>
DG_DEV void interior_point(const W3<Real>& a, const W3<Real>& b, Real hg, Real lnx, Real lny, Real g, Real H0,
                           Real feps, bool dryL, bool dryR, bool needL, bool needR, Real* FL, Real* FR) {
  Real Fc[3] = {Real(0), Real(0), Real(0)};
  bool exch;
  if (!dryL && !dryR) {
    num_flux<FLUX>(a, b, hg, lnx, lny, g, H0, Fc);
    exch = true;
  } else if (dryL && dryR) {
    exch = false;
  } else {
    W3<Real> a2 = a, b2 = b;
    if (dryR) { b2.x = Real(0); b2.y = Real(0); } else { a2.x = Real(0); a2.y = Real(0); }
    num_flux<FLUX>(a2, b2, hg, lnx, lny, g, H0, Fc);
    exch = dryR ? (Fc[0] > feps) : (Fc[0] < -feps);
  }
  if (exch) {
    FL[0] = Fc[0]; FL[1] = Fc[1]; FL[2] = Fc[2];
    FR[0] = -Fc[0]; FR[1] = -Fc[1]; FR[2] = -Fc[2];
  } else {
    if (needL) wall_flux<FLUX>(a, hg, lnx, lny, g, H0, FL);
    if (needR) wall_flux<FLUX>(b, hg, -lnx, -lny, g, H0, FR);
  }
}

// Outward flux at a boundary Gauss point (Sec. 2.1 boundary partition):
// land = mirrored normal discharge, outflow = interior state, ocean =
// elevation of its slot with the interior discharge, river = ghost normal
// discharge 2 q_river - q_n and the mass flux set to q_river.
template <int FLUX, typename Real>
DG_DEV void boundary_point(const W3<Real>& a, Real hg, Real nx, Real ny, Real g, Real H0, int type, Real tide,
                           Real qr, Real* F) {
  if (type == 0) {
    wall_flux<FLUX>(a, hg, nx, ny, g, H0, F);
  } else if (type == 3) {
    flux_normal(a, hg, nx, ny, g, H0, F[0], F[1], F[2]);
  } else if (type == 1) {
    W3<Real> gh{tide, a.x, a.y};
    num_flux<FLUX>(a, gh, hg, nx, ny, g, H0, F);
  } else {
    const Real qn = a.x * nx + a.y * ny;
    const Real dq = (Real(2) * qr - qn) - qn;
    W3<Real> gh{a.z, a.x + dq * nx, a.y + dq * ny};
    num_flux<FLUX>(a, gh, hg, nx, ny, g, H0, F);
    F[0] = qr;
  }
}

// Length of an edge vector and its inverse (FP32: one reciprocal square
// root).  Both neighbours of an edge hold the same vector up to sign, so they
// obtain the same bits.
template <typename Real>
DG_DEV void edge_length(Real ex, Real ey, Real& ell, Real& il) {
  const Real l2 = ex * ex + ey * ey;
  if constexpr (sizeof(Real) == 4) {
    il = __builtin_amdgcn_rsqf(l2);
    ell = l2 * il;
  } else {
    il = rsq(l2);
    ell = l2 * il;
  }
}

// Area integrals: volume flux, bed slope and bottom friction (Eq. SWE).
template <typename Real, int P>
DG_DEV void area_terms_unrolled(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], Real cx0, Real cx1, Real cy0,
                                Real cy1, Real detJ, Real idet, Real fc, int friction, Real g, Real H0,
                                Real (&acc)[3][Tab<P>::NP]) {
  constexpr int NP = Tab<P>::NP, NQ = Tab<P>::NQ;
  const Real dhr = Real(0.5) * (hb[1] - hb[0]), dhs = Real(0.5) * (hb[2] - hb[0]);
  const Real dhx = (cx0 * dhr + cx1 * dhs) * idet, dhy = (cy0 * dhr + cy1 * dhs) * idet;
  const Real gn2 = g * fc * fc;
  Real Sx[3] = {Real(0), Real(0), Real(0)}, Sy[3] = {Real(0), Real(0), Real(0)};
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
    Real iH, Hm43;   // 1/H and (Manning) H^(-4/3)
    if constexpr (sizeof(Real) == 4) {
      const float r = __builtin_amdgcn_rsqf(Hs);
      iH = r * r;
      Hm43 = friction == 0 ? __builtin_amdgcn_exp2f(-1.3333333333333333f * __builtin_amdgcn_logf(Hs)) : 0.0f;
    } else {
      const Real r = rsq(Hs);
      iH = r * r;
      Hm43 = friction == 0 ? rpow43(Hs) : Real(0);
    }
    const Real u = wq[1] * iH, vv_ = wq[2] * iH;
    const Real Pq = Real(0.5) * g * wq[0] * (wq[0] + Real(2) * hq);
    const Real spd = dsqrt(wq[1] * wq[1] + wq[2] * wq[2]) * iH;
    const Real tau = (friction == 0) ? gn2 * spd * Hm43 : fc * spd * iH;
    const Real Fx[3] = {wq[1], wq[1] * u + Pq, wq[2] * u};
    const Real Fy[3] = {wq[2], wq[1] * vv_, wq[2] * vv_ + Pq};
    const Real s1 = g * wq[0] * dhx - tau * wq[1];
    const Real s2 = g * wq[0] * dhy - tau * wq[2];
    const Real Wq = Real(Tab<P>::qw(q));
    const Real wdet = Wq * detJ;
    if (P == 1) {
      // linear modes have constant gradients: weight the fluxes first
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        Sx[v] += Wq * Fx[v];
        Sy[v] += Wq * Fy[v];
      }
    }
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      if (m > 0 && P != 1) {
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
  if (P == 1) {
#pragma unroll
    for (int m = 1; m < 3; ++m) {
      const Real dr = Real(B<P>::QR(0, m)), ds = Real(B<P>::QS(0, m));
      const Real gx = cx0 * dr + cx1 * ds, gy = cy0 * dr + cy1 * ds;
#pragma unroll
      for (int v = 0; v < 3; ++v) acc[v][m] += gx * Sx[v] + gy * Sy[v];
    }
  }
}

// Basis values, gradients, barycentric weights and weights at the area
// points, as a table in constant memory (built at compile time from the
// same closed forms) for the p = 2 loop below.
template <typename Real, int P>
struct AreaTable {
  Real Q[Tab<P>::NQ][Tab<P>::NP], QR[Tab<P>::NQ][Tab<P>::NP], QS[Tab<P>::NQ][Tab<P>::NP];
  Real L[Tab<P>::NQ][3], W[Tab<P>::NQ];
};
template <typename Real, int P>
constexpr AreaTable<Real, P> make_area_table() {
  AreaTable<Real, P> t{};
  for (int q = 0; q < Tab<P>::NQ; ++q) {
    for (int m = 0; m < Tab<P>::NP; ++m) {
      t.Q[q][m] = Real(B<P>::Q(q, m));
      t.QR[q][m] = Real(B<P>::QR(q, m));
      t.QS[q][m] = Real(B<P>::QS(q, m));
    }
    for (int i = 0; i < 3; ++i) t.L[q][i] = Real(lam_(i, Tab<P>::qr(q), Tab<P>::qs(q)));
    t.W[q] = Real(Tab<P>::qw(q));
  }
  return t;
}
__constant__ AreaTable<float, 2> c_area2f = make_area_table<float, 2>();
__constant__ AreaTable<double, 2> c_area2d = make_area_table<double, 2>();
__constant__ AreaTable<float, 3> c_area3f = make_area_table<float, 3>();
__constant__ AreaTable<double, 3> c_area3d = make_area_table<double, 3>();

template <typename Real, int P>
DG_DEV const AreaTable<Real, P>& area_table() {
  static_assert(P == 2 || P == 3, "tables for p = 2 and 3");
  if constexpr (P == 2)
    return *reinterpret_cast<const AreaTable<Real, 2>*>(
        sizeof(Real) == 4 ? static_cast<const void*>(&c_area2f) : static_cast<const void*>(&c_area2d));
  else
    return *reinterpret_cast<const AreaTable<Real, 3>*>(
        sizeof(Real) == 4 ? static_cast<const void*>(&c_area3f) : static_cast<const void*>(&c_area3d));
}

// Fluxes and sources at one area point (Eq. SWE: advective flux, pressure,
// bed slope, friction), from the point's state wq, bathymetry hq, bed
// gradient (dhx, dhy), the element's det J J^{-T} entries and quadrature
// weight Wq: the fluxes mapped to the reference directions, Gr = Wq (cx0 Fx
// + cy0 Fy), Gs = Wq (cx1 Fx + cy1 Fy), and the momentum sources s1, s2.
template <typename Real>
DG_DEV void area_point(const Real (&wq)[3], Real hq, Real dhx, Real dhy, Real cx0, Real cx1, Real cy0, Real cy1,
                       Real fc, Real gn2, int friction, Real g, Real H0, Real Wq, Real (&Gr)[3], Real (&Gs)[3],
                       Real& s1, Real& s2) {
  const Real Hs = dmax(wq[0] + hq, H0);
  Real iH, Hm43;
  if constexpr (sizeof(Real) == 4) {
    const float r = __builtin_amdgcn_rsqf(Hs);
    iH = r * r;
    Hm43 = friction == 0 ? __builtin_amdgcn_exp2f(-1.3333333333333333f * __builtin_amdgcn_logf(Hs)) : 0.0f;
  } else {
    const Real r = rsq(Hs);
    iH = r * r;
    Hm43 = friction == 0 ? rpow43(Hs) : Real(0);
  }
  const Real u = wq[1] * iH, vv_ = wq[2] * iH;
  const Real Pq = Real(0.5) * g * wq[0] * (wq[0] + Real(2) * hq);
  const Real spd = dsqrt(wq[1] * wq[1] + wq[2] * wq[2]) * iH;
  const Real tau = (friction == 0) ? gn2 * spd * Hm43 : fc * spd * iH;
  const Real Fx[3] = {wq[1], wq[1] * u + Pq, wq[2] * u};
  const Real Fy[3] = {wq[2], wq[1] * vv_, wq[2] * vv_ + Pq};
  s1 = g * wq[0] * dhx - tau * wq[1];
  s2 = g * wq[0] * dhy - tau * wq[2];
  // the weight goes into the four mapping coefficients once
  const Real ax = Wq * cx0, ay = Wq * cy0, bx = Wq * cx1, by = Wq * cy1;
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    Gr[v] = ax * Fx[v] + ay * Fy[v];
    Gs[v] = bx * Fx[v] + by * Fy[v];
  }
}

// p >= 2 area integrals: one quadrature point per loop trip with the table
// above (the unrolled form keeps far more registers live than the 3 Np
// accumulators need).  Per point the fluxes are mapped once to the
// reference directions (area_point), then every mode takes dphi/dr Gr +
// dphi/ds Gs.
template <typename Real, int P>
DG_DEV void area_terms_table(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], Real cx0, Real cx1, Real cy0,
                             Real cy1, Real detJ, Real idet, Real fc, int friction, Real g, Real H0,
                             Real (&acc)[3][Tab<P>::NP]) {
  constexpr int NP = Tab<P>::NP;
  const AreaTable<Real, P>& T = area_table<Real, P>();
  const Real dhr = Real(0.5) * (hb[1] - hb[0]), dhs = Real(0.5) * (hb[2] - hb[0]);
  const Real dhx = (cx0 * dhr + cx1 * dhs) * idet, dhy = (cy0 * dhr + cy1 * dhs) * idet;
  const Real gn2 = g * fc * fc;
#pragma unroll 1
  for (int q = 0; q < Tab<P>::NQ; ++q) {
    Real wq[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Real s = Real(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) s += T.Q[q][m] * w[v][m];
      wq[v] = s;
    }
    const Real hq = T.L[q][0] * hb[0] + T.L[q][1] * hb[1] + T.L[q][2] * hb[2];
    const Real Wq = T.W[q];
    const Real wdet = Wq * detJ;
    Real Gr[3], Gs[3], s1, s2;
    area_point<Real>(wq, hq, dhx, dhy, cx0, cx1, cy0, cy1, fc, gn2, friction, g, H0, Wq, Gr, Gs, s1, s2);
    const Real s1w = wdet * s1, s2w = wdet * s2;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      if (m > 0) {
        const Real dr = T.QR[q][m], ds = T.QS[q][m];
        // two fused multiply-adds into the accumulator (written as
        // acc + (dr Gr + ds Gs) the sum would take a third instruction)
#pragma unroll
        for (int v = 0; v < 3; ++v) acc[v][m] = fmac(ds, Gs[v], fmac(dr, Gr[v], acc[v][m]));
      }
      acc[1][m] = fmac(T.Q[q][m], s1w, acc[1][m]);
      acc[2][m] = fmac(T.Q[q][m], s2w, acc[2][m]);
    }
  }
}

// p = 3 area integrals on the matrix cores, FP32, for one wavefront of 64
// elements (lane l holds element l of the tile).  Per block of 16 elements:
// the state at the 16 area points is the product Q (16 points x 10 modes)
// times U (10 modes x 16 elements), three 16x16x4 products per variable with
// the modes padded to 12; each lane forms the fluxes and sources of the four
// points it holds (area_point); the projections back onto the modes are
// four products per operand (Gr against dphi/dr, Gs against dphi/ds, the
// momentum sources against phi), the points split over the four K-slices
// so that a lane's four point values are its B operands as they stand; the
// rows of the result return to the element's lane by cross-lane reads.
// v_mfma_f32_16x16x4f32 (one block): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16] and holds D[4 (l / 16) + r][l % 16] in register r.
// s_w: row v * 10 + m holds mode m of variable v for the 64 elements;
// s_hb, s_ev, s_fc: their vertex bathymetry, edge vectors and friction.
DG_DEV void area_terms_mfma_p3(const float (*s_w)[64], const float (*s_hb)[64], const float (*s_ev)[64],
                               const float* s_fc, int friction, float g, float H0, float (&acc)[3][10]) {
  typedef float f4 __attribute__((ext_vector_type(4)));
  constexpr int NP = 10;
  const AreaTable<float, 3>& AT = area_table<float, 3>();
  const int lane = threadIdx.x & 63, hi = lane >> 4, lo = lane & 15;
  // A of the point evaluation: Q[q = lo][m = 4 s + hi]
  float aQ[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const int m = 4 * s + hi;
    aQ[s] = m < NP ? AT.Q[lo][m < NP ? m : 0] : 0.0f;
  }
  // A of the projections at q = 4 hi + s, m = lo (dphi/dr, dphi/ds vanish for m = 0)
  float aR[4], aS[4], aP[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int q = 4 * hi + s, m = lo < NP ? lo : 0;
    aR[s] = (lo >= 1 && lo < NP) ? AT.QR[q][m] : 0.0f;
    aS[s] = (lo >= 1 && lo < NP) ? AT.QS[q][m] : 0.0f;
    aP[s] = lo < NP ? AT.Q[q][m] : 0.0f;
  }
#pragma unroll 1
  for (int b = 0; b < 4; ++b) {
    const int ee = 16 * b + lo;                     // the element whose points this lane holds
    f4 D[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      D[v] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const int m = 4 * s + hi;
        const float u = s_w[v * NP + (m < NP ? m : NP - 1)][ee];
        D[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(aQ[s], m < NP ? u : 0.0f, D[v], 0, 0, 0);
      }
    }
    // element ee's geometry (as load_elem forms it) and bed gradient
    const float ex0 = s_ev[0][ee], ey0 = s_ev[1][ee], ex2 = s_ev[4][ee], ey2 = s_ev[5][ee];
    const float hb0 = s_hb[0][ee], hb1 = s_hb[1][ee], hb2 = s_hb[2][ee], fc = s_fc[ee];
    const float detJ = 0.25f * (ex2 * ey0 - ex0 * ey2);
    const float idet = rcp(detJ);
    const float cx0 = -0.5f * ey2, cx1 = -0.5f * ey0, cy0 = 0.5f * ex2, cy1 = 0.5f * ex0;
    const float dhr = 0.5f * (hb1 - hb0), dhs = 0.5f * (hb2 - hb0);
    const float dhx = (cx0 * dhr + cx1 * dhs) * idet, dhy = (cy0 * dhr + cy1 * dhs) * idet;
    const float gn2 = g * fc * fc;
    f4 X[3], Y[3], Z1, Z2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * hi + r;
      const float wq[3] = {D[0][r], D[1][r], D[2][r]};
      const float hq = AT.L[q][0] * hb0 + AT.L[q][1] * hb1 + AT.L[q][2] * hb2;
      const float Wq = AT.W[q];
      float Gr[3], Gs[3], s1, s2;
      area_point<float>(wq, hq, dhx, dhy, cx0, cx1, cy0, cy1, fc, gn2, friction, g, H0, Wq, Gr, Gs, s1, s2);
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        X[v][r] = Gr[v];
        Y[v][r] = Gs[v];
      }
      const float wdet = Wq * detJ;
      Z1[r] = wdet * s1;
      Z2[r] = wdet * s2;
    }
    f4 Dp[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Dp[v] = f4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        Dp[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(aR[s], X[v][s], Dp[v], 0, 0, 0);
        Dp[v] = __builtin_amdgcn_mfma_f32_16x16x4f32(aS[s], Y[v][s], Dp[v], 0, 0, 0);
      }
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      Dp[1] = __builtin_amdgcn_mfma_f32_16x16x4f32(aP[s], Z1[s], Dp[1], 0, 0, 0);
      Dp[2] = __builtin_amdgcn_mfma_f32_16x16x4f32(aP[s], Z2[s], Dp[2], 0, 0, 0);
    }
    // mode m of element 16 b + lo sits in lane 16 (m / 4) + lo, register m % 4
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const int src = (16 * (m >> 2) + lo) << 2;
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        const float x = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(Dp[v][m & 3])));
        if (hi == b) acc[v][m] += x;
      }
    }
  }
}

template <typename Real, int P>
DG_DEV void area_terms(const Real (&w)[3][Tab<P>::NP], const Real (&hb)[3], Real cx0, Real cx1, Real cy0, Real cy1,
                       Real detJ, Real idet, Real fc, int friction, Real g, Real H0, Real (&acc)[3][Tab<P>::NP]) {
  if constexpr (P >= 2)
    area_terms_table<Real, P>(w, hb, cx0, cx1, cy0, cy1, detJ, idet, fc, friction, g, H0, acc);
  else
    area_terms_unrolled<Real, P>(w, hb, cx0, cx1, cy0, cy1, detJ, idet, fc, friction, g, H0, acc);
}

// Wind stress and atmospheric pressure (F_x, F_y of Eq. SWE): the nodal
// kinematic stress and pressure head of t^n are linear in the element, so
// grad psi is constant; at each area point the momentum rows take
// tau - g H grad psi with H = zeta + h_b.
// The storm's kinematic wind stress (tx, ty) and pressure head (ps) at the
// element's three vertices (node ids tn), from the nodal arrays of t^n.
template <typename Real>
DG_DEV void met_nodes(const Member<Real>& M, const int (&tn)[3], Real (&tx)[3], Real (&ty)[3], Real (&ps)[3]) {
  const int nn = M.n_nodes;
  const DG_G Real* __restrict__ met = gp(M.met);
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    tx[i] = ldx(met, tn[i]);
    ty[i] = ldc(met, nn, tn[i]);
    ps[i] = ldc(met, 2 * nn, tn[i]);
  }
}

template <typename Real, int P>
DG_DEV void met_terms(const Real (&tx)[3], const Real (&ty)[3], const Real (&ps)[3], const Real (&w)[3][Tab<P>::NP],
                      const Real (&hb)[3], Real cx0, Real cx1, Real cy0, Real cy1, Real detJ, Real idet, Real g,
                      Real (&acc)[3][Tab<P>::NP]) {
  constexpr int NP = Tab<P>::NP;
  const Real pr = Real(0.5) * (ps[1] - ps[0]), pq = Real(0.5) * (ps[2] - ps[0]);
  const Real px = (cx0 * pr + cx1 * pq) * idet, py = (cy0 * pr + cy1 * pq) * idet;
  auto point = [&](Real L0, Real L1, Real L2, Real zq, Real wdet, const Real* Qm) {
    const Real Hq = zq + (L0 * hb[0] + L1 * hb[1] + L2 * hb[2]);
    const Real s1 = (L0 * tx[0] + L1 * tx[1] + L2 * tx[2]) - g * Hq * px;
    const Real s2 = (L0 * ty[0] + L1 * ty[1] + L2 * ty[2]) - g * Hq * py;
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const Real c = wdet * Qm[m];
      acc[1][m] += c * s1;
      acc[2][m] += c * s2;
    }
  };
  if constexpr (P >= 2) {
    const AreaTable<Real, P>& T = area_table<Real, P>();
#pragma unroll 1
    for (int q = 0; q < Tab<P>::NQ; ++q) {
      Real zq = Real(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) zq += T.Q[q][m] * w[0][m];
      Real Qm[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) Qm[m] = T.Q[q][m];
      point(T.L[q][0], T.L[q][1], T.L[q][2], zq, T.W[q] * detJ, Qm);
    }
  } else {
#pragma unroll
    for (int q = 0; q < Tab<P>::NQ; ++q) {
      const double qr = Tab<P>::qr(q), qs = Tab<P>::qs(q);
      Real zq = Real(0), Qm[NP];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        Qm[m] = Real(B<P>::Q(q, m));
        zq += Qm[m] * w[0][m];
      }
      point(Real(lam_(0, qr, qs)), Real(lam_(1, qr, qs)), Real(lam_(2, qr, qs)), zq, Real(Tab<P>::qw(q)) * detJ, Qm);
    }
  }
}

// Element rain rate (Eq. rain).  With time-dependent rain the first stage of
// a step averages the nodal rates of t^n (rain_node_kernel), stores R for the
// later stages and returns the element's rain volume rate in part.
template <typename Real>
DG_DEV Real element_rain(const Member<Real>& M, const StageArgs& A, int E, int e, int ec, bool valid,
                         const Real (&ex)[3], const Real (&ey)[3], double& part) {
  if (A.stage == 0 && M.fo.rain_kind != RAIN_CONST) {
    const DG_G double* __restrict__ rn = gp(M.rn);
    const DG_G int* __restrict__ tri = gp(M.tri);
    const double r = (ldx(rn, ldx(tri, ec)) + ldx(rn, ldc(tri, E, ec)) + ldx(rn, ldc(tri, 2 * E, ec))) / 3.0;
    const Real R = Real(r);
    if (valid) stx(gp(M.R), e, R);
    const double area = 0.5 * (double(ex[2]) * double(ey[0]) - double(ex[0]) * double(ey[2]));
    part = valid ? area * double(R) : 0.0;
    return R;
  }
  part = 0.0;
  return ldx(gp(M.R), ec);
}

// w^n of the element when the stage blends it (a != 0), else zeros; loaded
// before the edge accumulation so that the loads overlap it.
template <typename Real, int P>
DG_DEV void load_blend(const Member<Real>& M, const StageArgs& A, int E, int ec, Real (&w0v)[3][Tab<P>::NP]) {
  constexpr int NP = Tab<P>::NP;
  if (A.a != 0.0) {
    const DG_G Real* __restrict__ W0 = gp(M.W[0]);
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int m = 0; m < NP; ++m) w0v[v][m] = ldc(W0, (v * NP + m) * E, ec);
  } else {
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int m = 0; m < NP; ++m) w0v[v][m] = Real(0);
  }
}

// Inverse mass, SSP combination, positive-depth operator (LIM = 0) or the
// fully-wet byte (LIM = 1), stores, and the wavefront's partials.  tile
// counts workgroups of T elements.
template <typename Real, int P, int LIM, int T = TILE>
DG_DEV void finish_stage(const Member<Real>& M, const StageArgs& A, int tile, int e, int ec, bool valid, int E,
                         Real (&w)[3][Tab<P>::NP], Real (&acc)[3][Tab<P>::NP], const Real (&hb)[3], const Real (&ex)[3],
                         const Real (&ey)[3], Real detJ, Real idet, double dt, double bout, double bin, Real Rv,
                         double rain_part, const Real (&w0v)[3][Tab<P>::NP]) {
  constexpr int NP = Tab<P>::NP;
  acc[0][0] += Real(2) * detJ * Rv;
  const Real cdt = Real(A.gam * dt);
  const Real ca = Real(A.a), cb = Real(A.b);
  // w <- a w^n + b w + (b gam dt / (det J m_k)) acc, one coefficient per mode
  Real km[NP];
  const Real bcd = cb * cdt * idet;
#pragma unroll
  for (int m = 0; m < NP; ++m) km[m] = bcd * Real(1.0 / mass_(m));
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) w[v][m] = km[m] * acc[v][m] + (cb * w[v][m] + ca * w0v[v][m]);
  double part[5] = {bout, bin, 0.0, __builtin_inf(), 0.0};
  bool neg = false, bad = false;      // negative / non-finite mean depth or speed (last stage)
  if (LIM == 0) {
    double hv[3], qxv[3], qyv[3];
    bool filled;
    // FP64 members keep the FP64 vertex values for the CFL speed
    const bool need_v = A.last != 0 && sizeof(Real) == 8;
    const bool dry = positive_depth<Real, P>(w, hb, M.H0, hv, qxv, qyv, need_v, filled);
    if (valid) {
      DG_G Real* __restrict__ Wout = gp(M.W[A.out_buf]);
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) stc(Wout, (v * NP + m) * E, e, w[v][m]);
      stx(gp(M.F[A.fout]), e, uint8_t(dry ? 1 : 0));
    }
    if (A.last) {
      const double lam = post_speed<Real, P>(filled, hv, qxv, qyv, w, hb, M.H0, M.g);
      const double area = 0.5 * (double(ex[2]) * double(ey[0]) - double(ex[0]) * double(ey[2]));
      const double md = double(w[0][0]) + (double(hb[0]) + double(hb[1]) + double(hb[2])) / 3.0;
      part[2] = valid ? area * md : 0.0;
      part[3] = (valid && lam > 0.0) ? double(ldx(gp(M.din), ec)) * rcp(lam) : __builtin_inf();
      part[4] = (valid && dry) ? 1.0 : 0.0;
      neg = valid && md < 0.0;
      bad = valid && !(__builtin_isfinite(md) && __builtin_isfinite(lam));
    }
  } else {
    if (valid) {
      // raw stage output; the post pass limits it in place
      DG_G Real* __restrict__ Wr = gp(M.W[A.out_buf]);
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) stc(Wr, (v * NP + m) * E, e, w[v][m]);
      stx(gp(M.fullwet[A.stage & 1]), e, uint8_t(fully_wet<Real, P>(w, hb, M.H0) ? 1 : 0));
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // bout/bin: volume out of and into this lane's element through its boundary edges
  const bool rain_here = A.stage == 0 && M.fo.rain_kind != RAIN_CONST;
  // most tiles have no boundary edge: skip those sums when the wavefront holds only zeros
  const bool any_b = __any(part[0] != 0.0 || part[1] != 0.0);
  const double s0 = any_b ? wave_sum(part[0]) : 0.0, s1 = any_b ? wave_sum(part[1]) : 0.0;
  double s2 = 0.0, s4 = 0.0, s5 = 0.0, s6 = 0.0, mn = __builtin_inf(), fb = __builtin_inf();
  if (LIM == 0 && A.last) {
    s2 = wave_sum(part[2]);
    s4 = double(__popcll(__ballot(part[4] != 0.0)));
    mn = wave_min(part[3]);
    s6 = double(__popcll(__ballot(neg)));
    fb = first_lane_id(__ballot(bad), tile * T + wv * 64);
  }
  if (rain_here) s5 = wave_sum(rain_part);
  // this wavefront's slot of the partials (a 512-element tile's second
  // half can lie past the last 256-element tile)
  const size_t row = part_row(M.n_tiles);
  const size_t slot = size_t(tile) * (T / 64) + wv;
  if (lane == 0 && slot < row) {
    DG_G double* __restrict__ pt = gp(A.part ? A.part : M.part);
    pt[(P_OUT0 + A.stage) * row + slot] = s0;
    pt[(P_IN0 + A.stage) * row + slot] = s1;
    if (LIM == 0 && A.last) {
      pt[P_VOL * row + slot] = s2;
      pt[P_MINR * row + slot] = mn;
      pt[P_NDRY * row + slot] = s4;
      pt[P_NNEG * row + slot] = s6;
      pt[P_BAD * row + slot] = fb;
    }
    if (rain_here) pt[P_RAIN * row + slot] = s5;
  }
}

// Own data of an element: modes, vertex bathymetry, edge vectors, Jacobian.
template <typename Real, int P>
struct ElemData {
  Real w[3][Tab<P>::NP];
  Real ex[3], ey[3], hb[3];
  Real detJ, idet, cx0, cx1, cy0, cy1;
};

template <typename Real, int P>
DG_DEV void load_elem(const Member<Real>& M, const DG_G Real* __restrict__ Win, int E, int ec, ElemData<Real, P>& d) {
  constexpr int NP = Tab<P>::NP;
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) d.w[v][m] = ldc(Win, (v * NP + m) * E, ec);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d.ex[k] = ldc(gp(M.ev), (2 * k) * E, ec);
    d.ey[k] = ldc(gp(M.ev), (2 * k + 1) * E, ec);
    d.hb[k] = ldc(gp(M.hbv), k * E, ec);
  }
  d.detJ = Real(0.25) * (d.ex[2] * d.ey[0] - d.ex[0] * d.ey[2]);
  d.idet = rcp(d.detJ);
  // det J * J^{-T} = [[-e2y, -e0y], [e2x, e0x]] / 2
  d.cx0 = Real(-0.5) * d.ey[2];
  d.cx1 = Real(-0.5) * d.ey[0];
  d.cy0 = Real(0.5) * d.ex[2];
  d.cy1 = Real(0.5) * d.ex[0];
}

// ------------------------------------------------- stage kernel, per element
// Every element evaluates its three edges itself (interior edge fluxes are
// computed by both neighbours).  LIM = 0: full stage + positive-depth
// operator; LIM = 1: unlimited stage output to the stage's output buffer
// plus the fully-wet byte (the post kernel limits it there).
template <typename Real, int P, int FLUX, int LIM>
__global__ DG_STAGE_ATTR void stage_kernel(const Member<Real>* __restrict__ mem,
                                                     const Tile* __restrict__ tiles, int n_tiles, StageArgs A) {
  constexpr int NP = Tab<P>::NP, NG = Tab<P>::NG;
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = A.single ? Tile{0, ti} : tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const DG_G Scalars* __restrict__ sc = gp((const Scalars*)M.sc);
  if (!sc->active) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const Real g = Real(M.g), H0 = Real(M.H0);
  const Real feps = Real(M.feps);
  const double dt = sc->dt;
  const DG_G Real* __restrict__ Win = gp(M.W[A.in_buf]);
  const DG_G uint8_t* __restrict__ Fin = gp(M.F[A.fin]);
  ElemData<Real, P> d;
  load_elem<Real, P>(M, Win, E, ec, d);
  const bool myflag = ldx(Fin, ec) & 1;
  // w^n for the blend: read before the edges, so that its loads overlap
  // them, except at p = 3, where holding it through the edge loop would cost
  // 30 registers per value (15 more wavefronts' worth of registers)
  constexpr bool kLateBlend = P >= 3;
  Real w0v[3][NP];
  if constexpr (!kLateBlend) load_blend<Real, P>(M, A, E, ec, w0v);
  const uint8_t nkp = ldx(gp(M.nk), ec);
  Real acc[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) acc[v][m] = Real(0);
  Real vv[3][3], mv[3][3];
  edge_nodes<Real, P>(d.w, vv, mv);
  double bout = 0.0, bin = 0.0;
  // Neighbour ids, then (where registers allow) the three neighbours' modes
  // and flags, are read together, so the edges wait for memory once rather
  // than once each.  A boundary edge reads the element itself (unused).
  constexpr bool kHoist = P == 1 || (P == 2 && sizeof(Real) == 4);
  int nbv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) nbv[k] = ldc(gp(M.nbr), k * E, ec);
  Real wnb[kHoist ? 3 : 1][3][NP];
  bool nfl[3] = {false, false, false};
  if constexpr (kHoist) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int n = nbv[k] < 0 ? ec : nbv[k];
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) wnb[k][v][m] = ldc(Win, (v * NP + m) * E, n);
      nfl[k] = ldx(Fin, n) & 1;
    }
  }
  // edges and Gauss points are expanded at compile time, so every basis
  // value below is a constant (p = 3 bodies are too large for the unroller)
  static_for<3>([&](auto kc) {
    constexpr int k = decltype(kc)::value;
    constexpr int k1 = (k + 1) % 3;
    Real ell, il;
    edge_length<Real>(d.ex[k], d.ey[k], ell, il);
    const Real nx = d.ey[k] * il, ny = -d.ex[k] * il;
    const Real half = Real(0.5) * ell;
    const int nb = nbv[k];
    if (nb >= 0) {
      const int kn = (nkp >> (2 * k)) & 3;
      Real wn[3][NP];
      bool nflag;
      // p = 3: both sides' traces at every Gauss point of their own
      // parametrisation, the neighbour's one variable at a time, so that only
      // ten of its modes are held at once
      Real tO[3][NG], tN[3][NG];
      if constexpr (kHoist) {
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int m = 0; m < NP; ++m) wn[v][m] = wnb[k][v][m];
        nflag = nfl[k];
      } else if constexpr (P >= 3) {
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Real wv[NP];
#pragma unroll
          for (int m = 0; m < NP; ++m) wv[m] = ldc(Win, (v * NP + m) * E, nb);
          static_for<NG>([&](auto gc) {
            constexpr int gg = decltype(gc)::value;
            tO[v][gg] = trace_modal<Real, P, gg>(d.w[v], k);
            tN[v][gg] = trace_modal<Real, P, gg>(wv, kn);
          });
        }
        nflag = ldx(Fin, nb) & 1;
      } else {
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int m = 0; m < NP; ++m) wn[v][m] = ldc(Win, (v * NP + m) * E, nb);
        nflag = ldx(Fin, nb) & 1;
      }
      Real nvv[3][3], nmv[3][3];
      if constexpr (P <= 2) edge_nodes<Real, P>(wn, nvv, nmv);
      const int kn1 = kn == 2 ? 0 : kn + 1;
      const bool meL = e < nb;
      Real La[3], Lc[3], Lb[3], Ra[3], Rc[3], Rb[3];
#pragma unroll
      for (int v = 0; v < 3 && P <= 2; ++v) {
        const Real oa = vv[v][k], oc = mv[v][k], ob = vv[v][k1];
        const Real na = kn == 0 ? nvv[v][0] : kn == 1 ? nvv[v][1] : nvv[v][2];
        const Real nc = kn == 0 ? nmv[v][0] : kn == 1 ? nmv[v][1] : nmv[v][2];
        const Real nbv = kn1 == 0 ? nvv[v][0] : kn1 == 1 ? nvv[v][1] : nvv[v][2];
        La[v] = meL ? oa : na; Lc[v] = meL ? oc : nc; Lb[v] = meL ? ob : nbv;
        Ra[v] = meL ? na : oa; Rc[v] = meL ? nc : oc; Rb[v] = meL ? nbv : ob;
      }
      const Real hLa = meL ? d.hb[k] : d.hb[k1], hLb = meL ? d.hb[k1] : d.hb[k];
      const Real lnx = meL ? nx : -nx, lny = meL ? ny : -ny;
      const bool dryL = meL ? myflag : nflag, dryR = meL ? nflag : myflag;
      static_for<NG>([&](auto gc) {
        constexpr int gL = decltype(gc)::value;
        constexpr int gR = NG - 1 - gL;
        W3<Real> a, b;
        if constexpr (P <= 2) {
          a = {trace<Real, P>(La[0], Lc[0], Lb[0], gL), trace<Real, P>(La[1], Lc[1], Lb[1], gL),
               trace<Real, P>(La[2], Lc[2], Lb[2], gL)};
          b = {trace<Real, P>(Ra[0], Rc[0], Rb[0], gR), trace<Real, P>(Ra[1], Rc[1], Rb[1], gR),
               trace<Real, P>(Ra[2], Rc[2], Rb[2], gR)};
        } else {
          // cubic traces come from the modes (L side at gL, R side at gR)
          Real tL[3], tR[3];
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            tL[v] = meL ? tO[v][gL] : tN[v][gL];
            tR[v] = meL ? tN[v][gR] : tO[v][gR];
          }
          a = {tL[0], tL[1], tL[2]};
          b = {tR[0], tR[1], tR[2]};
        }
        const Real hg = Real(lag_(1, 0, gl_t(P, gL))) * hLa + Real(lag_(1, 1, gl_t(P, gL))) * hLb;
        Real FL[3], FR[3];
        interior_point<FLUX>(a, b, hg, lnx, lny, g, H0, feps, dryL, dryR, meL, !meL, FL, FR);
        const Real wg = half * Real(gl_w(P, gL));
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const Real ph = meL ? Real(B<P>::EG(k, gL, m)) : Real(B<P>::EG(k, gR, m));
          const Real c = wg * ph;
          acc[0][m] -= c * (meL ? FL[0] : FR[0]);
          acc[1][m] -= c * (meL ? FL[1] : FR[1]);
          acc[2][m] -= c * (meL ? FL[2] : FR[2]);
        }
      });
    } else {
      const int code = -1 - nb;
      const int type = code & 3, slot = code >> 2;
      const Real tide = Real(sc->tide[A.stage][slot]), qr = Real(sc->river[A.stage][slot]);
      double fm = 0.0;
      static_for<NG>([&](auto gc) {
        constexpr int gi = decltype(gc)::value;
        W3<Real> a;
        if constexpr (P <= 2)
          a = {trace<Real, P>(vv[0][k], mv[0][k], vv[0][k1], gi), trace<Real, P>(vv[1][k], mv[1][k], vv[1][k1], gi),
               trace<Real, P>(vv[2][k], mv[2][k], vv[2][k1], gi)};
        else
          a = {trace_modal<Real, P, gi>(d.w[0], k), trace_modal<Real, P, gi>(d.w[1], k),
               trace_modal<Real, P, gi>(d.w[2], k)};
        const Real hg = Real(lag_(1, 0, gl_t(P, gi))) * d.hb[k] + Real(lag_(1, 1, gl_t(P, gi))) * d.hb[k1];
        Real F[3];
        boundary_point<FLUX>(a, hg, nx, ny, g, H0, type, tide, qr, F);
        const Real wg = half * Real(gl_w(P, gi));
        fm += double(wg * F[0]);
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const Real c = wg * Real(B<P>::EG(k, gi, m));
          acc[0][m] -= c * F[0];
          acc[1][m] -= c * F[1];
          acc[2][m] -= c * F[2];
        }
      });
      if (fm > 0.0) bout += fm; else bin -= fm;
    }
  });
  if constexpr (kLateBlend) load_blend<Real, P>(M, A, E, ec, w0v);
  area_terms<Real, P>(d.w, d.hb, d.cx0, d.cx1, d.cy0, d.cy1, d.detJ, d.idet, ldx(gp(M.fric), ec), M.friction, g, H0, acc);
  if (M.fo.met_kind != MET_NONE) {
    int tn[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) tn[i] = ldc(gp(M.tri), i * E, ec);
    Real tx[3], ty[3], ps[3];
    met_nodes<Real>(M, tn, tx, ty, ps);
    met_terms<Real, P>(tx, ty, ps, d.w, d.hb, d.cx0, d.cx1, d.cy0, d.cy1, d.detJ, d.idet, g, acc);
  }
  double rain_part;
  const Real Rv = element_rain<Real>(M, A, E, e, ec, valid, d.ex, d.ey, rain_part);
  // lanes past the end of the mesh evaluated a copy of the last element
  finish_stage<Real, P, LIM>(M, A, tl.tile, e, ec, valid, E, d.w, acc, d.hb, d.ex, d.ey, d.detJ, d.idet, dt,
                             valid ? bout : 0.0, valid ? bin : 0.0, Rv, rain_part, w0v);
}

// ---------------------------------------------------- stage kernel, per edge
// Same result, less arithmetic: the tile's point values go to LDS, every
// edge whose two sides are in the tile is evaluated once (by the thread of
// its lower-id element), and the lanes work through an LDS-compacted list of
// the tile's edges instead of three per element.  Edges to other tiles are
// still evaluated on both sides in the canonical orientation, so both tiles
// obtain the same bits.
//
// PRE = 1 (limiter on, p <= 2): the input is the previous stage's raw output,
// and this kernel applies that stage's post-processing (Sec. 2.3 limiter,
// Sec. 2.4 positive depth and flags) itself, to its own elements and to
// ring 1 of its tile (the outside elements across its cut edges), whose
// limited point values join the tile's in LDS: the previous stage needs no
// post pass, and cut edges read their neighbour from LDS.  The limiter of
// a ring-1 element reads the raw means of ring 2.  The arithmetic is the
// post kernel's (the same functions).
template <typename Real, int P, int FLUX, int LIM, int PRE, int T, int MF = 0>
__global__ DG_STAGE_ATTR_T(T) void stage_edge_kernel(const Member<Real>* __restrict__ mem,
                                                          const Tile* __restrict__ tiles, int n_tiles, StageArgs A) {
  constexpr int NP = Tab<P>::NP, NG = Tab<P>::NG;
  static_assert(!PRE || (LIM == 1 && P <= 2), "the fused post-processing needs the limiter and p <= 2");
  static_assert(T == 256 || ((T == 64 || T == 128 || (T == 512 && P == 1)) && !PRE),
                "tiles of 256; 64, 128 or (p = 1) 512 without the fused post-processing");
  // MF: the area integrals on the matrix cores (p = 3, FP32, one wavefront per tile)
  static_assert(!MF || (P == 3 && sizeof(Real) == 4 && T == 64 && !PRE), "matrix-core area integrals: p = 3, FP32, T = 64");
  constexpr int NW = T / 64;                            // wavefronts per workgroup
  constexpr int LB = T == 512 ? 9 : T == 256 ? 8 : T == 128 ? 7 : 6;   // bits of a local element index in an edge entry
  // point values per variable (vertices, midpoints); p = 3, p = 2 and FP64
  // p = 1 (but the fused kernel) keep their traces in s_flux instead (each
  // slot holds the element's own trace at that edge point until phase B
  // overwrites it with the flux there), which leaves the flux slots as the
  // only per-point LDS array (FP32 p = 1 measured faster with the vertex
  // values, three per variable against six traces)
  constexpr bool kTr = P == 3 || (P == 2 && !PRE) || (P == 1 && sizeof(Real) == 8 && !PRE);
  constexpr int NN = P == 1 ? 3 : P == 2 ? 6 : 1;
  constexpr int SL = T + (PRE ? HALO_R1 : 0);      // point-value slots: tile, then ring 1
  __shared__ Real s_node[kTr ? 1 : 3 * NN][SL];
  __shared__ Real s_hb[3][SL];
  __shared__ Real s_flux[3 * NG * 3][T];            // [(k NG + g) 3 + var][element], scaled by (l/2) w_g
  // edge vectors in LDS, except for FP32 p = 2, FP64 p = 1 and p = 3 on
  // 64-element tiles and the fused kernel, where dropping them (phase B
  // reads them from the cache instead) lets more workgroups share a CU
  // (FP64 p = 3: eight instead of six, with the 16-bit edge list below;
  // FP64 p = 1: fourteen, for three wavefronts per SIMD at 164 VGPRs)
  constexpr bool kEvLds = !PRE && !(P == 2 && sizeof(Real) == 4) && !(P != 2 && sizeof(Real) == 8 && T == 64);
  __shared__ Real s_ev[kEvLds ? 6 : 1][kEvLds ? T : 1];
  __shared__ uint8_t s_flag[SL];
  // PRE: raw means and fully-wet bytes of tile, ring 1 and ring 2, in the
  // flux slots' memory (used before phase B writes any flux)
  constexpr int SM = T + HALO_R1 + HALO_R2;
  static_assert(!PRE || 3 * SM * sizeof(Real) + SM <= sizeof(s_flux), "halo means fit the flux slots");
  Real* const s_mean = reinterpret_cast<Real*>(&s_flux[0][0]);
  uint8_t* const s_fw = reinterpret_cast<uint8_t*>(s_mean + 3 * SM);
  // edge list
  // (16-bit entries on 64-element tiles: 6 + 2 + 2 + 6 bits)
  using ListT = std::conditional_t<T == 64, uint16_t, uint32_t>;
  __shared__ double s_lbuf[3 * T * sizeof(ListT) / 8];
  ListT* s_list = reinterpret_cast<ListT*>(s_lbuf);
  __shared__ int s_wsum[2][NW];
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = A.single ? Tile{0, ti} : tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const DG_G Scalars* __restrict__ sc = gp((const Scalars*)M.sc);
  if (!sc->active) return;
  const int E = M.E;
  const int t0 = tl.tile * T;
  const int tend = t0 + T < E ? t0 + T : E;
  const int el = threadIdx.x;
  const int e = t0 + el;
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const Real g = Real(M.g), H0 = Real(M.H0);
  const Real feps = Real(M.feps);
  const double dt = sc->dt;
  const DG_G Real* __restrict__ Win = gp(M.W[A.in_buf]);
  const DG_G uint8_t* __restrict__ Fin = gp(M.F[A.fin]);
  const DG_G int* __restrict__ nbr = gp(M.nbr);

  // ---- phase A: own data, point values to LDS, owned-edge list, area terms
  ElemData<Real, P> d;
  load_elem<Real, P>(M, Win, E, ec, d);
  // neighbour ids, their edge codes, the dry flag and the friction are read
  // together with the element's own data, so phase A waits for memory once
  int nbv[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) nbv[k] = ldc(nbr, k * E, ec);
  const int nkp = ldx(gp(M.nk), ec);
  const uint8_t fin = PRE ? uint8_t(0) : ldx(Fin, ec);
  const Real fric = ldx(gp(M.fric), ec);
  // PRE: the own element's neighbour slots in the tile's numbering
  const uint32_t eslot = PRE ? ldx(gp(M.h_eslot), ec) : 0u;
  bool myflag = fin & 1;
  if constexpr (PRE) {
    // ---- phase 0: the previous stage's post-processing (limiter, positive
    // depth, flags) of the own element and of ring 1
    const DG_G uint8_t* __restrict__ fwin = gp(M.fullwet[(A.stage + 1) & 1]);   // written by stage - 1
    const int hoff = ldx(gp(M.h_off), tl.tile), hn1 = ldx(gp(M.h_n1), tl.tile);
    const int hn = ldx(gp(M.h_off), tl.tile + 1) - hoff;
    // every load of this phase is issued before the barrier: the own
    // limiter data, and (threads below hn1) one ring-1 element's raw state,
    // bathymetry and limiter data, in flight with the halo's means
    const uint8_t lc_own = ldx(gp(M.limc), ec);
    Real al_own[6];
#pragma unroll
    for (int j = 0; j < 6; ++j) al_own[j] = ldc(gp(M.lima), j * E, ec);
    const bool ring = el < hn1;
    const int y = ldx(gp(M.h_id), hoff + (ring ? el : 0));
    const uint32_t ns = ring ? ldx(gp(M.h_nslot), hoff + el) : 0u;
    Real wy[3][NP], hy[3], aly[6];
    uint8_t lcy = 0;
    if (ring) {
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) wy[v][m] = ldc(Win, (v * NP + m) * E, y);
#pragma unroll
      for (int k = 0; k < 3; ++k) hy[k] = ldc(gp(M.hbv), k * E, y);
#pragma unroll
      for (int j = 0; j < 6; ++j) aly[j] = ldc(gp(M.lima), j * E, y);
      lcy = ldx(gp(M.limc), y);
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) s_mean[v * SM + el] = d.w[v][0];
    s_fw[el] = valid ? ldx(fwin, ec) : uint8_t(0);
    for (int j = el; j < hn; j += T) {
      const int z = ldx(gp(M.h_id), hoff + j);
#pragma unroll
      for (int v = 0; v < 3; ++v) s_mean[v * SM + T + j] = ldc(Win, (v * NP) * E, z);
      s_fw[T + j] = ldx(fwin, z);
    }
    __syncthreads();
    myflag = post_from_slots<Real, P>(M, d.w, d.hb, lc_own, al_own, eslot, el, s_mean, s_fw, SM);
    if (ring) {
      const bool fy = post_from_slots<Real, P>(M, wy, hy, lcy, aly, ns, T + el, s_mean, s_fw, SM);
      Real vv[3][3], mv[3][3];
      edge_nodes<Real, P>(wy, vv, mv);
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          s_node[v * NN + i][T + el] = vv[v][i];
          if (P == 2) s_node[v * NN + 3 + i][T + el] = mv[v][i];
        }
#pragma unroll
      for (int k = 0; k < 3; ++k) s_hb[k][T + el] = hy[k];
      s_flag[T + el] = fy ? 1 : 0;
    }
  }
  // element rain (Eq. rain): the first stage of a step with time-dependent
  // rain averages the nodal rates of t^n (node ids now, rates before phase
  // B, the mean at the end); later stages read the stored value
  // (the stored value is read in both cases: a load in one branch only would
  // make the other wait for every load in flight before reusing its register)
  const bool rain_avg = A.stage == 0 && M.fo.rain_kind != RAIN_CONST;
  const bool met_on = M.fo.met_kind != MET_NONE;
  // FP32: the storm's wind and pressure at the vertices are read before
  // phase A's arithmetic (FP64, with twice the registers per value, reads
  // them just before the area terms, which measured faster there)
  constexpr bool kMetEarly = sizeof(Real) == 4;
  Real Rv = ldx(gp(M.R), ec);
  int tn[3] = {0, 0, 0};
  if (rain_avg || (kMetEarly && met_on)) {
#pragma unroll
    for (int i = 0; i < 3; ++i) tn[i] = ldc(gp(M.tri), i * E, ec);
  }
  Real mtx[3] = {Real(0), Real(0), Real(0)}, mty[3] = {Real(0), Real(0), Real(0)}, mps[3] = {Real(0), Real(0), Real(0)};
  if (kMetEarly && met_on) met_nodes<Real>(M, tn, mtx, mty, mps);
  if constexpr (P <= 2 && kTr) {
    // the same point-value interpolant as the fused kernel's phase B, so
    // both give the same bits
    Real vv[3][3], mv[3][3];
    edge_nodes<Real, P>(d.w, vv, mv);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
      for (int gg = 0; gg < NG; ++gg)
#pragma unroll
        for (int v = 0; v < 3; ++v)
          s_flux[(k * NG + gg) * 3 + v][el] = trace<Real, P>(vv[v][k], mv[v][k], vv[v][k == 2 ? 0 : k + 1], gg);
  } else if constexpr (P <= 2) {
    Real vv[3][3], mv[3][3];
    edge_nodes<Real, P>(d.w, vv, mv);
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        s_node[v * NN + i][el] = vv[v][i];
        if (P == 2) s_node[v * NN + 3 + i][el] = mv[v][i];
      }
  } else {
    static_for<3>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      static_for<NG>([&](auto gc) {
        constexpr int gg = decltype(gc)::value;
#pragma unroll
        for (int v = 0; v < 3; ++v) s_flux[(k * NG + gg) * 3 + v][el] = trace_modal<Real, P, gg>(d.w[v], k);
      });
    });
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    s_hb[k][el] = d.hb[k];
    if constexpr (kEvLds) {
      s_ev[2 * k][el] = d.ex[k];
      s_ev[2 * k + 1][el] = d.ey[k];
    }
  }
  s_flag[el] = myflag ? 1 : 0;
  if constexpr (MF) s_node[0][el] = fric;           // p = 3 keeps no point values here
  // The edges this element evaluates, in three classes listed one after the
  // other so that a wavefront mostly runs one code path: (0) interior edges
  // inside the tile, owned by the lower id; (1) edges to other tiles;
  // (2) boundary edges.  Entry: l | k << LB | kn << (LB + 2) | ln << (LB + 4).
  uint32_t ent[3];
  int cls[3];
  // counts per class: classes 0 and 1 in 16-bit fields, class 2 apart (a
  // class holds at most 3 T entries)
  int packed = 0, packed2 = 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int nb = nbv[k];
    const int kn = (nkp >> (2 * k)) & 3;
    const bool inside = nb >= t0 && nb < tend;
    cls[k] = !valid ? 3 : nb < 0 ? 2 : !inside ? 1 : (e < nb ? 0 : 3);
    // in the tile: the neighbour's local index; PRE, in ring 1: its slot
    const uint32_t at = inside ? uint32_t(nb - t0) : PRE ? (eslot >> (10 * k)) & HALO_SLOT_MASK : 0u;
    ent[k] = uint32_t(el) | uint32_t(k) << LB | uint32_t(kn) << (LB + 2) | at << (LB + 4);
    packed += cls[k] == 0 ? 1 : cls[k] == 1 ? 1 << 16 : 0;
    packed2 += cls[k] == 2 ? 1 : 0;
  }
  // block-wide exclusive scan of the counts
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int incl = wave_incl_scan(packed), incl2 = wave_incl_scan(packed2);
  if (lane == 63) {
    s_wsum[0][wv] = incl;
    s_wsum[1][wv] = incl2;
  }
  // area integrals and storm terms: in phase A, or (kAreaLate) after the
  // edge loop, so that their accumulators are not live across it
  Real acc[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) acc[v][m] = Real(0);
  auto volume = [&](const Real (&w)[3][NP]) {
    if constexpr (!MF)
      area_terms<Real, P>(w, d.hb, d.cx0, d.cx1, d.cy0, d.cy1, d.detJ, d.idet, fric, M.friction, g, H0, acc);
    if (met_on) {
      if constexpr (!kMetEarly) {
        int tm[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) tm[i] = ldc(gp(M.tri), i * E, ec);
        met_nodes<Real>(M, tm, mtx, mty, mps);
      }
      met_terms<Real, P>(mtx, mty, mps, w, d.hb, d.cx0, d.cx1, d.cy0, d.cy1, d.detJ, d.idet, g, acc);
    }
  };
  // FP64 p = 3 on 64-element tiles computes them after the edge loop and
  // reads its modes again there (they stay in the cache) rather than keeping
  // 60 registers of modes and 60 of accumulators live across the loop: with
  // the two-wavefront register budget this spills less.  (The fused kernel,
  // p <= 2, changes the modes in phase 0 and never reloads them.)
  constexpr bool kAreaLate = P == 3 && sizeof(Real) == 8 && T == 64;
  constexpr bool kReloadW = kAreaLate && !PRE;
  if constexpr (!kAreaLate) volume(d.w);
  __syncthreads();
  int base = 0, base2 = 0, tot = 0, tot2 = 0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    base += (i < wv) ? s_wsum[0][i] : 0;
    base2 += (i < wv) ? s_wsum[1][i] : 0;
    tot += s_wsum[0][i];
    tot2 += s_wsum[1][i];
  }
  const int n0 = tot & 0xFFFF, n1 = tot >> 16, n2 = tot2;
  const int n_list = n0 + n1 + n2;
  {
    const int ex_ = base + incl - packed, ex2 = base2 + incl2 - packed2;
    int pos[3] = {ex_ & 0xFFFF, n0 + (ex_ >> 16), n0 + n1 + ex2};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int c = cls[k];
      if (c < 3) {
        const int at = c == 0 ? pos[0]++ : c == 1 ? pos[1]++ : pos[2]++;
        s_list[at] = ListT(ent[k]);
      }
    }
  }
  __syncthreads();

  // nodal rain rates, consumed after phase B
  double rn3[3] = {0.0, 0.0, 0.0};
  if (rain_avg) {
#pragma unroll
    for (int i = 0; i < 3; ++i) rn3[i] = ldx(gp(M.rn), tn[i]);
  }

  // ---- phase B: edge fluxes, scaled by (l/2) w_g, into s_flux
  if constexpr (kTr) {
    // traces come from s_flux (own side, and the neighbour's when it is in
    // the tile) or from the neighbour's modes; only the thread of an edge
    // touches that edge's slots, so it reads them all before writing fluxes
    for (int it = threadIdx.x; it < n_list; it += T) {
      const uint32_t ent = s_list[it];
      const int l = ent & (T - 1), k = (ent >> LB) & 3, kn = (ent >> (LB + 2)) & 3;
      const int k1 = k == 2 ? 0 : k + 1;
      const int eg = t0 + l;
      const bool in_tile = it < n0;
      const int nb = in_tile ? t0 + int(ent >> (LB + 4)) : ldc(nbr, k * E, eg);
      const Real exk = kEvLds ? s_ev[2 * k][l] : ldc(gp(M.ev), (2 * k) * E, eg);
      const Real eyk = kEvLds ? s_ev[2 * k + 1][l] : ldc(gp(M.ev), (2 * k + 1) * E, eg);
      Real ell, il;
      edge_length<Real>(exk, eyk, ell, il);
      const Real nx = eyk * il, ny = -exk * il;
      const Real half = Real(0.5) * ell;
      Real tO[3][NG];
#pragma unroll
      for (int gg = 0; gg < NG; ++gg)
#pragma unroll
        for (int v = 0; v < 3; ++v) tO[v][gg] = s_flux[(k * NG + gg) * 3 + v][l];
      const Real hA = s_hb[k][l], hB = s_hb[k1][l];
      if (nb >= 0) {
        Real tN[3][NG];
        bool nflag;
        if (in_tile) {
          const int ln = nb - t0;
#pragma unroll
          for (int gg = 0; gg < NG; ++gg)
#pragma unroll
            for (int v = 0; v < 3; ++v) tN[v][gg] = s_flux[(kn * NG + gg) * 3 + v][ln];
          nflag = s_flag[ln];
        } else if constexpr (P <= 2) {
          Real wn[3][NP];
#pragma unroll
          for (int v = 0; v < 3; ++v)
#pragma unroll
            for (int m = 0; m < NP; ++m) wn[v][m] = ldc(Win, (v * NP + m) * E, nb);
          Real nvv[3][3], nmv[3][3];
          edge_nodes<Real, P>(wn, nvv, nmv);
          const int kn1 = kn == 2 ? 0 : kn + 1;
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            const Real Na = kn == 0 ? nvv[v][0] : kn == 1 ? nvv[v][1] : nvv[v][2];
            const Real Nb = kn1 == 0 ? nvv[v][0] : kn1 == 1 ? nvv[v][1] : nvv[v][2];
            const Real Nc = kn == 0 ? nmv[v][0] : kn == 1 ? nmv[v][1] : nmv[v][2];
#pragma unroll
            for (int gg = 0; gg < NG; ++gg) tN[v][gg] = trace<Real, P>(Na, Nc, Nb, gg);
          }
          nflag = ldx(Fin, nb) & 1;
        } else {
#pragma unroll
          for (int v = 0; v < 3; ++v) {
            Real wv[NP];
#pragma unroll
            for (int m = 0; m < NP; ++m) wv[m] = ldc(Win, (v * NP + m) * E, nb);
            static_for<NG>([&](auto gc) {
              constexpr int gg = decltype(gc)::value;
              tN[v][gg] = trace_modal<Real, P, gg>(wv, kn);
            });
          }
          nflag = ldx(Fin, nb) & 1;
        }
        const bool myflag = s_flag[l];
        const bool meL = eg < nb;
        const Real hLa = meL ? hA : hB, hLb = meL ? hB : hA;
        const Real lnx = meL ? nx : -nx, lny = meL ? ny : -ny;
        const bool dryL = meL ? myflag : nflag, dryR = meL ? nflag : myflag;
        static_for<NG>([&](auto gc) {
          constexpr int gL = decltype(gc)::value;
          constexpr int gR = NG - 1 - gL;
          const W3<Real> a{meL ? tO[0][gL] : tN[0][gL], meL ? tO[1][gL] : tN[1][gL], meL ? tO[2][gL] : tN[2][gL]};
          const W3<Real> b{meL ? tN[0][gR] : tO[0][gR], meL ? tN[1][gR] : tO[1][gR], meL ? tN[2][gR] : tO[2][gR]};
          const Real hg = Real(lag_(1, 0, gl_t(P, gL))) * hLa + Real(lag_(1, 1, gl_t(P, gL))) * hLb;
          Real FL[3], FR[3];
          interior_point<FLUX>(a, b, hg, lnx, lny, g, H0, feps, dryL, dryR, meL, !meL || in_tile, FL, FR);
          const Real wg = half * Real(gl_w(P, gL));
          const int gm = meL ? gL : gR;
#pragma unroll
          for (int v = 0; v < 3; ++v) s_flux[(k * NG + gm) * 3 + v][l] = wg * (meL ? FL[v] : FR[v]);
          if (in_tile) {
#pragma unroll
            for (int v = 0; v < 3; ++v) s_flux[(kn * NG + gR) * 3 + v][nb - t0] = wg * FR[v];
          }
          // one Gauss point at a time (interleaving them raises the register peak)
          if constexpr (kAreaLate) __builtin_amdgcn_sched_barrier(0);
        });
      } else {
        const int code = -1 - nb;
        const int type = code & 3, slot = code >> 2;
        const Real tide = Real(sc->tide[A.stage][slot]), qr = Real(sc->river[A.stage][slot]);
        static_for<NG>([&](auto gc) {
          constexpr int gi = decltype(gc)::value;
          const W3<Real> a{tO[0][gi], tO[1][gi], tO[2][gi]};
          const Real hg = Real(lag_(1, 0, gl_t(P, gi))) * hA + Real(lag_(1, 1, gl_t(P, gi))) * hB;
          Real F[3];
          boundary_point<FLUX>(a, hg, nx, ny, g, H0, type, tide, qr, F);
          const Real wg = half * Real(gl_w(P, gi));
#pragma unroll
          for (int v = 0; v < 3; ++v) s_flux[(k * NG + gi) * 3 + v][l] = wg * F[v];
        });
      }
    }
  } else
  for (int it = threadIdx.x; it < n_list; it += T) {
    const uint32_t ent = s_list[it];
    const int l = ent & (T - 1), k = (ent >> LB) & 3, kn = (ent >> (LB + 2)) & 3;
    const int k1 = k == 2 ? 0 : k + 1;
    const int eg = t0 + l;
    const bool in_tile = it < n0;
    // class 0: the neighbour's id is in the entry; otherwise re-read (cached)
    const int nb = in_tile ? t0 + int(ent >> (LB + 4)) : ldc(nbr, k * E, eg);
    const Real exk = kEvLds ? s_ev[2 * k][l] : ldc(gp(M.ev), (2 * k) * E, eg);
    const Real eyk = kEvLds ? s_ev[2 * k + 1][l] : ldc(gp(M.ev), (2 * k + 1) * E, eg);
    Real ell, il;
    edge_length<Real>(exk, eyk, ell, il);
    const Real nx = eyk * il, ny = -exk * il;
    const Real half = Real(0.5) * ell;
    Real Oa[3], Oc[3], Ob[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      Oa[v] = s_node[v * NN + k][l];
      Ob[v] = s_node[v * NN + k1][l];
      Oc[v] = (P == 2) ? s_node[v * NN + 3 + k][l] : Real(0);
    }
    const Real hA = s_hb[k][l], hB = s_hb[k1][l];
    if (nb >= 0) {
      const int kn1 = kn == 2 ? 0 : kn + 1;
      Real Na[3], Nc[3], Nb[3];
      bool nflag;
      if (in_tile) {
        const int ln = nb - t0;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Na[v] = s_node[v * NN + kn][ln];
          Nb[v] = s_node[v * NN + kn1][ln];
          Nc[v] = (P == 2) ? s_node[v * NN + 3 + kn][ln] : Real(0);
        }
        nflag = s_flag[ln];
      } else if constexpr (PRE) {
        // ring 1: post-processed in phase 0, point values in LDS
        const int sl = int(ent >> (LB + 4));
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Na[v] = s_node[v * NN + kn][sl];
          Nb[v] = s_node[v * NN + kn1][sl];
          Nc[v] = (P == 2) ? s_node[v * NN + 3 + kn][sl] : Real(0);
        }
        nflag = s_flag[sl];
      } else {
        Real wn[3][NP];
#pragma unroll
        for (int v = 0; v < 3; ++v)
#pragma unroll
          for (int m = 0; m < NP; ++m) wn[v][m] = ldc(Win, (v * NP + m) * E, nb);
        Real nvv[3][3], nmv[3][3];
        edge_nodes<Real, P>(wn, nvv, nmv);
#pragma unroll
        for (int v = 0; v < 3; ++v) {
          Na[v] = kn == 0 ? nvv[v][0] : kn == 1 ? nvv[v][1] : nvv[v][2];
          Nb[v] = kn1 == 0 ? nvv[v][0] : kn1 == 1 ? nvv[v][1] : nvv[v][2];
          Nc[v] = kn == 0 ? nmv[v][0] : kn == 1 ? nmv[v][1] : nmv[v][2];
        }
        nflag = ldx(Fin, nb) & 1;
      }
      const bool myflag = s_flag[l];
      const bool meL = eg < nb;
      Real La[3], Lc[3], Lb[3], Ra[3], Rc[3], Rb[3];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        La[v] = meL ? Oa[v] : Na[v]; Lc[v] = meL ? Oc[v] : Nc[v]; Lb[v] = meL ? Ob[v] : Nb[v];
        Ra[v] = meL ? Na[v] : Oa[v]; Rc[v] = meL ? Nc[v] : Oc[v]; Rb[v] = meL ? Nb[v] : Ob[v];
      }
      const Real hLa = meL ? hA : hB, hLb = meL ? hB : hA;
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
        Real FL[3], FR[3];
        // the neighbour's side is needed when it is in the tile (then this element is L)
        interior_point<FLUX>(a, b, hg, lnx, lny, g, H0, feps, dryL, dryR, meL, !meL || in_tile, FL, FR);
        const Real wg = half * Real(gl_w(P, gL));
        const int gm = meL ? gL : gR;
#pragma unroll
        for (int v = 0; v < 3; ++v) s_flux[(k * NG + gm) * 3 + v][l] = wg * (meL ? FL[v] : FR[v]);
        if (in_tile) {
#pragma unroll
          for (int v = 0; v < 3; ++v) s_flux[(kn * NG + gR) * 3 + v][nb - t0] = wg * FR[v];
        }
      }
    } else {
      const int code = -1 - nb;
      const int type = code & 3, slot = code >> 2;
      const Real tide = Real(sc->tide[A.stage][slot]), qr = Real(sc->river[A.stage][slot]);
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) {
        W3<Real> a{trace<Real, P>(Oa[0], Oc[0], Ob[0], gi), trace<Real, P>(Oa[1], Oc[1], Ob[1], gi),
                   trace<Real, P>(Oa[2], Oc[2], Ob[2], gi)};
        const Real hg = Real(lag_(1, 0, gl_t(P, gi))) * hA + Real(lag_(1, 1, gl_t(P, gi))) * hB;
        Real F[3];
        boundary_point<FLUX>(a, hg, nx, ny, g, H0, type, tide, qr, F);
        const Real wg = half * Real(gl_w(P, gi));
#pragma unroll
        for (int v = 0; v < 3; ++v) s_flux[(k * NG + gi) * 3 + v][l] = wg * F[v];
      }
    }
  }
  __syncthreads();
  // volume through this element's own boundary edges, from the mass
  // components of their fluxes (so that a wavefront's partials depend only
  // on its own elements, not on which thread evaluated an edge)
  double bout = 0.0, bin = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (valid && nbv[k] < 0) {
      double fm = 0.0;
#pragma unroll
      for (int gi = 0; gi < NG; ++gi) fm += double(s_flux[(k * NG + gi) * 3][el]);
      if (fm > 0.0) bout += fm; else bin -= fm;
    }

  // ---- phase C: edge contributions, inverse mass, stage combination, post
  Real wr[3][NP];
  if constexpr (kReloadW) {
#pragma unroll
    for (int v = 0; v < 3; ++v)
#pragma unroll
      for (int m = 0; m < NP; ++m) wr[v][m] = ldc(Win, (v * NP + m) * E, ec);
    volume(wr);
  } else if constexpr (kAreaLate) {
    volume(d.w);
  }
  Real (&wf)[3][NP] = kReloadW ? wr : d.w;
  Real w0v[3][NP];
  if constexpr (!MF) load_blend<Real, P>(M, A, E, ec, w0v);
  if constexpr (P >= 3) {
    // expanded at compile time so that every basis value is a constant
    static_for<3>([&](auto kc) {
      constexpr int k = decltype(kc)::value;
      static_for<NG>([&](auto gc) {
        constexpr int gi = decltype(gc)::value;
        const Real f0 = s_flux[(k * NG + gi) * 3 + 0][el], f1 = s_flux[(k * NG + gi) * 3 + 1][el],
                   f2 = s_flux[(k * NG + gi) * 3 + 2][el];
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const Real ph = Real(B<P>::EG(k, gi, m));
          acc[0][m] -= ph * f0;
          acc[1][m] -= ph * f1;
          acc[2][m] -= ph * f2;
        }
      });
    });
    if constexpr (MF) {
      // the flux slots are read: they take the tile's modes for the
      // matrix-core area integrals, and hold them for the combine (read
      // back afterwards instead of keeping 30 registers live across it);
      // w^n is read after it for the same reason
      __syncthreads();
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) s_flux[v * NP + m][el] = wf[v][m];
      __syncthreads();
      area_terms_mfma_p3(s_flux, s_hb, s_ev, s_node[0], M.friction, Real(g), Real(H0), acc);
      asm volatile("" ::: "memory");
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) wf[v][m] = s_flux[v * NP + m][el];
      load_blend<Real, P>(M, A, E, ec, w0v);
    }
  } else {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int gi = 0; gi < NG; ++gi) {
      const Real f0 = s_flux[(k * NG + gi) * 3 + 0][el], f1 = s_flux[(k * NG + gi) * 3 + 1][el],
                 f2 = s_flux[(k * NG + gi) * 3 + 2][el];
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const Real ph = Real(B<P>::EG(k, gi, m));
        acc[0][m] -= ph * f0;
        acc[1][m] -= ph * f1;
        acc[2][m] -= ph * f2;
      }
    }
  }
  double rain_part = 0.0;
  if (rain_avg) {
    Rv = Real((rn3[0] + rn3[1] + rn3[2]) / 3.0);
    if (valid) stx(gp(M.R), e, Rv);
    const double area = 0.5 * (double(d.ex[2]) * double(d.ey[0]) - double(d.ex[0]) * double(d.ey[2]));
    rain_part = valid ? area * double(Rv) : 0.0;
  }
  finish_stage<Real, P, LIM, T>(M, A, tl.tile, e, ec, valid, E, wf, acc, d.hb, d.ex, d.ey, d.detJ, d.idet, dt, bout,
                             bin, Rv, rain_part, w0v);
}

// ------------------------------------------------------------ post kernel
// Slope limiter (Cockburn-Shu, componentwise on zeta, qx, qy; nu = 1.5; only
// where the element and its three neighbours are fully wet), then the
// positive-depth operator, flags, CFL speed and tile partials.
// init: 0 = after a stage, in place on the stage's output buffer: only the
// elements that either operator modifies are written back; 1 = initial
// state in Wt (limiter if the member has it, positive depth) into W[0];
// 2 = flags and partials of W[0] only.
// In place is safe because a neighbour's means are used only when every
// element of the stencil is fully wet, and the pass never changes the means
// of a fully-wet element (the limiter moves slopes only, positive depth
// keeps means): other workgroups may rewrite those words, with the same
// bits.
template <typename Real, int P>
__global__ __launch_bounds__(TILE) void post_kernel(const Member<Real>* __restrict__ mem,
                                                    const Tile* __restrict__ tiles, int n_tiles, StageArgs A,
                                                    int init, int use_lim) {
  constexpr int NP = Tab<P>::NP;
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = A.single ? Tile{0, ti} : tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const DG_G Scalars* __restrict__ sc = gp((const Scalars*)M.sc);
  if (!sc->active && init == 0) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  // not restrict: with init = 0 the same buffer is written below
  const DG_G Real* Wsrc = gp(init == 2 ? M.W[0] : init == 1 ? M.Wt : M.W[A.out_buf]);
  bool changed = init == 1;
  Real w[3][NP];
#pragma unroll
  for (int v = 0; v < 3; ++v)
#pragma unroll
    for (int m = 0; m < NP; ++m) w[v][m] = ldc(Wsrc, (v * NP + m) * E, ec);
  Real hb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) hb[k] = ldc(gp(M.hbv), k * E, ec);

  if (init != 2 && use_lim) {
    const uint8_t lc = ldx(gp(M.limc), ec);
    // the neighbours' wet bytes and means are fetched together, before the
    // test that decides whether they are used (boundary ids read the element
    // itself), so the gather costs one memory round trip
    int nb[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int n = ldc(gp(M.nbr), k * E, ec);
      nb[k] = n < 0 ? ec : n;
    }
    const DG_G uint8_t* __restrict__ fw = gp(M.fullwet[A.stage & 1]);
    bool ok = ((lc & 1) != 0) & (ldx(fw, ec) != 0);
    Real nmean[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ok = ok & (ldx(fw, nb[k]) != 0);
#pragma unroll
      for (int v = 0; v < 3; ++v) nmean[v][k] = ldc(Wsrc, (v * NP) * E, nb[k]);
    }
    if (ok) {
      Real al[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) al[j] = ldc(gp(M.lima), j * E, ec);
      changed = limit_element<Real, P>(w, lc, al, nmean) || changed;
    }
  }
  bool dry, filled = true;
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
    const double Hd = dry_depth(M.H0);
    dry = (hv[0] <= Hd) & (hv[1] <= Hd) & (hv[2] <= Hd);
  } else {
    bool pd = false;
    dry = positive_depth<Real, P>(w, hb, M.H0, hv, qxv, qyv, (init != 0 || A.last != 0) && sizeof(Real) == 8,
                                  filled, &pd);
    changed = changed || pd;
  }
  const int ob = init ? 0 : A.out_buf;
  const int fo = init ? 0 : A.fout;
  if (valid) {
    if (init != 2 && changed) {
      DG_G Real* Wout = gp(M.W[ob]);
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int m = 0; m < NP; ++m) stc(Wout, (v * NP + m) * E, e, w[v][m]);
    }
    stx(gp(M.F[fo]), e, uint8_t(dry ? 1 : 0));
  }
  if (init || A.last) {
    Real ex[3], ey[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ex[k] = ldc(gp(M.ev), (2 * k) * E, ec);
      ey[k] = ldc(gp(M.ev), (2 * k + 1) * E, ec);
    }
    const double area = 0.5 * (double(ex[2]) * double(ey[0]) - double(ex[0]) * double(ey[2]));
    const double lam = post_speed<Real, P>(filled, hv, qxv, qyv, w, hb, M.H0, M.g);
    const double md = double(w[0][0]) + (double(hb[0]) + double(hb[1]) + double(hb[2])) / 3.0;
    const double vol = valid ? area * md : 0.0;
    const double mr = (valid && lam > 0.0) ? double(ldx(gp(M.din), ec)) * rcp(lam) : __builtin_inf();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const double s0 = wave_sum(vol), s1 = double(__popcll(__ballot(valid && dry))), mn = wave_min(mr);
    const double s2 = double(__popcll(__ballot(valid && md < 0.0)));
    const double fb = first_lane_id(__ballot(valid && !(__builtin_isfinite(md) && __builtin_isfinite(lam))),
                                    tl.tile * TILE + wv * 64);
    if (lane == 0) {
      DG_G double* __restrict__ pt = gp(A.part ? A.part : M.part);
      const size_t row = part_row(M.n_tiles), slot = size_t(tl.tile) * PSLOT + wv;
      pt[P_VOL * row + slot] = s0;
      pt[P_NDRY * row + slot] = s1;
      pt[P_MINR * row + slot] = mn;
      pt[P_NNEG * row + slot] = s2;
      pt[P_BAD * row + slot] = fb;
    }
  }
}

// fully-wet bytes of the state in Wt (initial limiting)
template <typename Real, int P>
__global__ __launch_bounds__(TILE) void classify_kernel(const Member<Real>* __restrict__ mem,
                                                        const Tile* __restrict__ tiles, int n_tiles) {
  constexpr int NP = Tab<P>::NP;
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  if (e >= E) return;
  Real w[3][NP], hb[3];
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    w[0][m] = gp(M.Wt)[(0 * NP + m) * E + e];
    w[1][m] = w[2][m] = Real(0);
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) hb[i] = gp(M.hbv)[i * E + e];
  gp(M.fullwet[0])[e] = fully_wet<Real, P>(w, hb, M.H0) ? 1 : 0;
}

// -------------------------------------------------------------- rain
DG_DEV double lattice(const DG_G float* __restrict__ v, int nx, int ny, double x0, double y0, double dx, double dy,
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

// Kinematic wind stress and pressure head of the storm vortex at a node
// (FP32 members evaluate it in FP32 from offsets formed in FP64).
template <typename Real>
DG_DEV void vortex_node(const DG_G Scalars* sc, double x, double y, double g, Real& tx, Real& ty, Real& psi) {
  const double xc = sc->wind[0], yc = sc->wind[1], dp = sc->wind[2], rm = sc->wind[3], Bh = sc->wind[4];
  const double wf = sc->wind[5], wbx = sc->wind[6], wby = sc->wind[7];
  if constexpr (sizeof(Real) == 4) {
    const float dx = float(x - xc), dy = float(y - yc), rmf = float(rm), Bf = float(Bh), dpf = float(dp);
    const float r = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
    const float rs = dmax(r, 1e-6f * rmf);
    const float s = __builtin_amdgcn_exp2f(Bf * __builtin_amdgcn_logf(rmf / rs));
    const float e = __builtin_amdgcn_exp2f(-1.4426950408889634f * s);
    const float dpa = -dpf * (1.0f - e);
    const float V = __builtin_amdgcn_sqrtf(Bf * dpf * s * e / float(RHO_AIR));
    const float Wx = float(wf) * V * (-dy) / rs + float(wbx), Wy = float(wf) * V * dx / rs + float(wby);
    const float sp = __builtin_amdgcn_sqrtf(Wx * Wx + Wy * Wy);
    const float k = float(RHO_AIR / RHO_WATER) * dmin((0.75f + 0.067f * sp) * 1e-3f, float(CD_MAX)) * sp;
    tx = k * Wx;
    ty = k * Wy;
    psi = dpa / float(RHO_WATER * g);
  } else {
    const double dx = x - xc, dy = y - yc;
    const double rs = fmax(hypot(dx, dy), 1e-6 * rm);
    const double s = pow(rm / rs, Bh);
    const double e = exp(-s);
    const double dpa = -dp * (1.0 - e);
    const double V = sqrt(Bh * dp * s * e / RHO_AIR);
    const double Wx = wf * V * (-dy) / rs + wbx, Wy = wf * V * dx / rs + wby;
    const double sp = hypot(Wx, Wy);
    const double k = (RHO_AIR / RHO_WATER) * fmin((0.75 + 0.067 * sp) * 1e-3, CD_MAX) * sp;
    tx = k * Wx;
    ty = k * Wy;
    psi = dpa / (RHO_WATER * g);
  }
}

// Nodal forcing at t^n, one thread per node (block t covers nodes
// [t TILE, (t+1) TILE)): the rain rate (Sec. 2.5 parametric storm profile or
// Sec. 3.3 rain lattice) and the storm's wind stress and pressure head.
template <typename Real>
__global__ __launch_bounds__(TILE) void node_forcing_kernel(const Member<Real>* __restrict__ mem,
                                                            const Tile* __restrict__ tiles, int n_tiles, int single) {
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = single ? Tile{0, ti} : tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const DG_G Scalars* __restrict__ sc = gp((const Scalars*)M.sc);
  const int kind = M.fo.rain_kind;
  const bool wind = M.fo.met_kind != MET_NONE;
  if (!sc->active || (kind == RAIN_CONST && !wind)) return;
  const int n = tl.tile * TILE + int(threadIdx.x);
  if (n >= M.n_nodes) return;
  const double x = gp(M.nxy)[n], y = gp(M.nxy)[M.n_nodes + n];
  if (wind) {
    Real tx, ty, psi;
    vortex_node<Real>(sc, x, y, M.g, tx, ty, psi);
    DG_G Real* __restrict__ met = gp(M.met);
    met[n] = tx;
    met[M.n_nodes + n] = ty;
    met[2 * M.n_nodes + n] = psi;
  }
  if (kind == RAIN_CONST) return;
  double r;
  if (kind == RAIN_PARAM) {
    const double xc = sc->storm[0], yc = sc->storm[1], pk = sc->storm[2], T0 = sc->storm[3];
    const double rm = sc->storm[4], re = sc->storm[5];
    if constexpr (sizeof(Real) == 4) {
      // FP32 members evaluate the profile in FP32 (offsets from the centre
      // are formed in FP64 first)
      const float dx = float(x - xc), dy = float(y - yc);
      const float d = __builtin_amdgcn_sqrtf(dx * dx + dy * dy);
      const float rmf = float(rm), pkf = float(pk), T0f = float(T0);
      r = d < rmf ? double(T0f + (pkf - T0f) * d / rmf)
                  : double(pkf * __builtin_amdgcn_exp2f(-(d - rmf) * (1.4426950408889634f / float(re))));
    } else {
      const double d = hypot(x - xc, y - yc);
      r = d < rm ? T0 + (pk - T0) * d / rm : pk * exp(-(d - rm) / re);
    }
  } else {
    const Forcing& f = M.fo;
    const size_t rs = size_t(f.gnx) * f.gny;
    const double th = sc->gth;
    const double a = lattice(gp(f.gvals) + rs * sc->gk0, f.gnx, f.gny, f.gx0, f.gy0, f.gdx, f.gdy, x, y);
    const double b = lattice(gp(f.gvals) + rs * sc->gk1, f.gnx, f.gny, f.gx0, f.gy0, f.gdx, f.gdy, x, y);
    r = (1.0 - th) * a + th * b;
  }
  gp(M.rn)[n] = r;
}

// Element rain (Eq. rain): the mean of the three nodal rates, and the tile's
// rain volume rate.  always = 1 runs even for constant rain (set-up).
template <typename Real>
__global__ __launch_bounds__(TILE) void rain_kernel(const Member<Real>* __restrict__ mem,
                                                    const Tile* __restrict__ tiles, int n_tiles, int always) {
  const int ti = xcd_tile();
  if (ti >= n_tiles) return;
  const Tile tl = tiles[ti];
  const Member<Real>& M = mem[tl.member];
  const DG_G Scalars* __restrict__ sc = gp((const Scalars*)M.sc);
  if (!always && (!sc->active || M.fo.rain_kind == RAIN_CONST)) return;
  const int E = M.E;
  const int e = tl.tile * TILE + int(threadIdx.x);
  const bool valid = e < E;
  const int ec = valid ? e : E - 1;
  const DG_G double* __restrict__ rn = gp(M.rn);
  const double r0 = ldx(rn, ldx(gp(M.tri), ec)), r1 = ldx(rn, ldc(gp(M.tri), E, ec)),
               r2 = ldx(rn, ldc(gp(M.tri), 2 * E, ec));
  const Real Re = Real((r0 + r1 + r2) / 3.0);
  if (valid) stx(gp(M.R), e, Re);
  const double area = 0.5 * (double(gp(M.ev)[4 * E + ec]) * double(gp(M.ev)[1 * E + ec]) -
                             double(gp(M.ev)[0 * E + ec]) * double(gp(M.ev)[5 * E + ec]));
  double v = valid ? area * double(Re) : 0.0;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) gp(M.part)[P_RAIN * part_row(M.n_tiles) + size_t(tl.tile) * PSLOT + wv] = v;
}

// ------------------------------------------------------------ reduce


// Per-member scalar update at the end of a step (or after set-up): fixed
// order sums of the tile partials, budgets, t, the next dt (FP64), the
// latched error, and the forcing values of the coming step (tide and river
// at every stage time, storm parameters and rain-lattice records at t^n).
// Grid (members, chunks): workgroup (m, c) sums tiles [c RED_CHUNK, (c+1)
// RED_CHUNK) of member m, one tile per thread, and stores a chunk record; the
// workgroup that finishes last (counted with a device-scope atomic) adds the
// records in chunk order, so the result does not depend on which one that
// is, and resets the counter for the next launch.
// The kernel is a chain of dependent memory round trips, so each phase
// issues all of its loads before it uses any of them.
template <typename Real>
__global__ __launch_bounds__(RED_CHUNK) void reduce_kernel(const Member<Real>* __restrict__ mem,
                                                           const int* __restrict__ ids, int init, RKInfo rk,
                                                           double* part_over) {
  // sums: volume, rain, dry count, out/in per stage, negative-depth count;
  // minima: d/lambda and the first non-finite element
  constexpr int NV = 4 + 2 * MAX_STAGES;
  constexpr int INEG = 3 + 2 * MAX_STAGES;
  constexpr int NW = RED_CHUNK / 64;
  constexpr int NT = RED_CHUNK;                // forcing-table rows staged in LDS, one per thread
  static_assert(NV + 2 <= NRED, "chunk record too small");
  __shared__ double lds[NW * (NV + 2)];
  __shared__ double s_storm[7 * NT];
  __shared__ double s_gt[NT];
  __shared__ double s_tide[3 * NT];
  __shared__ double s_riv[2 * NT];
  constexpr int NTW = 64;                      // wind records staged in LDS
  __shared__ double s_wind[9 * NTW];
  __shared__ double s_t, s_dt;
  __shared__ int s_last;
  // ids == nullptr: a single context, member 0 (no id to read first)
  const Member<Real>& M = mem[ids ? ids[blockIdx.x] : 0];
  DG_G Scalars* __restrict__ sc = gp(M.sc);
  const int nt = M.n_tiles;
  const int nch = red_chunks(nt);
  const int chunk = blockIdx.y;
  if (chunk >= nch) return;
  // the member's partials and records, or the same layout at part_over
  double* const part = part_over ? part_over : M.part;
  double* const redp = part_over ? part_over + size_t(NPART) * part_row(nt) : M.red;
  unsigned* const red_count = part_over ? reinterpret_cast<unsigned*>(redp + size_t(NRED) * nch) : M.red_count;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int ns = init ? 0 : rk.n;
  // ---- this chunk's tiles, loaded together with the member's active flag
  double v[NV];
  double mn, fb;
  {
    // the tile's four wavefront slots (one 32-byte load per row), combined
    // as (s0 + s1) + (s2 + s3); a slot that starts at or beyond E holds no
    // element and reads as empty
    const DG_G double* __restrict__ pt = gp(part);
    const size_t row = part_row(nt);
    const int t = chunk * RED_CHUNK + tid;
    const bool ok = t < nt;
    const size_t s0 = size_t(ok ? t : 0) * PSLOT;
    static_assert(PSLOT == 4, "four slots per tile");
    const int nslot = ok ? (M.E - t * TILE + 63) / 64 : 0;
    typedef double d4 __attribute__((ext_vector_type(4)));
    auto ld4 = [&](int r) -> d4 { return *reinterpret_cast<const DG_G d4*>(pt + r * row + s0); };
    auto sum4 = [&](const d4 q) -> double {
      return ((nslot > 0 ? q.x : 0.0) + (nslot > 1 ? q.y : 0.0)) + ((nslot > 2 ? q.z : 0.0) + (nslot > 3 ? q.w : 0.0));
    };
    auto min4 = [&](const d4 q) -> double {
      constexpr double inf = __builtin_inf();
      return fmin(fmin(nslot > 0 ? q.x : inf, nslot > 1 ? q.y : inf), fmin(nslot > 2 ? q.z : inf, nslot > 3 ? q.w : inf));
    };
    const d4 qv = ld4(P_VOL), qr = ld4(P_RAIN), qd = ld4(P_NDRY), qm = ld4(P_MINR), qn = ld4(P_NNEG),
             qb = ld4(P_BAD);
    d4 qo[MAX_STAGES], qi[MAX_STAGES];
#pragma unroll
    for (int s = 0; s < MAX_STAGES; ++s)
      if (s < ns) {
        qo[s] = ld4(P_OUT0 + s);
        qi[s] = ld4(P_IN0 + s);
      }
    v[0] = sum4(qv);
    v[1] = sum4(qr);
    v[2] = sum4(qd);
    mn = min4(qm);
#pragma unroll
    for (int s = 0; s < MAX_STAGES; ++s) {
      v[3 + s] = s < ns ? sum4(qo[s]) : 0.0;
      v[3 + MAX_STAGES + s] = s < ns ? sum4(qi[s]) : 0.0;
    }
    v[INEG] = sum4(qn);
    fb = min4(qb);
  }
  const bool act = init || sc->active;
  // fixed-order block sums: within each wavefront, then wavefronts 0..NW-1
  auto block_reduce = [&]() {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double x = wave_sum(v[i]);
      if (lane == 0) lds[wv * (NV + 2) + i] = x;
    }
    const double m = wave_min(mn), b = wave_min(fb);
    if (lane == 0) {
      lds[wv * (NV + 2) + NV] = m;
      lds[wv * (NV + 2) + NV + 1] = b;
    }
    __syncthreads();
    if (tid == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        double x = lds[i];
#pragma unroll
        for (int w = 1; w < NW; ++w) x += lds[w * (NV + 2) + i];
        v[i] = x;
      }
      double m2 = lds[NV], b2 = lds[NV + 1];
#pragma unroll
      for (int w = 1; w < NW; ++w) {
        m2 = fmin(m2, lds[w * (NV + 2) + NV]);
        b2 = fmin(b2, lds[w * (NV + 2) + NV + 1]);
      }
      mn = m2;
      fb = b2;
    }
    __syncthreads();
  };
  block_reduce();
  // an inactive member (finished or latched) keeps its scalars as they are
  if (!act) return;
  DG_G double* __restrict__ red = gp(redp);
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[chunk * NRED + i] = v[i];
    red[chunk * NRED + NV] = mn;
    red[chunk * NRED + NV + 1] = fb;
    __threadfence();
    const unsigned done = atomicAdd(red_count, 1u);
    s_last = done == unsigned(nch - 1);
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  // ---- last workgroup: chunk records, step scalars and forcing tables in
  // one round of loads
  const Forcing& f = M.fo;
  const int nst = f.rain_kind == RAIN_PARAM ? (f.n_storm < NT ? f.n_storm : NT) : 0;
  const int ngt = f.rain_kind == RAIN_GRID ? (f.gnrec < NT ? f.gnrec : NT) : 0;
  const bool tide_lds = f.n_tide <= NT, riv_lds = f.n_riv <= NT;
  const int ntc = tide_lds ? f.n_tide : 0, nrq = riv_lds ? f.n_riv : 0;
  const int nwd = f.met_kind == MET_VORTEX ? (f.n_wind < NTW ? f.n_wind : NTW) : 0;
  double r_storm[7], r_tide[3], r_riv[2], r_gt, r_wind[3];
#pragma unroll
  for (int k = 0; k < 7; ++k) r_storm[k] = k * NT + tid < 7 * nst ? gp(f.storm)[k * NT + tid] : 0.0;
  r_gt = tid < ngt ? gp(f.gt)[tid] : 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) r_tide[k] = k * NT + tid < 3 * ntc ? gp(f.tide_c)[k * NT + tid] : 0.0;
#pragma unroll
  for (int k = 0; k < 2; ++k) r_riv[k] = k * NT + tid < 2 * nrq ? gp(f.riv_tq)[k * NT + tid] : 0.0;
  static_assert(9 * NTW <= 3 * NT, "wind staging");
#pragma unroll
  for (int k = 0; k < 3; ++k) r_wind[k] = k * NT + tid < 9 * nwd ? gp(f.wind)[k * NT + tid] : 0.0;
  double t0 = 0.0, dt0 = 0.0, rain0 = 0.0, bo0 = 0.0, bi0 = 0.0;
  long long steps0 = 0, target0 = 0;
  if (tid == 0) {
    t0 = sc->t; dt0 = sc->dt; rain0 = sc->rain_in; bo0 = sc->bnd_out; bi0 = sc->bnd_in;
    steps0 = sc->steps; target0 = sc->target;
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  mn = __builtin_inf();
  fb = __builtin_inf();
  for (int c = tid; c < nch; c += RED_CHUNK) {
    // records written by other workgroups: device-coherent loads
#pragma unroll
    for (int i = 0; i < NV; ++i)
      v[i] += __hip_atomic_load(redp + c * NRED + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    mn = fmin(mn, __hip_atomic_load(redp + c * NRED + NV, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    fb = fmin(fb, __hip_atomic_load(redp + c * NRED + NV + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  }
#pragma unroll
  for (int k = 0; k < 7; ++k)
    if (k * NT + tid < 7 * nst) s_storm[k * NT + tid] = r_storm[k];
  if (tid < ngt) s_gt[tid] = r_gt;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k * NT + tid < 3 * ntc) s_tide[k * NT + tid] = r_tide[k];
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (k * NT + tid < 2 * nrq) s_riv[k * NT + tid] = r_riv[k];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (k * NT + tid < 9 * nwd) s_wind[k * NT + tid] = r_wind[k];
  block_reduce();
  if (tid == 0) {
    __hip_atomic_store(red_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    double t = t0;
    long long steps = steps0;
    if (!init) {
      double bo = 0.0, bi = 0.0;
      for (int s = 0; s < rk.n; ++s) {
        bo += rk.w[s] * v[3 + s];
        bi += rk.w[s] * v[3 + MAX_STAGES + s];
      }
      sc->rain_in = rain0 + dt0 * v[1];
      sc->bnd_out = bo0 + dt0 * bo;
      sc->bnd_in = bi0 + dt0 * bi;
      t = t0 + dt0;
      steps = steps0 + 1;
      sc->t = t;
      sc->steps = steps;
      sc->dt_last = dt0;
    }
    sc->volume = v[0];
    sc->n_dry = (long long)(v[2]);
    sc->n_neg = (long long)(v[INEG]);
    sc->bad = fb;
    // init 2 keeps a step already set (restored from a checkpoint, or the
    // current one when forcing changes between steps)
    const double dtn = M.dt_fixed > 0.0 ? M.dt_fixed
                       : (init == 2 && dt0 > 0.0) ? dt0 : fmin(M.dt_max, M.cfl * mn);
    const bool bad = !(v[0] == v[0]) || v[0] == __builtin_inf() || v[0] == -__builtin_inf() || !(dtn > 0.0) ||
                     fb != __builtin_inf();
    if (bad) sc->error = 1;
    if (bad || steps >= target0) sc->active = 0;
    sc->dt = dtn;
    s_t = t;
    s_dt = dtn;
  }
  __syncthreads();
  // forcing for the coming step.  Record times increase strictly (checked
  // when they are set), so the interval holding ts is found by bisection:
  // the k with time(k) <= ts < time(k+1), given time(0) < ts < time(n-1).
  auto bracket = [](auto time, int n, double ts) {
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (time(mid) <= ts) lo = mid;
      else hi = mid;
    }
    return lo;
  };
  const double t = s_t, dt = s_dt;
  if (tid < MAX_SLOTS) {
    const int s = tid;
    for (int st = 0; st < rk.n; ++st) {
      const double ts = t + rk.c[st] * dt;
      double lev = 0.0, q = 0.0;
      if (f.ocean_mask & (1u << s)) {
        lev = f.tide_mean[s];
        for (int k = 0; k < f.tide_cnt[s]; ++k) {
          const int j = 3 * (f.tide_off[s] + k);
          const double a = tide_lds ? s_tide[j] : gp(f.tide_c)[j];
          const double T = tide_lds ? s_tide[j + 1] : gp(f.tide_c)[j + 1];
          const double ph = tide_lds ? s_tide[j + 2] : gp(f.tide_c)[j + 2];
          lev += a * sin(2.0 * 3.14159265358979323846 * ts / T + ph);
        }
      }
      if (f.river_mask & (1u << s)) {
        const int n = f.riv_cnt[s], o = 2 * f.riv_off[s];
        auto RT = [&](int k) { return riv_lds ? s_riv[o + 2 * k] : gp(f.riv_tq)[o + 2 * k]; };
        auto RQ = [&](int k) { return riv_lds ? s_riv[o + 2 * k + 1] : gp(f.riv_tq)[o + 2 * k + 1]; };
        if (n == 1 || ts <= RT(0)) {
          q = RQ(0);
        } else if (ts >= RT(n - 1)) {
          q = RQ(n - 1);
        } else {
          const int k = bracket(RT, n, ts);
          const double th = (ts - RT(k)) / (RT(k + 1) - RT(k));
          q = (1.0 - th) * RQ(k) + th * RQ(k + 1);
        }
      }
      sc->tide[st][s] = lev;
      sc->river[st][s] = q;
    }
  } else if (tid == MAX_SLOTS && f.rain_kind == RAIN_PARAM && f.n_storm > 0) {
    const int n = f.n_storm;
    auto R = [&](int i) { return i < 7 * NT ? s_storm[i] : gp(f.storm)[i]; };
    auto RT = [&](int k) { return R(7 * k); };
    if (n == 1 || t <= R(0)) {
      for (int i = 0; i < 6; ++i) sc->storm[i] = R(1 + i);
    } else if (t >= R(7 * (n - 1))) {
      for (int i = 0; i < 6; ++i) sc->storm[i] = R(7 * (n - 1) + 1 + i);
    } else {
      const int k = bracket(RT, n, t);
      const double th = (t - R(7 * k)) / (R(7 * (k + 1)) - R(7 * k));
      for (int i = 0; i < 6; ++i) sc->storm[i] = (1.0 - th) * R(7 * k + 1 + i) + th * R(7 * (k + 1) + 1 + i);
    }
  }
  if (tid == MAX_SLOTS + 2 && f.met_kind == MET_VORTEX && f.n_wind > 0) {
    const int n = f.n_wind;
    auto R = [&](int i) { return i < 9 * NTW ? s_wind[i] : gp(f.wind)[i]; };
    auto RT = [&](int k) { return R(9 * k); };
    if (n == 1 || t <= R(0)) {
      for (int i = 0; i < 8; ++i) sc->wind[i] = R(1 + i);
    } else if (t >= R(9 * (n - 1))) {
      for (int i = 0; i < 8; ++i) sc->wind[i] = R(9 * (n - 1) + 1 + i);
    } else {
      const int k = bracket(RT, n, t);
      const double th = (t - R(9 * k)) / (R(9 * (k + 1)) - R(9 * k));
      for (int i = 0; i < 8; ++i) sc->wind[i] = (1.0 - th) * R(9 * k + 1 + i) + th * R(9 * (k + 1) + 1 + i);
    }
  }
  if (tid == MAX_SLOTS + 1 && f.rain_kind == RAIN_GRID && f.gnrec > 0) {
    const int n = f.gnrec;
    auto TR = [&](int i) { return i < NT ? s_gt[i] : gp(f.gt)[i]; };
    if (n == 1 || t <= TR(0)) {
      sc->gk0 = 0; sc->gk1 = 0; sc->gth = 0.0;
    } else if (t >= TR(n - 1)) {
      sc->gk0 = n - 1; sc->gk1 = n - 1; sc->gth = 0.0;
    } else {
      const int k = bracket(TR, n, t);
      sc->gk0 = k; sc->gk1 = k + 1; sc->gth = (t - TR(k)) / (TR(k + 1) - TR(k));
    }
  }
}

// ------------------------------------------------------------ launchers
template <typename Real>
hipError_t launch_stage(int P, int flux, int limiter, int variant, const Member<Real>* m, const Tile* t, int n,
                        StageArgs a, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, int fused, int tile) {
  if (n <= 0) return hipSuccess;
  dim3 grid(xcd_grid(n)), block(tile);
  const bool timed = ev0 != nullptr || ev1 != nullptr;
#define DG_LAUNCH(KERNEL)                                                                       \
  {                                                                                            \
    if (timed) hipExtLaunchKernelGGL((KERNEL), grid, block, 0, s, ev0, ev1, 0, m, t, n, a);      \
    else hipLaunchKernelGGL((KERNEL), grid, block, 0, s, m, t, n, a);                          \
    return hipGetLastError();                                                                  \
  }
#define DG_STAGE(PP, FF, LL)                                                                    \
  if (P == PP && flux == FF && limiter == LL) {                                                 \
    if (variant == 1) DG_LAUNCH((stage_edge_kernel<Real, PP, FF, LL, 0, TILE>))                 \
    else DG_LAUNCH((stage_kernel<Real, PP, FF, LL>))                                            \
  }
  if (variant == 2) {
    // per-edge kernel with the area integrals on the matrix cores: p = 3,
    // FP32, 64-element tiles
    if constexpr (sizeof(Real) == 4) {
      if (P != 3 || tile != 64 || fused) return hipErrorInvalidValue;
      if (flux == 0 && limiter == 0) DG_LAUNCH((stage_edge_kernel<Real, 3, 0, 0, 0, 64, 1>))
      if (flux == 1 && limiter == 0) DG_LAUNCH((stage_edge_kernel<Real, 3, 1, 0, 0, 64, 1>))
      if (flux == 0 && limiter == 1) DG_LAUNCH((stage_edge_kernel<Real, 3, 0, 1, 0, 64, 1>))
      if (flux == 1 && limiter == 1) DG_LAUNCH((stage_edge_kernel<Real, 3, 1, 1, 0, 64, 1>))
    }
    return hipErrorInvalidValue;
  }
  if (tile != TILE) {
    // per-edge kernel on tiles of 64 or 128 elements (any p) or 512 (p = 1),
    // without the fused post-processing
    if (variant != 1 || fused || !(tile == 64 || tile == 128 || (tile == 512 && P == 1)))
      return hipErrorInvalidValue;
#define DG_TILED(PP, FF, LL)                                                                    \
  if (P == PP && flux == FF && limiter == LL) {                                                 \
    if (tile == 64) DG_LAUNCH((stage_edge_kernel<Real, PP, FF, LL, 0, 64>))                     \
    DG_LAUNCH((stage_edge_kernel<Real, PP, FF, LL, 0, 128>))                                    \
  }
    if (tile == 512) {
      if (flux == 0 && limiter == 0) DG_LAUNCH((stage_edge_kernel<Real, 1, 0, 0, 0, 512>))
      if (flux == 1 && limiter == 0) DG_LAUNCH((stage_edge_kernel<Real, 1, 1, 0, 0, 512>))
      if (flux == 0 && limiter == 1) DG_LAUNCH((stage_edge_kernel<Real, 1, 0, 1, 0, 512>))
      if (flux == 1 && limiter == 1) DG_LAUNCH((stage_edge_kernel<Real, 1, 1, 1, 0, 512>))
      return hipErrorInvalidValue;
    }
    DG_TILED(1, 0, 0) DG_TILED(1, 1, 0) DG_TILED(1, 0, 1) DG_TILED(1, 1, 1)
    DG_TILED(2, 0, 0) DG_TILED(2, 1, 0) DG_TILED(2, 0, 1) DG_TILED(2, 1, 1)
    DG_TILED(3, 0, 0) DG_TILED(3, 1, 0) DG_TILED(3, 0, 1) DG_TILED(3, 1, 1)
#undef DG_TILED
    return hipErrorInvalidValue;
  }
  if (fused) {
    if (variant != 1 || limiter != 1 || P > 2) return hipErrorInvalidValue;
    if (P == 1 && flux == 0) DG_LAUNCH((stage_edge_kernel<Real, 1, 0, 1, 1, TILE>))
    if (P == 1 && flux == 1) DG_LAUNCH((stage_edge_kernel<Real, 1, 1, 1, 1, TILE>))
    if (P == 2 && flux == 0) DG_LAUNCH((stage_edge_kernel<Real, 2, 0, 1, 1, TILE>))
    if (P == 2 && flux == 1) DG_LAUNCH((stage_edge_kernel<Real, 2, 1, 1, 1, TILE>))
    return hipErrorInvalidValue;
  }
  DG_STAGE(1, 0, 0) DG_STAGE(1, 1, 0) DG_STAGE(1, 0, 1) DG_STAGE(1, 1, 1)
  DG_STAGE(2, 0, 0) DG_STAGE(2, 1, 0) DG_STAGE(2, 0, 1) DG_STAGE(2, 1, 1)
  DG_STAGE(3, 0, 0) DG_STAGE(3, 1, 0) DG_STAGE(3, 0, 1) DG_STAGE(3, 1, 1)
#undef DG_STAGE
#undef DG_LAUNCH
  return hipErrorInvalidValue;
}

template <typename Real>
hipError_t launch_post(int P, int use_lim, const Member<Real>* m, const Tile* t, int n, StageArgs a, int init,
                       hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(xcd_grid(n)), block(TILE);
  if (P == 1) hipLaunchKernelGGL((post_kernel<Real, 1>), grid, block, 0, s, m, t, n, a, init, use_lim);
  else if (P == 2) hipLaunchKernelGGL((post_kernel<Real, 2>), grid, block, 0, s, m, t, n, a, init, use_lim);
  else if (P == 3) hipLaunchKernelGGL((post_kernel<Real, 3>), grid, block, 0, s, m, t, n, a, init, use_lim);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_classify(int P, const Member<Real>* m, const Tile* t, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  dim3 grid(xcd_grid(n)), block(TILE);
  if (P == 1) hipLaunchKernelGGL((classify_kernel<Real, 1>), grid, block, 0, s, m, t, n);
  else if (P == 2) hipLaunchKernelGGL((classify_kernel<Real, 2>), grid, block, 0, s, m, t, n);
  else hipLaunchKernelGGL((classify_kernel<Real, 3>), grid, block, 0, s, m, t, n);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_rain(const Member<Real>* m, const Tile* t, int n, int always, const Tile* node_tiles, int n_node_tiles,
                       hipStream_t s, int single) {
  if (!always && node_tiles && n_node_tiles > 0)
    hipLaunchKernelGGL((node_forcing_kernel<Real>), dim3(xcd_grid(n_node_tiles)), dim3(TILE), 0, s, m, node_tiles,
                       n_node_tiles, single);
  if (n > 0) hipLaunchKernelGGL((rain_kernel<Real>), dim3(xcd_grid(n)), dim3(TILE), 0, s, m, t, n, always);
  return hipGetLastError();
}

template <typename Real>
hipError_t launch_reduce(const Member<Real>* m, const int* ids, int n_members, int max_chunks, int init,
                         const RKInfo& rk, hipStream_t s, double* part_over) {
  if (n_members <= 0) return hipSuccess;
  hipLaunchKernelGGL((reduce_kernel<Real>), dim3(n_members, max_chunks < 1 ? 1 : max_chunks), dim3(RED_CHUNK), 0, s,
                     m, ids, init, rk, part_over);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void fill_zero_kernel(double* p, int n) {
  const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (i < n) p[i] = 0.0;
}

hipError_t launch_fill_zero(double* p, int n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

// Active flags of the members of a batch, gathered into one array so the
// host reads them in one copy.
template <typename Real>
__global__ __launch_bounds__(256) void active_flags_kernel(const Member<Real>* __restrict__ mem, int n,
                                                           int* __restrict__ out) {
  const int i = int(blockIdx.x) * 256 + int(threadIdx.x);
  if (i < n) out[i] = gp((const Scalars*)mem[i].sc)->active;
}

template <typename Real>
hipError_t launch_active_flags(const Member<Real>* m, int n, int* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((active_flags_kernel<Real>), dim3((n + 255) / 256), dim3(256), 0, s, m, n, out);
  return hipGetLastError();
}

#define DG_INST(R)                                                                                              \
  template hipError_t launch_stage<R>(int, int, int, int, const Member<R>*, const Tile*, int, StageArgs, hipStream_t, \
                                      hipEvent_t, hipEvent_t, int, int);                                    \
  template hipError_t launch_post<R>(int, int, const Member<R>*, const Tile*, int, StageArgs, int, hipStream_t);  \
  template hipError_t launch_classify<R>(int, const Member<R>*, const Tile*, int, hipStream_t);                   \
  template hipError_t launch_rain<R>(const Member<R>*, const Tile*, int, int, const Tile*, int, hipStream_t, int); \
  template hipError_t launch_reduce<R>(const Member<R>*, const int*, int, int, int, const RKInfo&, hipStream_t,  \
                                       double*);                                                              \
  template hipError_t launch_active_flags<R>(const Member<R>*, int, int*, hipStream_t);
DG_INST(float)
DG_INST(double)

}  // namespace dg
