// Host-side mesh preprocessing for the DG solver.
//
// Builds, from the caller's nodes, triangles and typed boundary edges
// (Sec. 2.1 boundary partition), everything the element-local operator of
// Sec. 2.3 needs: CCW orientation, the neighbour across every local edge
// (local edge k joins local vertices k -> k+1) and that neighbour's local
// edge, boundary codes, FP64 edge vectors, inscribed-circle diameters and the
// slope-limiter stencil; then renumbers elements along a Hilbert curve so
// that neighbours are close in memory.
#include "mesh.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <numeric>

namespace dg {

namespace {

// Hilbert-curve index of (x, y) in [0, 2^order)^2
uint64_t hilbert(uint32_t x, uint32_t y, int order) {
  const uint32_t n = 1u << order;
  uint64_t d = 0;
  for (uint32_t s = n >> 1; s > 0; s >>= 1) {
    const uint32_t rx = (x & s) ? 1u : 0u;
    const uint32_t ry = (y & s) ? 1u : 0u;
    d += uint64_t(s) * s * ((3u * rx) ^ ry);
    if (ry == 0) {
      if (rx == 1) {
        x = n - 1 - x;
        y = n - 1 - y;
      }
      const uint32_t t = x;
      x = y;
      y = t;
    }
  }
  return d;
}

}  // namespace

int build_mesh(int64_t n_nodes, const double* xy, const double* hb, const double* fric, int64_t n_tri,
               const int32_t* tri_in, int64_t n_bedges, const int32_t* bnodes, const int32_t* btype,
               const int32_t* bslot, HostMesh& M, std::string& err) {
  char buf[256];
  if (n_nodes < 0 || n_tri < 0 || n_bedges < 0) { err = "negative size"; return -1; }
  if (n_tri > (int64_t(1) << 30)) { err = "too many triangles"; return -1; }
  if ((n_nodes > 0 && (!xy || !hb || !fric)) || (n_tri > 0 && !tri_in) || (n_bedges > 0 && !bnodes)) {
    err = "null array";
    return -1;
  }
  for (int64_t i = 0; i < n_nodes; ++i) {
    if (!std::isfinite(xy[2 * i]) || !std::isfinite(xy[2 * i + 1]) || !std::isfinite(hb[i]) ||
        !std::isfinite(fric[i]) || fric[i] < 0.0) {
      snprintf(buf, sizeof buf, "node %lld: non-finite coordinate/bathymetry or bad friction", (long long)i);
      err = buf;
      return -1;
    }
  }
  const int64_t E = n_tri;
  M.E = E;
  M.n_nodes = n_nodes;
  std::vector<int32_t> tri(3 * E);
  M.n_flipped = 0;
  for (int64_t e = 0; e < E; ++e) {
    int32_t a = tri_in[3 * e], b = tri_in[3 * e + 1], c = tri_in[3 * e + 2];
    if (a < 0 || b < 0 || c < 0 || a >= n_nodes || b >= n_nodes || c >= n_nodes) {
      snprintf(buf, sizeof buf, "triangle %lld: node id out of range", (long long)e);
      err = buf;
      return -1;
    }
    const double cr = (xy[2 * b] - xy[2 * a]) * (xy[2 * c + 1] - xy[2 * a + 1]) -
                      (xy[2 * b + 1] - xy[2 * a + 1]) * (xy[2 * c] - xy[2 * a]);
    if (cr == 0.0) {
      snprintf(buf, sizeof buf, "triangle %lld: zero area", (long long)e);
      err = buf;
      return -1;
    }
    if (cr < 0.0) { std::swap(b, c); ++M.n_flipped; }
    tri[3 * e] = a; tri[3 * e + 1] = b; tri[3 * e + 2] = c;
  }
  // ---- edges: sort (min, max) node keys
  std::vector<std::pair<uint64_t, uint32_t>> keys(3 * E);
  for (int64_t e = 0; e < E; ++e)
    for (int k = 0; k < 3; ++k) {
      const uint32_t a = tri[3 * e + k], b = tri[3 * e + (k + 1) % 3];
      keys[3 * e + k] = {(uint64_t(std::min(a, b)) << 32) | std::max(a, b), uint32_t(3 * e + k)};
    }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> nbr(3 * E, -1);
  std::vector<int8_t> nbe(3 * E, -1);
  int64_t n_edges = 0;
  std::vector<std::pair<uint64_t, uint32_t>> bkeys;   // boundary local edges
  for (size_t i = 0; i < keys.size();) {
    size_t j = i;
    while (j < keys.size() && keys[j].first == keys[i].first) ++j;
    if (j - i > 2) {
      snprintf(buf, sizeof buf, "edge (%u,%u) shared by more than two triangles", unsigned(keys[i].first >> 32),
               unsigned(keys[i].first & 0xffffffffu));
      err = buf;
      return -1;
    }
    if (j - i == 2) {
      const uint32_t f0 = keys[i].second, f1 = keys[i + 1].second;
      nbr[f0] = f1 / 3; nbe[f0] = f1 % 3;
      nbr[f1] = f0 / 3; nbe[f1] = f0 % 3;
    } else {
      bkeys.push_back(keys[i]);
    }
    ++n_edges;
    i = j;
  }
  M.n_edges = n_edges;
  // boundary codes: LAND unless listed
  std::vector<int32_t> bcode(3 * E, 0);
  for (int64_t i = 0; i < n_bedges; ++i) {
    const int32_t a = bnodes[2 * i], b = bnodes[2 * i + 1];
    if (a < 0 || b < 0 || a >= n_nodes || b >= n_nodes) { err = "boundary edge node id out of range"; return -1; }
    const int32_t ty = btype ? btype[i] : 0, sl = bslot ? bslot[i] : 0;
    if (ty < 0 || ty > 3) { err = "bad boundary type"; return -1; }
    if (sl < 0 || sl >= 16) { err = "boundary slot out of range"; return -1; }
    const uint64_t key = (uint64_t(std::min(a, b)) << 32) | uint32_t(std::max(a, b));
    auto it = std::lower_bound(bkeys.begin(), bkeys.end(), std::make_pair(key, uint32_t(0)));
    if (it == bkeys.end() || it->first != key) {
      snprintf(buf, sizeof buf, "boundary edge %lld is not on the mesh boundary", (long long)i);
      err = buf;
      return -1;
    }
    bcode[it->second] = ty | (sl << 2);
  }
  // ---- geometry in the caller's order
  std::vector<double> ev(6 * E), din(E), area(E), cen(2 * E);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t* t = &tri[3 * e];
    double per = 0.0;
    for (int k = 0; k < 3; ++k) {
      const double dx = xy[2 * t[(k + 1) % 3]] - xy[2 * t[k]];
      const double dy = xy[2 * t[(k + 1) % 3] + 1] - xy[2 * t[k] + 1];
      ev[6 * e + 2 * k] = dx;
      ev[6 * e + 2 * k + 1] = dy;
      per += std::hypot(dx, dy);
    }
    const double j00 = 0.5 * (xy[2 * t[1]] - xy[2 * t[0]]), j01 = 0.5 * (xy[2 * t[2]] - xy[2 * t[0]]);
    const double j10 = 0.5 * (xy[2 * t[1] + 1] - xy[2 * t[0] + 1]), j11 = 0.5 * (xy[2 * t[2] + 1] - xy[2 * t[0] + 1]);
    area[e] = 2.0 * (j00 * j11 - j01 * j10);
    din[e] = 4.0 * area[e] / per;
    cen[2 * e] = (xy[2 * t[0]] + xy[2 * t[1]] + xy[2 * t[2]]) / 3.0;
    cen[2 * e + 1] = (xy[2 * t[0] + 1] + xy[2 * t[1] + 1] + xy[2 * t[2] + 1]) / 3.0;
  }
  // ---- limiter stencil: m_i - b0 = a_j (b_j - b0) + a_k (b_k - b0), a >= 0,
  // j = neighbour across edge i, k = the next (then the one after) neighbour
  std::vector<double> lim(6 * E, 0.0);
  std::vector<uint8_t> limc(E, 0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t* nb = &nbr[3 * e];
    if (nb[0] < 0 || nb[1] < 0 || nb[2] < 0) continue;
    const int32_t* t = &tri[3 * e];
    bool ok = true;
    uint8_t code = 0;
    for (int i = 0; i < 3 && ok; ++i) {
      const double mx = 0.5 * (xy[2 * t[i]] + xy[2 * t[(i + 1) % 3]]) - cen[2 * e];
      const double my = 0.5 * (xy[2 * t[i] + 1] + xy[2 * t[(i + 1) % 3] + 1]) - cen[2 * e + 1];
      bool found = false;
      for (int off = 1; off <= 2 && !found; ++off) {
        const int j = i, k = (i + off) % 3;
        const double ax = cen[2 * nb[j]] - cen[2 * e], ay = cen[2 * nb[j] + 1] - cen[2 * e + 1];
        const double bx = cen[2 * nb[k]] - cen[2 * e], by = cen[2 * nb[k] + 1] - cen[2 * e + 1];
        const double det = ax * by - ay * bx;
        if (det == 0.0) continue;
        const double aj = (mx * by - my * bx) / det;
        const double ak = (ax * my - ay * mx) / det;
        if (aj >= 0.0 && ak >= 0.0) {
          lim[6 * e + 2 * i] = aj;
          lim[6 * e + 2 * i + 1] = ak;
          if (off == 2) code |= uint8_t(1u << (1 + i));
          found = true;
        }
      }
      ok = found;
    }
    limc[e] = ok ? uint8_t(code | 1u) : 0;
  }
  // ---- Hilbert order of the centroids
  double x0 = 1e300, x1 = -1e300, y0 = 1e300, y1 = -1e300;
  for (int64_t e = 0; e < E; ++e) {
    x0 = std::min(x0, cen[2 * e]); x1 = std::max(x1, cen[2 * e]);
    y0 = std::min(y0, cen[2 * e + 1]); y1 = std::max(y1, cen[2 * e + 1]);
  }
  const double span = std::max(x1 - x0, y1 - y0);
  const double sc = span > 0.0 ? 65535.0 / span : 0.0;
  std::vector<std::pair<uint64_t, int32_t>> hk(E);
  for (int64_t e = 0; e < E; ++e) {
    const uint32_t ix = uint32_t((cen[2 * e] - x0) * sc), iy = uint32_t((cen[2 * e + 1] - y0) * sc);
    hk[e] = {hilbert(ix, iy, 16), int32_t(e)};
  }
  std::sort(hk.begin(), hk.end());
  M.perm.resize(E);
  M.inv.resize(E);
  for (int64_t i = 0; i < E; ++i) {
    M.perm[i] = hk[i].second;
    M.inv[hk[i].second] = int32_t(i);
  }
  // ---- permuted SoA arrays
  M.ev.assign(6 * E, 0.0);
  M.hbv.assign(3 * E, 0.0);
  M.fric.assign(E, 0.0);
  M.nbr.assign(3 * E, 0);
  M.nk.assign(E, 0);
  M.din.assign(E, 0.0);
  M.tri.assign(3 * E, 0);
  M.lima.assign(6 * E, 0.0);
  M.limc.assign(E, 0);
  M.area.assign(E, 0.0);
  for (int64_t i = 0; i < E; ++i) {
    const int64_t e = M.perm[i];
    for (int j = 0; j < 6; ++j) {
      M.ev[j * E + i] = ev[6 * e + j];
      M.lima[j * E + i] = lim[6 * e + j];
    }
    uint8_t nk = 0;
    double f = 0.0;
    for (int k = 0; k < 3; ++k) {
      const int32_t node = tri[3 * e + k];
      M.tri[k * E + i] = node;
      M.hbv[k * E + i] = hb[node];
      const int32_t n = nbr[3 * e + k];
      if (n >= 0) {
        M.nbr[k * E + i] = M.inv[n];
        nk |= uint8_t(nbe[3 * e + k] << (2 * k));
      } else {
        M.nbr[k * E + i] = -1 - bcode[3 * e + k];
      }
    }
    f = (fric[tri[3 * e]] + fric[tri[3 * e + 1]]) + fric[tri[3 * e + 2]];
    M.fric[i] = f / 3.0;
    M.nk[i] = nk;
    M.din[i] = din[e];
    M.limc[i] = limc[e];
    M.area[i] = area[e];
  }
  M.xy.assign(2 * n_nodes, 0.0);
  for (int64_t n = 0; n < n_nodes; ++n) {
    M.xy[n] = xy[2 * n];
    M.xy[n_nodes + n] = xy[2 * n + 1];
  }
  return 0;
}

int build_halo(const HostMesh& M, int T, Halo& H, std::string& err) {
  const int64_t E = M.E;
  const int64_t nt = (E + T - 1) / T;
  H = Halo{};
  H.T = T;
  H.off.assign(nt + 1, 0);
  H.n1.assign(nt, 0);
  H.eslot.assign(E, 0);
  std::vector<int32_t> r1, r2;
  for (int64_t t = 0; t < nt; ++t) {
    const int64_t a = t * T, b = std::min<int64_t>(E, a + T);
    auto outside = [&](int32_t x) { return x >= 0 && (x < a || x >= b); };
    r1.clear();
    r2.clear();
    for (int64_t e = a; e < b; ++e)
      for (int k = 0; k < 3; ++k) {
        const int32_t n = M.nbr[k * E + e];
        if (outside(n)) r1.push_back(n);
      }
    std::sort(r1.begin(), r1.end());
    r1.erase(std::unique(r1.begin(), r1.end()), r1.end());
    for (int32_t y : r1)
      for (int k = 0; k < 3; ++k) {
        const int32_t n = M.nbr[k * E + y];
        if (outside(n) && !std::binary_search(r1.begin(), r1.end(), n)) r2.push_back(n);
      }
    std::sort(r2.begin(), r2.end());
    r2.erase(std::unique(r2.begin(), r2.end()), r2.end());
    const int64_t n1 = int64_t(r1.size()), n2 = int64_t(r2.size());
    if (T + n1 + n2 > int64_t(HALO_NONE)) {
      err = "tile " + std::to_string(t) + " has too large a neighbourhood for 10-bit slots";
      return -1;
    }
    H.max_n1 = std::max<int>(H.max_n1, int(n1));
    H.max_n2 = std::max<int>(H.max_n2, int(n2));
    H.n1[t] = int32_t(n1);
    H.off[t + 1] = H.off[t] + int32_t(n1 + n2);
    auto slot = [&](int32_t x) -> uint32_t {
      if (x < 0) return HALO_NONE;
      if (x >= a && x < b) return uint32_t(x - a);
      auto i1 = std::lower_bound(r1.begin(), r1.end(), x);
      if (i1 != r1.end() && *i1 == x) return uint32_t(T + (i1 - r1.begin()));
      auto i2 = std::lower_bound(r2.begin(), r2.end(), x);
      return uint32_t(T + n1 + (i2 - r2.begin()));   // x is in ring 2
    };
    for (int64_t e = a; e < b; ++e) {
      uint32_t v = 0;
      for (int k = 0; k < 3; ++k) v |= slot(M.nbr[k * E + e]) << (10 * k);
      H.eslot[e] = v;
    }
    for (int32_t y : r1) {
      uint32_t v = 0;
      for (int k = 0; k < 3; ++k) v |= slot(M.nbr[k * E + y]) << (10 * k);
      H.id.push_back(y);
      H.nslot.push_back(v);
    }
    for (int32_t z : r2) {
      H.id.push_back(z);
      H.nslot.push_back(0);
    }
  }
  return 0;
}

}  // namespace dg
