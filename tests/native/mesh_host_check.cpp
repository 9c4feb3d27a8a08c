// Host-side checks of the mesh preprocessing (build_mesh, build_halo), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitizers.py: valid meshes of several shapes and sizes
// with their invariants, and invalid inputs that must be refused with a
// message rather than read out of bounds.  Prints "ok" and exits 0 on
// success; any failed check exits 1.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <vector>

#include "mesh.h"

namespace {

int failures = 0;

void check(bool c, const char* what, const std::string& ctx = "") {
  if (!c) {
    std::fprintf(stderr, "FAILED: %s %s\n", what, ctx.c_str());
    ++failures;
  }
}

struct Grid {
  std::vector<double> xy, hb, fric;
  std::vector<int32_t> tri, bnodes, btype, bslot;
};

// nx x ny quads over a jittered rectangle, two triangles each (alternating
// diagonals, some triangles listed clockwise), every side a boundary of its
// own type and slot
Grid grid(int nx, int ny, unsigned seed) {
  Grid g;
  std::mt19937 rng(seed);
  std::uniform_real_distribution<double> jit(-0.2, 0.2);
  auto id = [&](int i, int j) { return j * (nx + 1) + i; };
  for (int j = 0; j <= ny; ++j)
    for (int i = 0; i <= nx; ++i) {
      const bool inner = i > 0 && i < nx && j > 0 && j < ny;
      g.xy.push_back(100.0 * (i + (inner ? jit(rng) : 0.0)));
      g.xy.push_back(80.0 * (j + (inner ? jit(rng) : 0.0)));
      g.hb.push_back(5.0 + std::sin(0.3 * i) * std::cos(0.2 * j));
      g.fric.push_back(0.02);
    }
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const int a = id(i, j), b = id(i + 1, j), c = id(i + 1, j + 1), d = id(i, j + 1);
      const bool flip = ((i + j) & 1) != 0, cw = ((i * 7 + j * 3) % 5) == 0;
      if (!flip) {
        g.tri.insert(g.tri.end(), {a, b, c});
        if (cw) g.tri.insert(g.tri.end(), {a, d, c}); else g.tri.insert(g.tri.end(), {a, c, d});
      } else {
        g.tri.insert(g.tri.end(), {a, b, d});
        if (cw) g.tri.insert(g.tri.end(), {b, d, c}); else g.tri.insert(g.tri.end(), {b, c, d});
      }
    }
  auto side = [&](int a, int b, int type, int slot) {
    g.bnodes.push_back(a); g.bnodes.push_back(b); g.btype.push_back(type); g.bslot.push_back(slot);
  };
  for (int i = 0; i < nx; ++i) side(id(i, 0), id(i + 1, 0), 1, 0);          // ocean
  for (int j = 0; j < ny; ++j) side(id(nx, j), id(nx, j + 1), 2, 3);       // river
  for (int i = 0; i < nx; ++i) side(id(i, ny), id(i + 1, ny), 3, 0);       // outflow
  // the left side stays land (not listed)
  return g;
}

int build(const Grid& g, dg::HostMesh& M, std::string& err, int64_t n_bedges = -1) {
  const int64_t nb = n_bedges < 0 ? int64_t(g.btype.size()) : n_bedges;
  return dg::build_mesh(int64_t(g.hb.size()), g.xy.data(), g.hb.data(), g.fric.data(), int64_t(g.tri.size() / 3),
                        g.tri.data(), nb, g.bnodes.data(), g.btype.data(), g.bslot.data(), M, err);
}

void valid_mesh(int nx, int ny, unsigned seed) {
  const std::string ctx = std::to_string(nx) + "x" + std::to_string(ny);
  Grid g = grid(nx, ny, seed);
  dg::HostMesh M;
  std::string err;
  check(build(g, M, err) == 0, "valid mesh refused", ctx + ": " + err);
  if (failures) return;
  const int64_t E = M.E;
  check(E == 2 * nx * ny, "element count", ctx);
  check(M.n_edges == (3 * E + 2 * (nx + ny)) / 2, "edge count", ctx);
  // perm and inv are inverse permutations
  std::vector<int> seen(E, 0);
  for (int64_t e = 0; e < E; ++e) {
    const int32_t p = M.perm[e];
    check(p >= 0 && p < E, "perm range", ctx);
    if (p >= 0 && p < E) {
      ++seen[p];
      check(M.inv[p] == e, "inv(perm) = id", ctx);
    }
  }
  for (int64_t e = 0; e < E; ++e) check(seen[e] == 1, "perm is a permutation", ctx);
  // neighbours are mutual through the stored local edge ids; boundary codes
  // carry the listed types
  int64_t nbnd = 0;
  int types[4] = {0, 0, 0, 0};
  for (int64_t e = 0; e < E; ++e) {
    check(M.area[e] > 0.0, "positive area", ctx);
    for (int k = 0; k < 3; ++k) {
      const int32_t f = M.nbr[k * E + e];
      if (f >= 0) {
        check(f < E && f != e, "neighbour range", ctx);
        const int kn = (M.nk[e] >> (2 * k)) & 3;
        check(kn < 3 && M.nbr[kn * E + f] == int32_t(e), "neighbour is mutual", ctx);
      } else {
        ++nbnd;
        const int code = -1 - f;
        ++types[code & 3];
      }
    }
  }
  check(nbnd == 2 * (nx + ny), "boundary edge count", ctx);
  check(types[0] == ny && types[1] == nx && types[2] == ny && types[3] == nx, "boundary types", ctx);
  for (const int T : {64, 128, 256, 512}) {
    dg::Halo H;
    std::string herr;
    const int rc = dg::build_halo(M, T, H, herr);
    if (rc == 0) {
      const int64_t nt = (E + T - 1) / T;
      check(int64_t(H.off.size()) == nt + 1 && int64_t(H.n1.size()) == nt, "halo sizes", ctx);
      for (size_t i = 0; i < H.id.size(); ++i) check(H.id[i] >= 0 && H.id[i] < E, "halo id range", ctx);
    }
  }
}

void refused(Grid g, const char* what, int64_t n_bedges = -1) {
  dg::HostMesh M;
  std::string err;
  const int rc = build(g, M, err, n_bedges);
  check(rc == -1 && !err.empty(), what, err);
}

}  // namespace

int main() {
  valid_mesh(1, 1, 1);
  valid_mesh(3, 2, 2);
  valid_mesh(17, 9, 3);
  valid_mesh(64, 40, 4);
  valid_mesh(150, 120, 5);
  // an empty mesh is accepted
  {
    dg::HostMesh M;
    std::string err;
    check(dg::build_mesh(0, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, M, err) == 0,
          "empty mesh", err);
  }
  Grid base = grid(6, 5, 7);
  { Grid g = base; g.tri[4] = int32_t(g.hb.size()); refused(g, "node id past the end"); }
  { Grid g = base; g.tri[0] = -3; refused(g, "negative node id"); }
  { Grid g = base; g.tri[2] = g.tri[1]; refused(g, "zero-area triangle"); }
  { Grid g = base; g.xy[9] = NAN; refused(g, "non-finite coordinate"); }
  { Grid g = base; g.fric[3] = -1.0; refused(g, "negative friction"); }
  { Grid g = base; g.tri.insert(g.tri.end(), {g.tri[0], g.tri[1], g.tri[2] + 1}); refused(g, "edge of three triangles"); }
  { Grid g = base; g.bnodes[0] = int32_t(g.hb.size()) + 5; refused(g, "boundary node past the end"); }
  { Grid g = base; g.btype[1] = 4; refused(g, "boundary type out of range"); }
  { Grid g = base; g.bslot[2] = 16; refused(g, "boundary slot out of range"); }
  { Grid g = base; g.bnodes[0] = 8; g.bnodes[1] = 9; refused(g, "interior edge listed as boundary"); }
  {
    dg::HostMesh M;
    std::string err;
    check(dg::build_mesh(-1, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, M, err) == -1,
          "negative node count", err);
    check(dg::build_mesh(4, nullptr, nullptr, nullptr, 0, nullptr, 0, nullptr, nullptr, nullptr, M, err) == -1,
          "nodes without coordinates", err);
    check(dg::build_mesh(int64_t(base.hb.size()), base.xy.data(), base.hb.data(), base.fric.data(),
                         int64_t(base.tri.size() / 3), base.tri.data(), 2, nullptr, nullptr, nullptr, M, err) == -1,
          "boundary edges without their nodes", err);
  }
  if (failures) {
    std::fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  std::printf("ok\n");
  return 0;
}
