// Host-side mesh preprocessing (see mesh.cpp).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace dg {

struct HostMesh {
  int64_t E = 0, n_nodes = 0, n_edges = 0, n_flipped = 0;
  std::vector<int32_t> perm;   // perm[internal] = caller's element id
  std::vector<int32_t> inv;    // inv[caller's id] = internal id
  // structure-of-arrays in internal (Hilbert) order
  std::vector<double> ev;      // [6][E] edge vectors v1-v0, v2-v1, v0-v2
  std::vector<double> hbv;     // [3][E]
  std::vector<double> fric;    // [E]
  std::vector<int32_t> nbr;    // [3][E] neighbour or -1 - (type | slot << 2)
  std::vector<uint8_t> nk;     // [E]
  std::vector<double> din;     // [E]
  std::vector<int32_t> tri;    // [3][E] node ids
  std::vector<double> lima;    // [6][E]
  std::vector<uint8_t> limc;   // [E]
  std::vector<double> area;    // [E]
  std::vector<double> xy;      // [2][n_nodes]
};

// Returns 0, or -1 with a message in err.
int build_mesh(int64_t n_nodes, const double* xy, const double* hb, const double* fric, int64_t n_tri,
               const int32_t* tri, int64_t n_bedges, const int32_t* bnodes, const int32_t* btype,
               const int32_t* bslot, HostMesh& out, std::string& err);

}  // namespace dg
