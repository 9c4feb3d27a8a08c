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

// Neighbourhood of every tile of T consecutive (internal-order) elements,
// for a stage kernel that applies the limiter and positive-depth operator
// of the previous stage itself: ring 1 = elements outside the tile that
// share an edge with it, ring 2 = elements outside tile and ring 1 that
// share an edge with ring 1.  A tile numbers its slots 0 .. T-1 (its own
// elements, local index), T .. T+n1-1 (ring 1), T+n1 .. T+n1+n2-1 (ring 2);
// neighbour slots are packed 10 bits each (k-th neighbour in bits 10k),
// HALO_NONE for a boundary edge.
constexpr uint32_t HALO_NONE = 0x3FF;
struct Halo {
  int T = 0;
  int max_n1 = 0, max_n2 = 0;       // largest ring sizes over the tiles
  std::vector<int32_t> off;         // [n_tiles + 1] first entry of each tile
  std::vector<int32_t> n1;          // [n_tiles] ring-1 entries (ring 2 follows)
  std::vector<int32_t> id;          // [entries] internal element id
  std::vector<uint32_t> nslot;      // [entries] neighbour slots of a ring-1 entry (0 for ring 2)
  std::vector<uint32_t> eslot;      // [E] neighbour slots of every element within its own tile
};

// Builds the halo of every tile of T elements (T <= 512).  Returns 0, or -1
// when some tile's slots do not fit 10 bits.
int build_halo(const HostMesh& M, int T, Halo& H, std::string& err);

// Returns 0, or -1 with a message in err.
int build_mesh(int64_t n_nodes, const double* xy, const double* hb, const double* fric, int64_t n_tri,
               const int32_t* tri, int64_t n_bedges, const int32_t* bnodes, const int32_t* btype,
               const int32_t* bslot, HostMesh& out, std::string& err);

}  // namespace dg
