// Internal data layout of the DG solver (device structs and launchers).
//
// Element-major structure of arrays: every per-element quantity is an array
// of length E in Hilbert-curve element order, so that the 64 lanes of a
// wavefront read consecutive addresses and the neighbours they gather sit in
// nearby cache lines.  The state of one buffer is 3 * Np arrays
// W[(var * Np + mode) * E + e] for var in (zeta, qx, qy).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dg {

constexpr int TILE = 256;          // elements per workgroup (4 wavefronts)
// Largest halo a tile may have for the fused stage kernel (ring 1: outside
// elements sharing an edge with the tile; ring 2: those sharing an edge with
// ring 1); a mesh with a larger one keeps the separate post pass.
constexpr int HALO_R1 = 112, HALO_R2 = 144;
constexpr uint32_t HALO_SLOT_MASK = 0x3FF;   // 10-bit slot; all ones: boundary edge
constexpr int MAX_STAGES = 5;
constexpr int MAX_SLOTS = 16;
// per-tile FP64 partial sums: boundary out/in flux per stage, volume,
// min(d/lambda), rain volume, dry count, count of elements with a negative
// mean depth, smallest element id with a non-finite mean depth or wave
// speed (infinity if none)
enum PartKind {
  P_OUT0 = 0, P_IN0 = MAX_STAGES, P_VOL = 2 * MAX_STAGES, P_MINR, P_RAIN, P_NDRY, P_NNEG, P_BAD, NPART
};
// Partials are kept per wavefront: PSLOT slots per 256-element tile, slot s
// of tile t covering elements 256 t + 64 s .. 256 t + 64 s + 63, so kernels
// of any workgroup size write them alike and nothing is combined across
// workgroups; the reduction combines a tile's slots as (s0 + s1) + (s2 + s3)
// (minima alike) and takes a slot that starts at or beyond E as empty.
constexpr int PSLOT = TILE / 64;
__host__ __device__ inline size_t part_row(int n_tiles) { return size_t(PSLOT) * (n_tiles > 0 ? n_tiles : 1); }
enum RainKind { RAIN_CONST = 0, RAIN_PARAM = 1, RAIN_GRID = 2 };
enum MetKind { MET_NONE = 0, MET_VORTEX = 1 };
// wind stress and pressure forcing: air and water densities (kg/m^3), cap
// of the drag coefficient
constexpr double RHO_AIR = 1.15, RHO_WATER = 1000.0, CD_MAX = 3.5e-3;
// end-of-step reduction: one workgroup per RED_CHUNK tiles writes a record of
// NRED doubles (the NPART-style sums, the dt minimum and the first
// non-finite element); the last workgroup to finish combines the records in
// chunk order
constexpr int RED_CHUNK = 256;
constexpr int NRED = 16;
__host__ __device__ inline int red_chunks(int n_tiles) { return n_tiles > 0 ? (n_tiles + RED_CHUNK - 1) / RED_CHUNK : 1; }

// Device-resident time/budget/forcing scalars of one member.  Written only
// by the reduce kernel (the last launch of a step) and by the host between
// steps, read by every other kernel.
struct Scalars {
  double t, dt, dt_last;
  double volume, rain_in, bnd_in, bnd_out;
  long long steps, n_dry, target;
  long long n_neg;                      // elements with a negative mean depth
  double bad;                           // first element (internal order) with a non-finite state, or inf
  int active, error;
  double tide[MAX_STAGES][MAX_SLOTS];   // ocean level at each stage time
  double river[MAX_STAGES][MAX_SLOTS];  // river normal flux at each stage time
  double storm[6];                      // xc, yc, peak, T0, r_m, r_e at t^n
  double wind[8];                       // xc, yc, dp, rm, B, wf, wbx, wby at t^n
  int gk0, gk1;                         // rain-lattice records around t^n
  double gth;                           // weight of record gk1
};

struct Forcing {
  int rain_kind;
  int n_storm;                // records of (t, xc, yc, peak, T0, rm, re)
  const double* storm;
  int gnx, gny, gnrec;
  double gx0, gy0, gdx, gdy;
  const double* gt;           // [gnrec]
  const float* gvals;         // [gnrec][gny][gnx]
  unsigned ocean_mask, river_mask;
  double tide_mean[MAX_SLOTS];
  int tide_off[MAX_SLOTS], tide_cnt[MAX_SLOTS];   // triples in tide_c
  int riv_off[MAX_SLOTS], riv_cnt[MAX_SLOTS];     // (t, q) pairs in riv_tq
  const double* tide_c;
  const double* riv_tq;
  int n_tide, n_riv;          // rows in tide_c (triples) and riv_tq (pairs)
  int met_kind;               // MetKind
  int n_wind;                 // wind records (t, xc, yc, dp, rm, B, wf, wbx, wby)
  const double* wind;
};

template <typename Real>
struct Member {
  int E, n_nodes, n_tiles, friction;
  double H0, g, cfl, dt_fixed, dt_max;
  double feps;                // exchange threshold 1e-3 H0 sqrt(g H0) of a wet-dry edge
  // static mesh data (read-only, shareable between members)
  const Real* ev;             // [6][E] edge vectors v1-v0, v2-v1, v0-v2 (x, y)
  const Real* hbv;            // [3][E] bathymetry at the vertices
  const Real* fric;           // [E]    element friction coefficient
  const int* nbr;             // [3][E] neighbour id, or -1 - (type | slot << 2)
  const uint8_t* nk;          // [E]    neighbours' local edge ids, 2 bits each
  const Real* din;            // [E]    inscribed-circle diameter
  const int* tri;             // [3][E] node ids
  const double* nxy;          // [2][n_nodes] node coordinates
  const Real* lima;           // [6][E] limiter weights (alpha_j, alpha_k) per midpoint
  const uint8_t* limc;        // [E]    bit0: limitable; bit 1+i: second neighbour of midpoint i is i+2
  // dynamic
  Real* W[3];                 // state buffers
  Real* Wt;                   // initial state as given, before the set-up pass
  uint8_t* F[3];              // dry flags of the state in W[i] (bit 0)
  // [2][E] fully-wet bytes of a stage's raw output (limiter on): stage i
  // writes fullwet[i & 1], its post pass or the next stage reads it
  uint8_t* fullwet[2];
  // halo of every stage tile (see HaloDims), for the stage kernel that
  // applies the previous stage's limiter and positive depth itself; null
  // when the mesh has none
  const int* h_off;           // [n_tiles + 1] first halo entry of each tile
  const int* h_n1;            // [n_tiles] ring-1 entries (ring 2 follows)
  const int* h_id;            // [entries] element id
  const uint32_t* h_nslot;    // [entries] a ring-1 entry's neighbour slots, 10 bits each
  const uint32_t* h_eslot;    // [E] an element's neighbour slots in its own tile
  Real* R;                    // [E] element rain rate
  double* rn;                 // [n_nodes] nodal rain rate
  Real* met;                  // [3][n_nodes] kinematic wind stress (x, y) and pressure head at t^n
  double* part;               // [NPART][PSLOT * n_tiles], see part_row
  double* red;                // [red_chunks(n_tiles)][NRED] chunk records
  unsigned* red_count;        // chunks finished in the current reduction (0 between launches)
  Scalars* sc;
  Forcing fo;
};

struct StageArgs {
  int stage;                  // 0-based stage index
  int last;                   // 1 on the last stage of a step
  int in_buf, out_buf;        // state buffer indices
  int fin, fout;              // flag buffer indices
  double a, b, gam;           // w_out = a w^n + b (w_in + gam dt L(w_in))
  int single;                 // 1: one member, tile i of the launch is tile i of member 0
  double* part;               // tile partials, chunk records and counter laid out as the
                              // member's part array, used instead of it (nullptr: the member's)
};

struct Tile { int member, tile; };

struct RKInfo {
  int n;
  double w[MAX_STAGES];       // weight of each stage's boundary flux in w^{n+1}
  double c[MAX_STAGES];       // stage times t^n + c_i dt
};

// launchers (kernels.hip)
// ev0/ev1, when given, receive the start and end time of the stage kernel's
// own dispatch (no marker packets around it)
// fused = 1 (variant 1, limiter on, p <= 2, members with a halo): the stage
// reads the previous stage's raw output and applies its limiter and
// positive-depth operator itself, in place of that stage's post pass
// tile = 64, 128 or (p = 1) 512 (variant 1, not fused): workgroups of that
// many elements; the tile list and count are then those of such tiles
template <typename Real>
hipError_t launch_stage(int P, int flux, int limiter, int variant, const Member<Real>* d_members,
                        const Tile* d_tiles, int n_tiles, StageArgs a, hipStream_t s, hipEvent_t ev0 = nullptr,
                        hipEvent_t ev1 = nullptr, int fused = 0, int tile = TILE);
template <typename Real>
hipError_t launch_post(int P, int use_lim, const Member<Real>* d_members, const Tile* d_tiles, int n_tiles,
                       StageArgs a, int init, hipStream_t s);
template <typename Real>
hipError_t launch_classify(int P, const Member<Real>* d_members, const Tile* d_tiles, int n_tiles,
                           hipStream_t s);
// rain at t^n: nodal rates (node tiles), then element means (element tiles);
// always = 1 only averages (constant nodal rain at set-up)
template <typename Real>
hipError_t launch_rain(const Member<Real>* d_members, const Tile* d_tiles, int n_tiles, int always,
                       const Tile* d_node_tiles, int n_node_tiles, hipStream_t s,
                       int single = 0);
// grid: n_members x max_chunks workgroups (max_chunks = largest red_chunks
// over the members); d_member_ids == nullptr for a single context (member 0).
// init: 0 = end of a step; 1 = set-up (dt from the state); 2 = set-up that
// keeps a dt > 0 already in the scalars (restored or current)
// part_over: as StageArgs::part (single member only)
template <typename Real>
hipError_t launch_reduce(const Member<Real>* d_members, const int* d_member_ids, int n_members, int max_chunks,
                         int init, const RKInfo& rk, hipStream_t s, double* part_over = nullptr);
// zero n doubles at p (a kernel, so that it can sit in a captured graph)
hipError_t launch_fill_zero(double* p, int n, hipStream_t s);
// out[i] = active flag of member i, i < n
template <typename Real>
hipError_t launch_active_flags(const Member<Real>* d_members, int n, int* out, hipStream_t s);

}  // namespace dg
