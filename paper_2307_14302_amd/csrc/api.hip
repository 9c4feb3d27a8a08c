// C ABI of the DG solver: contexts, state I/O, forcing, stepping, batches.
// See include/dgswe.h for the contract of every call.
#include "dgswe.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "device_common.h"
#include "internal.h"
#include "mesh.h"

using namespace dg;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(x)                                                                              \
  do {                                                                                         \
    hipError_t e_ = (x);                                                                       \
    if (e_ == hipErrorOutOfMemory)                                                             \
      return fail(DGSWE_ENOMEM, std::string(#x) + ": " + oom_message());                       \
    if (e_ != hipSuccess) return fail(DGSWE_EHIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Device memory handed over by the caller (dgswe_workspace_bind): a
// first-fit sub-allocator over [base, base + cap) with 256-byte blocks and
// coalescing of freed neighbours.  The caller keeps ownership of the memory.
struct Arena {
  static constexpr size_t ALIGN = 256;
  char* base = nullptr;
  size_t cap = 0;
  std::map<size_t, size_t> free_;      // offset -> length of free ranges
  Arena(void* p, size_t n) : base(static_cast<char*>(p)), cap(n / ALIGN * ALIGN) { free_[0] = cap; }
  void* take(size_t n) {
    n = (n + ALIGN - 1) / ALIGN * ALIGN;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      return base + off;
    }
    return nullptr;
  }
  void give(void* p, size_t n) {
    n = (n + ALIGN - 1) / ALIGN * ALIGN;
    size_t off = size_t(static_cast<char*>(p) - base);
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + n == next->first) {
      n += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += n;
        return;
      }
    }
    free_[off] = n;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
};

// Arena of the context whose API call is running on this thread (null: the
// allocations go to hipMalloc).  Set for the duration of a call by ArenaScope.
thread_local std::shared_ptr<Arena> t_arena;
struct ArenaScope {
  std::shared_ptr<Arena> prev;
  explicit ArenaScope(const std::shared_ptr<Arena>& a) : prev(t_arena) { t_arena = a; }
  ~ArenaScope() { t_arena = prev; }
};

std::string oom_message() {
  if (t_arena)
    return "the bound workspace is exhausted (largest free block " + std::to_string(t_arena->largest_free()) +
           " bytes)";
  return "out of device memory";
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  std::shared_ptr<Arena> arena;      // set when the block came from a bound workspace
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes), arena(std::move(o.arena)) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      arena = std::move(o.arena);
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      if (arena) arena->give(p, bytes);
      else (void)hipFree(p);
    }
    p = nullptr;
    bytes = 0;
    arena.reset();
  }
  hipError_t alloc(size_t n) {
    release();
    if (n == 0) return hipSuccess;
    if (t_arena) {
      p = t_arena->take(n);
      if (!p) return hipErrorOutOfMemory;
      arena = t_arena;
      bytes = n;
      return hipSuccess;
    }
    hipError_t e = hipMalloc(&p, n);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

template <typename T>
hipError_t upload(DevBuf& b, const std::vector<T>& v) {
  hipError_t e = b.alloc(v.size() * sizeof(T));
  if (e != hipSuccess || v.empty()) return e;
  return hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
}

template <typename R>
std::vector<R> cast(const std::vector<double>& v) {
  return std::vector<R>(v.begin(), v.end());
}

// Shu-Osher coefficients (a_i, b_i, g_i, c_i): stage i computes
// w(i) = a_i w^n + b_i (w(i-1) + g_i dt L(w(i-1), t^n + c_i dt)).
struct RKTable {
  int n = 0;
  double a[MAX_STAGES], b[MAX_STAGES], g[MAX_STAGES], c[MAX_STAGES], w[MAX_STAGES];
};

bool make_rk(int stages, RKTable& T) {
  T.n = stages;
  if (stages == 2) {  // SSP(2,2)
    const double t[2][4] = {{0, 1, 1, 0}, {0.5, 0.5, 1, 1}};
    for (int i = 0; i < 2; ++i) { T.a[i] = t[i][0]; T.b[i] = t[i][1]; T.g[i] = t[i][2]; T.c[i] = t[i][3]; }
  } else if (stages == 3) {  // SSP(3,3)
    const double t[3][4] = {{0, 1, 1, 0}, {0.75, 0.25, 1, 1}, {1.0 / 3.0, 2.0 / 3.0, 1, 0.5}};
    for (int i = 0; i < 3; ++i) { T.a[i] = t[i][0]; T.b[i] = t[i][1]; T.g[i] = t[i][2]; T.c[i] = t[i][3]; }
  } else if (stages == 5) {  // SSP(5,2): four forward-Euler stages of dt/4, then the 1/5 - 4/5 blend
    for (int i = 0; i < 5; ++i) { T.a[i] = 0; T.b[i] = 1; T.g[i] = 0.25; T.c[i] = 0.25 * i; }
    T.a[4] = 0.2;
    T.b[4] = 0.8;
  } else {
    return false;
  }
  // weight of each stage's L in w^{n+1}: e_i = b_i (e_{i-1} + g_i delta_i)
  double e[MAX_STAGES] = {0, 0, 0, 0, 0};
  for (int i = 0; i < stages; ++i) {
    for (int j = 0; j < i; ++j) e[j] *= T.b[i];
    e[i] = T.b[i] * T.g[i];
  }
  for (int i = 0; i < stages; ++i) T.w[i] = e[i];
  return true;
}

struct MeshDev {
  HostMesh host;
  int real_size = 8, p = 1, limiter = 0;
  DevBuf ev, hbv, fric, din, lima, nbr, nk, tri, limc, nxy;
  // tile halos of the fused stage kernel (limiter on, p <= 2), when every
  // tile's rings fit its LDS slots
  bool halo_ok = false;
  DevBuf h_off, h_n1, h_id, h_nslot, h_eslot;
  size_t device_bytes() const {
    return ev.bytes + hbv.bytes + fric.bytes + din.bytes + lima.bytes + nbr.bytes + nk.bytes + tri.bytes +
           limc.bytes + nxy.bytes + h_off.bytes + h_n1.bytes + h_id.bytes + h_nslot.bytes + h_eslot.bytes;
  }
};

// value of Dubiner mode m at reference vertex k
inline double dg_vertex_basis(int k, int m) { return phi_(m, vr_(k), vs_(k)); }

enum KName { K_STAGE = 0, K_POST, K_RAIN, K_REDUCE, K_N };
const char* kname[K_N] = {"stage", "post", "rain", "reduce"};

struct Pending {
  int k;
  hipEvent_t a, b;
};

}  // namespace

struct dgswe_ctx {
  dgswe_params prm{};
  int rs = 8;                       // bytes per Real
  RKTable rk;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int device = 0;                   // HIP device current at creation
  std::shared_ptr<MeshDev> mesh;
  std::shared_ptr<Arena> arena;     // caller's device memory (dgswe_workspace_bind), or null
  int n_tiles = 0;
  int variant = 1;                  // stage kernel: 0 per element, 1 per edge, 2 per edge with matrix-core area terms
  int fused = 0;                    // limiter on, per-edge kernel: later stages post-process their input
  int tile = TILE;                  // elements per workgroup of the per-edge stage kernel (64, 128, 256, 512)
  int n_tiles64 = 0;
  // tiles of 64 elements {0, t}: its first ceil(E / T) entries list the
  // stage tiles of any size T
  DevBuf W[3], Wt, F[3], fullwet[2], R, part, sc, memb, tiles, tiles64, ids, rnode, met, node_tiles;
  int n_node_tiles = 0;
  DevBuf storm, gt, gvals, tide_c, riv_tq, wind;
  Forcing fo{};
  std::vector<double> tide_rows[MAX_SLOTS];
  double tide_mean[MAX_SLOTS] = {0};
  std::vector<double> riv_rows[MAX_SLOTS];
  bool have_state = false;
  bool in_batch = false;
  hipStream_t batch_stream = nullptr;   // stream of the batch this context belongs to
  // profiling
  int prof = 0;                     // 0 off, 1 every kernel, 2 stage kernel only
  std::vector<Pending> pending;
  std::vector<hipEvent_t> free_events;
  int64_t k_launches[K_N] = {0, 0, 0, 0};
  double k_ms[K_N] = {0, 0, 0, 0};
  // graph of one step
  hipGraphExec_t graph = nullptr;
  bool graph_dirty = true;

  ~dgswe_ctx() {
    if (graph) (void)hipGraphExecDestroy(graph);
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : free_events) (void)hipEventDestroy(e);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
  int E() const { return mesh ? int(mesh->host.E) : 0; }
  int NP() const { return prm.p == 1 ? 3 : prm.p == 2 ? 6 : 10; }
  // elements per workgroup of the stage kernel as launched: the chosen
  // tile for the per-edge kernel (512 only at p = 1), else 256
  int stage_tile() const {
    if (variant == 2) return 64;
    if (variant != 1 || (tile == 512 && prm.p != 1)) return TILE;
    return tile;
  }
  // the fused stage kernel runs: limiter on, per-edge kernel, a halo built,
  // 256-element tiles
  bool use_fused() const {
    return fused && variant == 1 && prm.limiter && mesh && mesh->halo_ok && stage_tile() == TILE;
  }
};

struct dgswe_batch {
  dgswe_params prm{};
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int64_t budget = 0;
  struct Slot {
    dgswe_ctx* ctx = nullptr;
    int64_t target = 0;
    bool live = false;
  };
  std::vector<Slot> slots;
  bool dirty = true;
  struct Group {
    int p, flux, limiter, variant, fused, tile;
    RKTable rk;
    std::vector<int> members;       // indices into the member array
    int n_tiles = 0, n_node_tiles = 0, max_chunks = 1, n_stage_tiles = 0;
    DevBuf tiles, node_tiles, ids, stage_tiles;   // stage_tiles: tiles of `tile` elements when not 256
    bool node_forcing = false;    // some member needs the per-step node kernel
  };
  std::vector<Group> groups;
  DevBuf memb;
  std::vector<int> member_slot;     // member index (as in memb) -> slot
  DevBuf flags;                     // [members] active flags gathered by dgswe_batch_poll
  int* flags_host = nullptr;        // pinned copy of flags
  size_t flags_cap = 0;
  hipGraphExec_t graph = nullptr;   // one step of every group, replayed
  bool graph_dirty = true;
  ~dgswe_batch() {
    if (stream) (void)hipStreamSynchronize(stream);
    if (graph) (void)hipGraphExecDestroy(graph);
    if (flags_host) (void)hipHostFree(flags_host);
    if (own_stream && stream) (void)hipStreamDestroy(stream);
  }
};

namespace {

// ------------------------------------------------------------ helpers
template <typename Real>
Member<Real> member_struct(const dgswe_ctx* c) {
  Member<Real> m{};
  const MeshDev* md = c->mesh.get();
  m.E = c->E();
  m.n_nodes = md ? int(md->host.n_nodes) : 0;
  m.n_tiles = c->n_tiles;
  m.friction = c->prm.friction;
  m.H0 = c->prm.H0;
  m.g = c->prm.g;
  m.cfl = c->prm.cfl;
  m.dt_fixed = c->prm.dt_fixed;
  m.dt_max = c->prm.dt_max;
  m.feps = 1e-3 * m.H0 * std::sqrt(m.g * m.H0);
  if (md) {
    m.ev = md->ev.as<Real>();
    m.hbv = md->hbv.as<Real>();
    m.fric = md->fric.as<Real>();
    m.nbr = md->nbr.as<int>();
    m.nk = md->nk.as<uint8_t>();
    m.din = md->din.as<Real>();
    m.tri = md->tri.as<int>();
    m.nxy = md->nxy.as<double>();
    m.lima = md->lima.as<Real>();
    m.limc = md->limc.as<uint8_t>();
  }
  for (int i = 0; i < 3; ++i) {
    m.W[i] = c->W[i].as<Real>();
    m.F[i] = c->F[i].as<uint8_t>();
  }
  m.Wt = c->Wt.as<Real>();
  m.fullwet[0] = c->fullwet[0].as<uint8_t>();
  m.fullwet[1] = c->fullwet[1].as<uint8_t>();
  if (md && md->halo_ok) {
    m.h_off = md->h_off.as<int>();
    m.h_n1 = md->h_n1.as<int>();
    m.h_id = md->h_id.as<int>();
    m.h_nslot = md->h_nslot.as<uint32_t>();
    m.h_eslot = md->h_eslot.as<uint32_t>();
  }
  m.R = c->R.as<Real>();
  m.rn = c->rnode.as<double>();
  m.met = c->met.as<Real>();
  m.part = c->part.as<double>();
  m.red = m.part ? m.part + size_t(NPART) * part_row(c->n_tiles) : nullptr;
  m.red_count = m.red ? reinterpret_cast<unsigned*>(m.red + size_t(NRED) * red_chunks(c->n_tiles)) : nullptr;
  m.sc = c->sc.as<Scalars>();
  m.fo = c->fo;
  return m;
}

int push_member(dgswe_ctx* c) {
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  if (c->rs == 8) {
    Member<double> m = member_struct<double>(c);
    HIPCHK(hipMemcpy(c->memb.p, &m, sizeof m, hipMemcpyHostToDevice));
  } else {
    Member<float> m = member_struct<float>(c);
    HIPCHK(hipMemcpy(c->memb.p, &m, sizeof m, hipMemcpyHostToDevice));
  }
  c->graph_dirty = true;
  return DGSWE_OK;
}

hipEvent_t get_event(dgswe_ctx* c) {
  if (!c->free_events.empty()) {
    hipEvent_t e = c->free_events.back();
    c->free_events.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

void harvest(dgswe_ctx* c) {
  for (auto& p : c->pending) {
    (void)hipEventSynchronize(p.b);
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      c->k_ms[p.k] += ms;
      c->k_launches[p.k] += 1;
    }
    c->free_events.push_back(p.a);
    c->free_events.push_back(p.b);
  }
  c->pending.clear();
}

// Timing of one launch while profiling is on.  With own = true the launcher
// hands a and b to the kernel's dispatch (start and end of the kernel
// itself); otherwise marker events are recorded around the launch.
struct ProfScope {
  dgswe_ctx* c;
  int k;
  bool own;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(dgswe_ctx* c_, int k_, bool own_ = false)
      : c((c_ && (c_->prof == 1 || (c_->prof == 2 && k_ == K_STAGE))) ? c_ : nullptr), k(k_), own(own_) {
    if (c) {
      a = get_event(c);
      if (own) b = get_event(c);
      else (void)hipEventRecord(a, c->stream);
    }
  }
  ~ProfScope() {
    if (c) {
      if (!own) {
        b = get_event(c);
        (void)hipEventRecord(b, c->stream);
      }
      c->pending.push_back({k, a, b});
      if (c->pending.size() > 4096) harvest(c);
    }
  }
};

RKInfo rk_info(const RKTable& T) {
  RKInfo r{};
  r.n = T.n;
  for (int i = 0; i < MAX_STAGES; ++i) {
    r.w[i] = i < T.n ? T.w[i] : 0.0;
    r.c[i] = i < T.n ? T.c[i] : 0.0;
  }
  return r;
}

// Buffers of stage i: in/out state and flag buffers (the last stage writes
// buffer 0 in place; intermediate stages alternate between 1 and 2).
StageArgs stage_args(const RKTable& T, int i) {
  StageArgs a{};
  a.stage = i;
  a.last = (i == T.n - 1);
  a.in_buf = (i == 0) ? 0 : 1 + ((i - 1) % 2);
  a.out_buf = a.last ? 0 : 1 + (i % 2);
  a.fin = a.in_buf;
  a.fout = a.out_buf;
  a.a = T.a[i];
  a.b = T.b[i];
  a.gam = T.g[i];
  return a;
}

// One time step of a set of members sharing (precision, p, flux, limiter,
// stages): nodal forcing, stages (+ post when limiting), reduce.
// part_over (single member only): the tile partials, chunk records and
// reduction counter at this address instead of the member's own arrays.
template <typename Real>
int enqueue_step_group(const Member<Real>* d_m, const Tile* d_t, int n_tiles, const Tile* d_nt, int n_node_tiles,
                       const int* d_ids, int n_members, int max_chunks, int p, int flux, int limiter, int variant,
                       const RKTable& T, bool node_forcing, hipStream_t s, dgswe_ctx* prof, bool single,
                       double* part_over = nullptr, bool fused = false, const Tile* d_ts = nullptr, int n_ts = 0,
                       int st_tile = TILE) {
  // stage launches over tiles of st_tile elements (list d_ts, n_ts of them)
  // when it is not 256
  const Tile* st_tiles = st_tile != TILE ? d_ts : d_t;
  const int st_n = st_tile != TILE ? n_ts : n_tiles;
  if (node_forcing) {
    ProfScope ps(prof, K_RAIN);
    // nodal rain rates, wind stress and pressure head at t^n; the first
    // stage averages the rain per element
    HIPCHK(launch_rain<Real>(d_m, d_t, 0, 0, d_nt, n_node_tiles, s, single ? 1 : 0));
  }
  for (int i = 0; i < T.n; ++i) {
    StageArgs a = stage_args(T, i);
    a.single = single ? 1 : 0;
    a.part = part_over;
    if (limiter) {
      // the stage writes its raw output to the stage's buffer; the post
      // pass limits it there, or (fused) the next stage does it for itself
      {
        ProfScope ps(prof, K_STAGE, true);
        HIPCHK(launch_stage<Real>(p, flux, 1, variant, d_m, st_tiles, st_n, a, s, ps.a, ps.b, fused && i > 0 ? 1 : 0,
                                  st_tile));
      }
      if (!fused || a.last) {
        ProfScope ps(prof, K_POST);
        HIPCHK(launch_post<Real>(p, 1, d_m, d_t, n_tiles, a, 0, s));
      }
    } else {
      ProfScope ps(prof, K_STAGE, true);
      HIPCHK(launch_stage<Real>(p, flux, 0, variant, d_m, st_tiles, st_n, a, s, ps.a, ps.b, 0, st_tile));
    }
  }
  ProfScope ps(prof, K_REDUCE);
  HIPCHK(launch_reduce<Real>(d_m, single ? nullptr : d_ids, n_members, max_chunks, 0, rk_info(T), s, part_over));
  return DGSWE_OK;
}

int ctx_enqueue_step(dgswe_ctx* c, double* part_over = nullptr) {
  const bool rain = c->fo.rain_kind != RAIN_CONST || c->fo.met_kind != MET_NONE;
  if (c->rs == 8)
    return enqueue_step_group<double>(c->memb.as<Member<double>>(), c->tiles.as<Tile>(), c->n_tiles,
                                      c->node_tiles.as<Tile>(), c->n_node_tiles, c->ids.as<int>(), 1, red_chunks(c->n_tiles),
                                      c->prm.p, c->prm.flux, c->prm.limiter, c->variant, c->rk, rain, c->stream, c, true,
                                      part_over, c->use_fused(), c->tiles64.as<Tile>(),
                                      (c->E() + c->stage_tile() - 1) / c->stage_tile(), c->stage_tile());
  return enqueue_step_group<float>(c->memb.as<Member<float>>(), c->tiles.as<Tile>(), c->n_tiles,
                                   c->node_tiles.as<Tile>(), c->n_node_tiles, c->ids.as<int>(), 1, red_chunks(c->n_tiles),
                                   c->prm.p, c->prm.flux, c->prm.limiter, c->variant, c->rk, rain, c->stream, c, true,
                                   part_over, c->use_fused(), c->tiles64.as<Tile>(),
                                   (c->E() + c->stage_tile() - 1) / c->stage_tile(), c->stage_tile());
}

// Doubles of a context's partials array: wavefront partials, the
// reduction's chunk records, then its counter.
size_t part_doubles(int n_tiles) {
  return size_t(NPART) * part_row(n_tiles) + size_t(NRED) * red_chunks(n_tiles) + 1;
}

// Set-up reduction (mode 1: dt from the state; mode 2: keep a dt > 0 that is
// already in the scalars).
int ctx_reduce_init(dgswe_ctx* c, int mode) {
  if (c->rs == 8)
    HIPCHK(launch_reduce<double>(c->memb.as<Member<double>>(), nullptr, 1, red_chunks(c->n_tiles), mode,
                                 rk_info(c->rk), c->stream));
  else
    HIPCHK(launch_reduce<float>(c->memb.as<Member<float>>(), nullptr, 1, red_chunks(c->n_tiles), mode,
                                rk_info(c->rk), c->stream));
  return DGSWE_OK;
}

// Message of a latched device error, naming the first element (caller's
// order) whose state became non-finite when there is one.
std::string nonfinite_message(const dgswe_ctx* c, const Scalars& s) {
  std::string m = "the state, the volume or the time step became non-finite";
  if (c->mesh && s.bad >= 0.0 && s.bad < double(c->mesh->host.E))
    m += " (first non-finite element: " + std::to_string(c->mesh->host.perm[int64_t(s.bad)]) + ")";
  return m;
}

int check_ctx(const dgswe_ctx* c, bool need_mesh = true, bool need_state = false) {
  if (!c) return fail(DGSWE_EINVAL, "null context");
  if (need_mesh && !c->mesh) return fail(DGSWE_ESTATE, "no mesh uploaded");
  if (need_state && !c->have_state) return fail(DGSWE_ESTATE, "no state set");
  return DGSWE_OK;
}

int read_scalars(dgswe_ctx* c, Scalars& s) {
  if (c->batch_stream) HIPCHK(hipStreamSynchronize(c->batch_stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(&s, c->sc.p, sizeof s, hipMemcpyDeviceToHost));
  return DGSWE_OK;
}

int write_scalars(dgswe_ctx* c, const Scalars& s) {
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(hipMemcpy(c->sc.p, &s, sizeof s, hipMemcpyHostToDevice));
  return DGSWE_OK;
}

int refresh_forcing(dgswe_ctx* c) {
  int rc = push_member(c);
  if (rc) return rc;
  if (!c->have_state) return DGSWE_OK;
  // the forcing of the coming step at the current t and dt
  rc = ctx_reduce_init(c, 2);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  return DGSWE_OK;
}

int upload_boundary_forcing(dgswe_ctx* c) {
  std::vector<double> tc, rq;
  c->fo.ocean_mask = 0;
  c->fo.river_mask = 0;
  for (int s = 0; s < MAX_SLOTS; ++s) {
    c->fo.tide_mean[s] = c->tide_mean[s];
    c->fo.tide_off[s] = int(tc.size() / 3);
    c->fo.tide_cnt[s] = int(c->tide_rows[s].size() / 3);
    tc.insert(tc.end(), c->tide_rows[s].begin(), c->tide_rows[s].end());
    c->fo.riv_off[s] = int(rq.size() / 2);
    c->fo.riv_cnt[s] = int(c->riv_rows[s].size() / 2);
    rq.insert(rq.end(), c->riv_rows[s].begin(), c->riv_rows[s].end());
  }
  for (int s = 0; s < MAX_SLOTS; ++s) {
    if (c->tide_mean[s] != 0.0 || !c->tide_rows[s].empty()) c->fo.ocean_mask |= 1u << s;
    if (!c->riv_rows[s].empty()) c->fo.river_mask |= 1u << s;
  }
  c->fo.n_tide = int(tc.size() / 3);
  c->fo.n_riv = int(rq.size() / 2);
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  if (tc.empty()) tc.push_back(0.0);
  if (rq.empty()) rq.push_back(0.0);
  HIPCHK(upload(c->tide_c, tc));
  HIPCHK(upload(c->riv_tq, rq));
  c->fo.tide_c = c->tide_c.as<double>();
  c->fo.riv_tq = c->riv_tq.as<double>();
  return refresh_forcing(c);
}

int alloc_state(dgswe_ctx* c) {
  const int64_t E = c->E();
  const size_t st = size_t(3) * c->NP() * E * c->rs;
  for (int i = 0; i < 3; ++i) {
    HIPCHK(c->W[i].alloc(st));
    HIPCHK(c->F[i].alloc(size_t(E)));
    if (E) HIPCHK(hipMemset(c->F[i].p, 0, size_t(E)));
  }
  HIPCHK(c->Wt.alloc(st));                     // the initial state, staged before its set-up pass
  if (c->prm.limiter) {
    // fully-wet bytes of a stage's raw output, two buffers: a fused stage
    // reads the previous stage's while it writes its own
    HIPCHK(c->fullwet[0].alloc(size_t(E)));
    HIPCHK(c->fullwet[1].alloc(size_t(E)));
  } else {
    c->fullwet[0].release();
    c->fullwet[1].release();
  }
  HIPCHK(c->R.alloc(size_t(E) * c->rs));
  if (E) HIPCHK(hipMemset(c->R.p, 0, size_t(E) * c->rs));
  const int64_t nn = c->mesh->host.n_nodes;
  HIPCHK(c->rnode.alloc(size_t(std::max<int64_t>(nn, 1)) * sizeof(double)));
  HIPCHK(hipMemset(c->rnode.p, 0, c->rnode.bytes));
  HIPCHK(c->met.alloc(size_t(3) * std::max<int64_t>(nn, 1) * c->rs));
  HIPCHK(hipMemset(c->met.p, 0, c->met.bytes));
  c->n_node_tiles = int((nn + TILE - 1) / TILE);
  std::vector<Tile> ntl(c->n_node_tiles);
  for (int t = 0; t < c->n_node_tiles; ++t) ntl[t] = {0, t};
  if (ntl.empty()) ntl.push_back({0, 0});
  HIPCHK(upload(c->node_tiles, ntl));
  c->n_tiles = int((E + TILE - 1) / TILE);
  // tile partials, then the reduction's chunk records, then its counter
  const size_t pb = part_doubles(c->n_tiles) * sizeof(double);
  HIPCHK(c->part.alloc(pb));
  HIPCHK(hipMemset(c->part.p, 0, pb));
  std::vector<Tile> tl(c->n_tiles);
  for (int t = 0; t < c->n_tiles; ++t) tl[t] = {0, t};
  if (tl.empty()) tl.push_back({0, 0});
  HIPCHK(upload(c->tiles, tl));
  // stage tiles of other sizes: prefixes of the 64-element list
  c->n_tiles64 = int((E + 63) / 64);
  std::vector<Tile> t64(std::max(c->n_tiles64, 1), Tile{0, 0});
  for (int t = 0; t < c->n_tiles64; ++t) t64[t] = {0, t};
  HIPCHK(upload(c->tiles64, t64));
  return push_member(c);
}

template <typename R>
int upload_mesh_arrays(MeshDev& md) {
  const HostMesh& h = md.host;
  HIPCHK(upload(md.ev, cast<R>(h.ev)));
  HIPCHK(upload(md.hbv, cast<R>(h.hbv)));
  HIPCHK(upload(md.fric, cast<R>(h.fric)));
  HIPCHK(upload(md.din, cast<R>(h.din)));
  HIPCHK(upload(md.nbr, h.nbr));
  HIPCHK(upload(md.nk, h.nk));
  HIPCHK(upload(md.tri, h.tri));
  HIPCHK(upload(md.nxy, h.xy));
  if (md.limiter) {
    HIPCHK(upload(md.lima, cast<R>(h.lima)));
    HIPCHK(upload(md.limc, h.limc));
  }
  md.halo_ok = false;
  if (md.limiter && md.p <= 2 && h.E > 0) {
    Halo H;
    std::string err;
    if (build_halo(h, TILE, H, err) == 0 && H.max_n1 <= HALO_R1 && H.max_n2 <= HALO_R2) {
      HIPCHK(upload(md.h_off, H.off));
      HIPCHK(upload(md.h_n1, H.n1));
      if (H.id.empty()) { H.id.push_back(0); H.nslot.push_back(0); }
      HIPCHK(upload(md.h_id, H.id));
      HIPCHK(upload(md.h_nslot, H.nslot));
      HIPCHK(upload(md.h_eslot, H.eslot));
      md.halo_ok = true;
    }
  }
  return DGSWE_OK;
}

// modal coefficients of the linear interpolant of vertex values (n0, n1, n2)
inline void modal_from_vertex(double n0, double n1, double n2, double* w) {
  w[0] = (n0 + n1 + n2) / 3.0;
  w[1] = (n1 - n0) / 2.0;
  w[2] = (2.0 * n2 - n0 - n1) / 6.0;
}

int upload_state(dgswe_ctx* c, const std::vector<double>& wint /* [3*NP][E] internal order */, DevBuf& dst) {
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->rs == 8) {
    if (!wint.empty()) HIPCHK(hipMemcpy(dst.p, wint.data(), wint.size() * 8, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(wint.begin(), wint.end());
    if (!f.empty()) HIPCHK(hipMemcpy(dst.p, f.data(), f.size() * 4, hipMemcpyHostToDevice));
  }
  return DGSWE_OK;
}

int reset_scalars(dgswe_ctx* c, double t) {
  Scalars s{};
  s.t = t;
  s.active = 1;
  s.target = std::numeric_limits<long long>::max();
  return write_scalars(c, s);
}

int post_initial(dgswe_ctx* c, int init) {
  StageArgs a{};
  const int p = c->prm.p;
  if (c->rs == 8) {
    auto* m = c->memb.as<Member<double>>();
    if (init == 1 && c->prm.limiter) HIPCHK(launch_classify<double>(p, m, c->tiles.as<Tile>(), c->n_tiles, c->stream));
    HIPCHK(launch_post<double>(p, init == 1 ? c->prm.limiter : 0, m, c->tiles.as<Tile>(), c->n_tiles, a, init, c->stream));
  } else {
    auto* m = c->memb.as<Member<float>>();
    if (init == 1 && c->prm.limiter) HIPCHK(launch_classify<float>(p, m, c->tiles.as<Tile>(), c->n_tiles, c->stream));
    HIPCHK(launch_post<float>(p, init == 1 ? c->prm.limiter : 0, m, c->tiles.as<Tile>(), c->n_tiles, a, init, c->stream));
  }
  int rc = ctx_reduce_init(c, init == 1 ? 1 : 2);
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(c->stream));
  c->have_state = true;
  c->graph_dirty = true;
  return DGSWE_OK;
}

// Device bytes of a context with its own mesh: every allocation of
// dgswe_create, dgswe_upload_mesh and the state, each rounded up to the
// 256-byte blocks of a bound workspace, as they are made (the forcing
// tables beyond one value per series, and the autotuner's copy, are not
// included).
int64_t footprint(const dgswe_params* p, int64_t E, int64_t n_nodes) {
  const int64_t rs = p->precision == DGSWE_FP32 ? 4 : 8;
  const int64_t NP = p->p == 1 ? 3 : p->p == 2 ? 6 : 10;
  const int64_t tiles = (E + TILE - 1) / TILE, node_tiles = (n_nodes + TILE - 1) / TILE;
  const int64_t nn = std::max<int64_t>(n_nodes, 1);
  auto blk = [](int64_t n) -> int64_t { return n <= 0 ? 0 : (n + 255) / 256 * 256; };
  const int64_t memb = int64_t(std::max(sizeof(Member<double>), sizeof(Member<float>)));
  // made with the context: scalars, member record, member id, one tide and
  // one river value
  int64_t b = blk(sizeof(Scalars)) + blk(memb) + blk(sizeof(int)) + 2 * blk(sizeof(double));
  // mesh: edge vectors, vertex bathymetry, friction, inscribed diameter,
  // neighbours, edge codes, node ids, node coordinates, limiter stencil
  b += blk(6 * E * rs) + blk(3 * E * rs) + blk(E * rs) + blk(E * rs) + blk(3 * E * 4) + blk(E) + blk(3 * E * 4) +
       blk(2 * n_nodes * 8);
  if (p->limiter) b += blk(6 * E * rs) + blk(E);
  // halos of the fused stage kernel (limiter on, p <= 2), at their largest
  if (p->limiter && p->p <= 2 && E > 0)
    b += blk((tiles + 1) * 4) + blk(tiles * 4) + 2 * blk(tiles * (HALO_R1 + HALO_R2) * 4) + blk(E * 4);
  // state: three buffers and the staged initial state, flags, fully-wet
  // bytes (two buffers), element rain, nodal rain, nodal wind and pressure,
  // tile lists, tile partials with the reduction's records and counter
  b += 4 * blk(3 * NP * E * rs) + 3 * blk(E) + (p->limiter ? 2 * blk(E) : 0) + blk(E * rs);
  b += blk(nn * 8) + blk(3 * nn * rs);
  b += blk(std::max<int64_t>(node_tiles, 1) * int64_t(sizeof(Tile))) + blk(std::max<int64_t>(tiles, 1) * int64_t(sizeof(Tile)));
  b += blk(std::max<int64_t>((E + 63) / 64, 1) * int64_t(sizeof(Tile)));        // 64-element tiles
  b += blk(int64_t(part_doubles(int(tiles))) * 8);
  return b;
}

}  // namespace

// ---------------------------------------------------- allocation-free step
// The partials, chunk records and counter of dgswe_step_noalloc live in one
// file-scope device array per GPU, held until the process ends.  In host
// code `scratch` names a host-side stand-in, never the device array: its
// device address is taken once per device with hipGetSymbolAddress (with
// that device current) and only that address is used.
constexpr size_t SCRATCH_BYTES = size_t(4) << 20;
static __device__ __align__(256) double scratch[SCRATCH_BYTES / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::map<int, double*> g_scratch_ptr;      // device id -> device address of scratch

// Device address of scratch on device dev (which must be current), taken on
// the first call for that device.  nullptr and a message on failure.
double* scratch_on(int dev, std::string& err) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it != g_scratch_ptr.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    return nullptr;
  }
  g_scratch_ptr[dev] = static_cast<double*>(ptr);
  return static_cast<double*>(ptr);
}
}  // namespace

// ======================================================================= API
extern "C" {

const char* dgswe_last_error(void) { return g_err.c_str(); }

int dgswe_default_params(dgswe_params* out) {
  if (!out) return fail(DGSWE_EINVAL, "null params");
  *out = dgswe_params{};
  out->p = 1;
  out->precision = DGSWE_FP64;
  out->flux = DGSWE_ROE;
  out->rk_stages = 2;
  out->limiter = 0;
  out->friction = DGSWE_MANNING;
  out->cfl = 0.3;
  out->dt_fixed = 0.0;
  out->dt_max = 1e30;
  out->H0 = 1e-3;
  out->g = 9.81;
  return DGSWE_OK;
}

static int check_params(const dgswe_params* p) {
  if (!p) return fail(DGSWE_EINVAL, "null params");
  if (p->p < 1 || p->p > 3) return fail(DGSWE_EINVAL, "p must be 1, 2 or 3");
  if (p->precision != DGSWE_FP32 && p->precision != DGSWE_FP64) return fail(DGSWE_EINVAL, "bad precision");
  if (p->flux != DGSWE_ROE && p->flux != DGSWE_LLF) return fail(DGSWE_EINVAL, "bad flux");
  if (p->rk_stages != 2 && p->rk_stages != 3 && p->rk_stages != 5) return fail(DGSWE_EINVAL, "rk_stages must be 2, 3 or 5");
  if (p->friction != DGSWE_MANNING && p->friction != DGSWE_QUADRATIC) return fail(DGSWE_EINVAL, "bad friction law");
  if (!(p->H0 > 0.0) || !(p->g > 0.0) || !std::isfinite(p->H0) || !std::isfinite(p->g))
    return fail(DGSWE_EINVAL, "H0 and g must be positive");
  if (!(p->dt_fixed > 0.0) && !(p->cfl > 0.0 && p->dt_max > 0.0)) return fail(DGSWE_EINVAL, "need dt_fixed > 0 or cfl, dt_max > 0");
  return DGSWE_OK;
}

int dgswe_create(const dgswe_params* params, void* hip_stream, dgswe_ctx** out) {
  if (!out) return fail(DGSWE_EINVAL, "null output pointer");
  *out = nullptr;
  int rc = check_params(params);
  if (rc) return rc;
  auto c = std::make_unique<dgswe_ctx>();
  c->prm = *params;
  HIPCHK(hipGetDevice(&c->device));
  c->rs = params->precision == DGSWE_FP32 ? 4 : 8;
  make_rk(params->rk_stages, c->rk);
  c->variant = 1;
  c->fused = 0;
  if (hip_stream) {
    c->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    HIPCHK(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    c->own_stream = true;
  }
  HIPCHK(c->sc.alloc(sizeof(Scalars)));
  HIPCHK(c->memb.alloc(std::max(sizeof(Member<double>), sizeof(Member<float>))));
  std::vector<int> ids{0};
  HIPCHK(upload(c->ids, ids));
  rc = reset_scalars(c.get(), 0.0);
  if (rc) return rc;
  c->fo.rain_kind = RAIN_CONST;
  rc = upload_boundary_forcing(c.get());
  if (rc) return rc;
  *out = c.release();
  return DGSWE_OK;
}

int dgswe_destroy(dgswe_ctx* c) {
  if (!c) return DGSWE_OK;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  delete c;
  return DGSWE_OK;
}

int dgswe_workspace_bind(dgswe_ctx* c, void* dev_ptr, size_t bytes) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (c->mesh) return fail(DGSWE_ESTATE, "bind the workspace before uploading or sharing a mesh");
  if (c->arena) return fail(DGSWE_ESTATE, "a workspace is already bound");
  if (!dev_ptr || reinterpret_cast<uintptr_t>(dev_ptr) % Arena::ALIGN != 0)
    return fail(DGSWE_EINVAL, "workspace must be a non-null device pointer aligned to 256 bytes");
  if (bytes < 65536) return fail(DGSWE_EINVAL, "workspace smaller than 64 KiB");
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, dev_ptr) != hipSuccess || at.type != hipMemoryTypeDevice) {
    (void)hipGetLastError();
    return fail(DGSWE_EINVAL, "workspace is not device memory");
  }
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  auto arena = std::make_shared<Arena>(dev_ptr, bytes);
  ArenaScope arena_scope(arena);
  // the buffers made at creation move into the workspace
  for (DevBuf* b : {&c->sc, &c->memb, &c->ids, &c->tide_c, &c->riv_tq, &c->storm, &c->wind, &c->gt, &c->gvals}) {
    if (!b->p) continue;
    DevBuf nb;
    HIPCHK(nb.alloc(b->bytes));
    HIPCHK(hipMemcpy(nb.p, b->p, b->bytes, hipMemcpyDeviceToDevice));
    *b = std::move(nb);
  }
  c->fo.tide_c = c->tide_c.as<double>();
  c->fo.riv_tq = c->riv_tq.as<double>();
  c->fo.storm = c->storm.as<double>();
  c->fo.wind = c->wind.as<double>();
  c->fo.gt = c->gt.as<double>();
  c->fo.gvals = c->gvals.as<float>();
  c->arena = arena;
  return push_member(c);
}

int dgswe_upload_mesh(dgswe_ctx* c, int64_t n_nodes, const double* xy, const double* hb, const double* fric,
                      int64_t n_tri, const int32_t* tri, int64_t n_bedges, const int32_t* bedge_nodes,
                      const int32_t* bedge_type, const int32_t* bedge_slot) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->mesh) return fail(DGSWE_ESTATE, "mesh already uploaded");
  if (n_bedges > 0 && !bedge_nodes) return fail(DGSWE_EINVAL, "null boundary edge array");
  {
    // the kernels address every array with 32-bit byte offsets: the largest
    // per-element array is the modal state (3 Np values per element), the
    // largest per-node one the storm forcing (3 values per node, at most 8
    // bytes each)
    const int64_t np = int64_t(c->prm.p + 1) * (c->prm.p + 2) / 2;
    const int64_t lim = int64_t(1) << 32;
    if (n_tri > 0 && 3 * np * n_tri * int64_t(c->rs) >= lim)
      return fail(DGSWE_EINVAL, "mesh too large for one context: the modal state array would exceed 4 GiB (" +
                                    std::to_string(lim / (3 * np * int64_t(c->rs))) + " triangles at most at this p and precision)");
    if (n_nodes > 0 && 3 * n_nodes * 8 >= lim)
      return fail(DGSWE_EINVAL, "mesh too large for one context: too many nodes for 32-bit array offsets");
  }
  auto md = std::make_shared<MeshDev>();
  std::string err;
  if (build_mesh(n_nodes, xy, hb, fric, n_tri, tri, n_bedges, bedge_nodes, bedge_type, bedge_slot, md->host, err))
    return fail(DGSWE_EINVAL, err);
  md->real_size = c->rs;
  md->p = c->prm.p;
  md->limiter = c->prm.limiter;
  rc = c->rs == 8 ? upload_mesh_arrays<double>(*md) : upload_mesh_arrays<float>(*md);
  if (rc) return rc;
  c->mesh = md;
  return alloc_state(c);
}

int dgswe_share_mesh(dgswe_ctx* dst, const dgswe_ctx* src) {
  int rc = check_ctx(dst, false);
  if (rc) return rc;
  rc = check_ctx(src, true);
  if (rc) return rc;
  ArenaScope arena_scope(dst->arena);
  if (dst->mesh) return fail(DGSWE_ESTATE, "mesh already uploaded");
  if (dst->rs != src->rs || dst->prm.p != src->prm.p || dst->prm.limiter != src->prm.limiter)
    return fail(DGSWE_EINVAL, "precision, p and limiter must match to share a mesh");
  dst->mesh = src->mesh;
  return alloc_state(dst);
}

int dgswe_set_initial_nodal(dgswe_ctx* c, const double* zeta, const double* qx, const double* qy) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  const HostMesh& h = c->mesh->host;
  const int64_t E = h.E, NP = c->NP();
  if (E > 0 && (!zeta || !qx || !qy)) return fail(DGSWE_EINVAL, "null state array");
  for (int64_t n = 0; n < h.n_nodes; ++n)
    if (!std::isfinite(zeta[n]) || !std::isfinite(qx[n]) || !std::isfinite(qy[n]))
      return fail(DGSWE_EINVAL, "non-finite initial value at node " + std::to_string(n));
  std::vector<double> w(size_t(3) * NP * E, 0.0);
  const double* src[3] = {zeta, qx, qy};
  for (int64_t i = 0; i < E; ++i) {
    const int n0 = h.tri[i], n1 = h.tri[E + i], n2 = h.tri[2 * E + i];
    for (int v = 0; v < 3; ++v) {
      double m[3];
      modal_from_vertex(src[v][n0], src[v][n1], src[v][n2], m);
      for (int k = 0; k < 3; ++k) w[(v * NP + k) * E + i] = m[k];
    }
  }
  rc = reset_scalars(c, 0.0);
  if (rc) return rc;
  rc = upload_state(c, w, c->Wt);
  if (rc) return rc;
  return post_initial(c, 1);
}

int dgswe_set_state(dgswe_ctx* c, int layout, const double* w, double t, const dgswe_mass* acc) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (layout != DGSWE_MODAL && layout != DGSWE_VERTEX) return fail(DGSWE_EINVAL, "bad layout");
  if (!std::isfinite(t)) return fail(DGSWE_EINVAL, "non-finite time");
  if (acc) {
    if (acc->t != t) return fail(DGSWE_EINVAL, "acc->t differs from t");
    if (!std::isfinite(acc->rain_in) || !std::isfinite(acc->bnd_in) || !std::isfinite(acc->bnd_out) ||
        !std::isfinite(acc->dt_last) || !std::isfinite(acc->dt_next) || acc->steps < 0)
      return fail(DGSWE_EINVAL, "non-finite or negative totals in acc");
  }
  const HostMesh& h = c->mesh->host;
  const int64_t E = h.E, NP = c->NP();
  if (E > 0 && !w) return fail(DGSWE_EINVAL, "null state array");
  std::vector<double> wi(size_t(3) * NP * E, 0.0);
  for (int64_t i = 0; i < E; ++i) {
    const int64_t e = h.perm[i];
    for (int v = 0; v < 3; ++v) {
      if (layout == DGSWE_MODAL) {
        for (int m = 0; m < NP; ++m) {
          const double x = w[(e * 3 + v) * NP + m];
          if (!std::isfinite(x)) return fail(DGSWE_EINVAL, "non-finite state value");
          wi[(v * NP + m) * E + i] = x;
        }
      } else {
        const double* n = w + (e * 3 + v) * 3;
        if (!std::isfinite(n[0]) || !std::isfinite(n[1]) || !std::isfinite(n[2]))
          return fail(DGSWE_EINVAL, "non-finite state value");
        double md[3];
        modal_from_vertex(n[0], n[1], n[2], md);
        for (int m = 0; m < 3; ++m) wi[(v * NP + m) * E + i] = md[m];
      }
    }
  }
  Scalars s{};
  s.t = t;
  s.active = 1;
  s.target = std::numeric_limits<long long>::max();
  if (acc) {
    // continue the budgets, the step count and the step size of the run
    s.rain_in = acc->rain_in;
    s.bnd_in = acc->bnd_in;
    s.bnd_out = acc->bnd_out;
    s.steps = acc->steps;
    s.dt_last = acc->dt_last;
    s.dt = acc->dt_next > 0.0 ? acc->dt_next : 0.0;
  }
  rc = write_scalars(c, s);
  if (rc) return rc;
  rc = upload_state(c, wi, c->W[0]);
  if (rc) return rc;
  return post_initial(c, 2);
}

int dgswe_set_rain_nodal(dgswe_ctx* c, const double* r) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  const HostMesh& h = c->mesh->host;
  if (h.n_nodes > 0 && !r) return fail(DGSWE_EINVAL, "null rain array");
  for (int64_t i = 0; i < h.n_nodes; ++i)
    if (!std::isfinite(r[i])) return fail(DGSWE_EINVAL, "non-finite rain rate");
  HIPCHK(hipStreamSynchronize(c->stream));
  if (h.n_nodes) HIPCHK(hipMemcpy(c->rnode.p, r, size_t(h.n_nodes) * sizeof(double), hipMemcpyHostToDevice));
  c->fo.rain_kind = RAIN_CONST;
  rc = push_member(c);
  if (rc) return rc;
  if (c->rs == 8)
    HIPCHK(launch_rain<double>(c->memb.as<Member<double>>(), c->tiles.as<Tile>(), c->n_tiles, 1, nullptr, 0, c->stream));
  else
    HIPCHK(launch_rain<float>(c->memb.as<Member<float>>(), c->tiles.as<Tile>(), c->n_tiles, 1, nullptr, 0, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  return refresh_forcing(c);
}

int dgswe_clear_rain(dgswe_ctx* c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  HIPCHK(hipStreamSynchronize(c->stream));
  if (c->R.bytes) HIPCHK(hipMemset(c->R.p, 0, c->R.bytes));
  HIPCHK(hipMemset(c->part.as<double>() + size_t(P_RAIN) * part_row(c->n_tiles), 0,
                   sizeof(double) * part_row(c->n_tiles)));
  c->fo.rain_kind = RAIN_CONST;
  return refresh_forcing(c);
}

int dgswe_set_rain_parametric(dgswe_ctx* c, int32_t n_rec, const double* rec) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  if (n_rec < 1 || !rec) return fail(DGSWE_EINVAL, "need at least one storm record");
  for (int i = 0; i < 7 * n_rec; ++i)
    if (!std::isfinite(rec[i])) return fail(DGSWE_EINVAL, "non-finite storm record");
  for (int i = 0; i < n_rec; ++i) {
    if (!(rec[7 * i + 5] > 0.0) || !(rec[7 * i + 6] > 0.0)) return fail(DGSWE_EINVAL, "r_m and r_e must be positive");
    if (i > 0 && !(rec[7 * i] > rec[7 * (i - 1)])) return fail(DGSWE_EINVAL, "storm record times must increase");
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(upload(c->storm, std::vector<double>(rec, rec + 7 * n_rec)));
  c->fo.rain_kind = RAIN_PARAM;
  c->fo.n_storm = n_rec;
  c->fo.storm = c->storm.as<double>();
  return refresh_forcing(c);
}

int dgswe_set_wind_vortex(dgswe_ctx* c, int32_t n_rec, const double* rec) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  if (n_rec < 1 || !rec) return fail(DGSWE_EINVAL, "need at least one wind record");
  for (int i = 0; i < 9 * n_rec; ++i)
    if (!std::isfinite(rec[i])) return fail(DGSWE_EINVAL, "non-finite wind record");
  for (int i = 0; i < n_rec; ++i) {
    const double* r = rec + 9 * i;
    if (!(r[3] >= 0.0)) return fail(DGSWE_EINVAL, "pressure deficit must be >= 0");
    if (!(r[4] > 0.0)) return fail(DGSWE_EINVAL, "radius of maximum wind must be positive");
    if (!(r[5] > 0.0 && r[5] <= 3.0)) return fail(DGSWE_EINVAL, "vortex shape B must be in (0, 3]");
    if (i > 0 && !(r[0] > rec[9 * (i - 1)])) return fail(DGSWE_EINVAL, "wind record times must increase");
  }
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(upload(c->wind, std::vector<double>(rec, rec + 9 * n_rec)));
  c->fo.met_kind = MET_VORTEX;
  c->fo.n_wind = n_rec;
  c->fo.wind = c->wind.as<double>();
  return refresh_forcing(c);
}

int dgswe_clear_wind(dgswe_ctx* c) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  HIPCHK(hipStreamSynchronize(c->stream));
  c->fo.met_kind = MET_NONE;
  c->fo.n_wind = 0;
  return refresh_forcing(c);
}

int dgswe_set_rain_gridded(dgswe_ctx* c, double x0, double y0, double dx, double dy, int32_t nx, int32_t ny,
                           int32_t n_rec, const double* t_rec, const float* vals) {
  int rc = check_ctx(c);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  if (nx < 2 || ny < 2 || n_rec < 1 || !t_rec || !vals) return fail(DGSWE_EINVAL, "lattice needs nx, ny >= 2 and a record");
  if (!(dx > 0.0) || !(dy > 0.0) || !std::isfinite(x0) || !std::isfinite(y0)) return fail(DGSWE_EINVAL, "bad lattice geometry");
  for (int i = 1; i < n_rec; ++i)
    if (!(t_rec[i] > t_rec[i - 1])) return fail(DGSWE_EINVAL, "record times must increase");
  const size_t nv = size_t(n_rec) * nx * ny;
  for (size_t i = 0; i < nv; ++i)
    if (!std::isfinite(vals[i])) return fail(DGSWE_EINVAL, "non-finite rain value");
  HIPCHK(hipStreamSynchronize(c->stream));
  HIPCHK(upload(c->gt, std::vector<double>(t_rec, t_rec + n_rec)));
  HIPCHK(upload(c->gvals, std::vector<float>(vals, vals + nv)));
  c->fo.rain_kind = RAIN_GRID;
  c->fo.gnx = nx;
  c->fo.gny = ny;
  c->fo.gnrec = n_rec;
  c->fo.gx0 = x0;
  c->fo.gy0 = y0;
  c->fo.gdx = dx;
  c->fo.gdy = dy;
  c->fo.gt = c->gt.as<double>();
  c->fo.gvals = c->gvals.as<float>();
  return refresh_forcing(c);
}

int dgswe_set_ocean_tide(dgswe_ctx* c, int32_t slot, double mean, int32_t n_const, const double* apt) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  if (slot < 0 || slot >= MAX_SLOTS) return fail(DGSWE_EINVAL, "slot out of range");
  if (n_const < 0 || (n_const > 0 && !apt)) return fail(DGSWE_EINVAL, "bad constituent array");
  if (!std::isfinite(mean)) return fail(DGSWE_EINVAL, "non-finite mean level");
  for (int i = 0; i < 3 * n_const; ++i)
    if (!std::isfinite(apt[i])) return fail(DGSWE_EINVAL, "non-finite constituent");
  for (int i = 0; i < n_const; ++i)
    if (apt[3 * i + 1] == 0.0) return fail(DGSWE_EINVAL, "zero tidal period");
  c->tide_mean[slot] = mean;
  c->tide_rows[slot].assign(apt, apt + 3 * n_const);
  return upload_boundary_forcing(c);
}

int dgswe_set_river_flux(dgswe_ctx* c, int32_t slot, int32_t n, const double* t, const double* q) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch; retire it first");
  if (slot < 0 || slot >= MAX_SLOTS) return fail(DGSWE_EINVAL, "slot out of range");
  if (n < 1 || !t || !q) return fail(DGSWE_EINVAL, "need at least one river sample");
  std::vector<double> rows;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(t[i]) || !std::isfinite(q[i])) return fail(DGSWE_EINVAL, "non-finite river sample");
    if (i > 0 && !(t[i] > t[i - 1])) return fail(DGSWE_EINVAL, "river sample times must increase");
    rows.push_back(t[i]);
    rows.push_back(q[i]);
  }
  c->riv_rows[slot] = rows;
  return upload_boundary_forcing(c);
}

static int build_graph(dgswe_ctx* c) {
  if (c->graph) {
    (void)hipGraphExecDestroy(c->graph);
    c->graph = nullptr;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
  const int prof = c->prof;
  c->prof = 0;
  int rc = ctx_enqueue_step(c);
  c->prof = prof;
  hipError_t e = hipStreamEndCapture(c->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(DGSWE_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&c->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(DGSWE_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  c->graph_dirty = false;
  return DGSWE_OK;
}

int dgswe_step_noalloc(dgswe_ctx* c, int64_t n) {
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (n < 0) return fail(DGSWE_EINVAL, "negative step count");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != c->device) return fail(DGSWE_ESTATE, "the context's device is not the current device");
  const size_t nd = part_doubles(c->n_tiles);
  if (nd * sizeof(double) > SCRATCH_BYTES) {
    int tmax = int(SCRATCH_BYTES / sizeof(double) / (NPART * PSLOT));
    while (tmax > 0 && part_doubles(tmax) * sizeof(double) > SCRATCH_BYTES) --tmax;
    return fail(DGSWE_EINVAL, "mesh too large for the static scratch: its partials need " +
                                  std::to_string(nd * sizeof(double)) + " bytes, the scratch holds " +
                                  std::to_string(SCRATCH_BYTES) + " (" + std::to_string(int64_t(tmax) * TILE) +
                                  " triangles at most)");
  }
  std::string err;
  double* const ptr = scratch_on(dev, err);
  if (!ptr) return fail(DGSWE_EHIP, err);
  const size_t row = part_row(c->n_tiles);
  // the array keeps the last call's contents: bring in what a step carries
  // over (the rain partial, written once for constant rain) and clear the
  // reduction counter, which must start at zero
  HIPCHK(hipMemcpyAsync(ptr + size_t(P_RAIN) * row, c->part.as<double>() + size_t(P_RAIN) * row,
                        sizeof(double) * row, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(launch_fill_zero(ptr + nd - 1, 1, c->stream));
  const int prof = c->prof;
  c->prof = 0;                             // no events: nothing is created
  for (int64_t i = 0; i < n && !rc; ++i) rc = ctx_enqueue_step(c, ptr);
  c->prof = prof;
  if (rc) return rc;
  // leave the context's own arrays as dgswe_step would (later set-up calls
  // read the last step's partials from them)
  HIPCHK(hipMemcpyAsync(c->part.p, ptr, nd * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return DGSWE_OK;
}

int dgswe_step(dgswe_ctx* c, int64_t n) {
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (n < 0) return fail(DGSWE_EINVAL, "negative step count");
  const bool use_graph = !c->prof && n >= 2;
  if (use_graph && c->graph_dirty) {
    rc = build_graph(c);
    if (rc) return rc;
  }
  for (int64_t i = 0; i < n; ++i) {
    if (use_graph) {
      HIPCHK(hipGraphLaunch(c->graph, c->stream));
    } else {
      rc = ctx_enqueue_step(c);
      if (rc) return rc;
    }
  }
  return DGSWE_OK;
}

int dgswe_sync(dgswe_ctx* c) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  Scalars s;
  rc = read_scalars(c, s);
  if (rc) return rc;
  if (s.error) return fail(DGSWE_ENONFINITE, nonfinite_message(c, s));
  return DGSWE_OK;
}

int dgswe_read_state(dgswe_ctx* c, int layout, double* out) {
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  if (layout != DGSWE_MODAL && layout != DGSWE_VERTEX) return fail(DGSWE_EINVAL, "bad layout");
  const HostMesh& h = c->mesh->host;
  const int64_t E = h.E, NP = c->NP();
  if (E > 0 && !out) return fail(DGSWE_EINVAL, "null output array");
  if (c->batch_stream) HIPCHK(hipStreamSynchronize(c->batch_stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<double> w(size_t(3) * NP * E);
  if (c->rs == 8) {
    if (E) HIPCHK(hipMemcpy(w.data(), c->W[0].p, w.size() * 8, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(w.size());
    if (E) HIPCHK(hipMemcpy(f.data(), c->W[0].p, f.size() * 4, hipMemcpyDeviceToHost));
    std::copy(f.begin(), f.end(), w.begin());
  }
  for (int64_t i = 0; i < E; ++i) {
    const int64_t e = h.perm[i];
    for (int v = 0; v < 3; ++v) {
      if (layout == DGSWE_MODAL) {
        for (int m = 0; m < NP; ++m) out[(e * 3 + v) * NP + m] = w[(v * NP + m) * E + i];
      } else {
        for (int k = 0; k < 3; ++k) {
          double s = 0.0;
          for (int m = 0; m < NP; ++m)
            s += dg_vertex_basis(k, m) * w[(v * NP + m) * E + i];
          out[(e * 3 + v) * 3 + k] = s;
        }
      }
    }
  }
  return DGSWE_OK;
}

int dgswe_read_flags(dgswe_ctx* c, uint8_t* out) {
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  const HostMesh& h = c->mesh->host;
  if (h.E > 0 && !out) return fail(DGSWE_EINVAL, "null output array");
  if (c->batch_stream) HIPCHK(hipStreamSynchronize(c->batch_stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  std::vector<uint8_t> f(h.E);
  if (h.E) HIPCHK(hipMemcpy(f.data(), c->F[0].p, h.E, hipMemcpyDeviceToHost));
  for (int64_t i = 0; i < h.E; ++i) out[h.perm[i]] = f[i] & 1;
  return DGSWE_OK;
}

int dgswe_mass_totals(dgswe_ctx* c, dgswe_mass* out) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (!out) return fail(DGSWE_EINVAL, "null output");
  if (c->prof) harvest(c);
  Scalars s;
  rc = read_scalars(c, s);
  if (rc) return rc;
  out->t = s.t;
  out->dt_last = s.dt_last;
  out->dt_next = s.dt;
  out->volume = s.volume;
  out->rain_in = s.rain_in;
  out->bnd_in = s.bnd_in;
  out->bnd_out = s.bnd_out;
  out->steps = s.steps;
  out->n_dry = s.n_dry;
  out->n_negative = s.n_neg;
  out->bad_element = -1;
  if (c->mesh && s.bad >= 0.0 && s.bad < double(c->mesh->host.E)) out->bad_element = c->mesh->host.perm[int64_t(s.bad)];
  if (s.error) return fail(DGSWE_ENONFINITE, nonfinite_message(c, s));
  return DGSWE_OK;
}

int dgswe_info(const dgswe_ctx* c, int64_t* n_tri, int64_t* n_nodes, int64_t* n_edges, int64_t* n_flipped) {
  int rc = check_ctx(c, true);
  if (rc) return rc;
  const HostMesh& h = c->mesh->host;
  if (n_tri) *n_tri = h.E;
  if (n_nodes) *n_nodes = h.n_nodes;
  if (n_edges) *n_edges = h.n_edges;
  if (n_flipped) *n_flipped = h.n_flipped;
  return DGSWE_OK;
}

int64_t dgswe_footprint_bytes(const dgswe_params* p, int64_t n_tri, int64_t n_nodes) {
  if (check_params(p)) return DGSWE_EINVAL;
  if (n_tri < 0 || n_nodes < 0) return fail(DGSWE_EINVAL, "negative size");
  return footprint(p, n_tri, n_nodes);
}

int dgswe_set_tuning(dgswe_ctx* c, int key, int value) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (key != DGSWE_TUNE_STAGE_VARIANT && key != DGSWE_TUNE_FUSED_POST && key != DGSWE_TUNE_STAGE_TILE)
    return fail(DGSWE_EINVAL, "unknown tuning key");
  if (key == DGSWE_TUNE_STAGE_TILE ? (value != 64 && value != 128 && value != TILE && value != 512)
      : key == DGSWE_TUNE_STAGE_VARIANT ? (value < 0 || value > 2) : (value != 0 && value != 1))
    return fail(DGSWE_EINVAL, "tuning values are 0 or 1 (stage variant: 0, 1, 2; stage tile: 64, 128, 256 or 512)");
  if (key == DGSWE_TUNE_STAGE_VARIANT && value == 2 && !(c->prm.p == 3 && c->prm.precision == DGSWE_FP32))
    return fail(DGSWE_EINVAL, "stage variant 2 (matrix-core area integrals) is built for p = 3 in FP32");
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  if (key == DGSWE_TUNE_STAGE_VARIANT) c->variant = value;
  else if (key == DGSWE_TUNE_FUSED_POST) c->fused = value;
  else c->tile = value;
  c->graph_dirty = true;
  return DGSWE_OK;
}

int dgswe_get_tuning(const dgswe_ctx* c, int key, int* value) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (!value || (key != DGSWE_TUNE_STAGE_VARIANT && key != DGSWE_TUNE_FUSED_POST && key != DGSWE_TUNE_STAGE_TILE))
    return fail(DGSWE_EINVAL, "unknown tuning key or null output");
  *value = key == DGSWE_TUNE_STAGE_VARIANT ? c->variant
           : key == DGSWE_TUNE_FUSED_POST  ? (c->use_fused() ? 1 : 0)
                                           : c->stage_tile();
  return DGSWE_OK;
}

int dgswe_autotune(dgswe_ctx* c, int n_steps, int* chosen, double* ms_per_step) {
  constexpr int NCFG = 7;
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  ArenaScope arena_scope(c->arena);
  if (c->in_batch) return fail(DGSWE_ESTATE, "context is a member of a batch");
  if (n_steps < 1) return fail(DGSWE_EINVAL, "autotune needs at least one timed step");
  Scalars s0;
  rc = read_scalars(c, s0);
  if (rc) return rc;
  if (s0.error) return fail(DGSWE_ENONFINITE, nonfinite_message(c, s0));
  // what a step carries over: the state, its flags, the tile partials (the
  // rain partial of constant rain is written once) and the scalars
  const size_t wb = c->W[0].bytes, fb = c->F[0].bytes, pb = c->part.bytes;
  DevBuf w0, f0, p0;
  HIPCHK(w0.alloc(wb));
  HIPCHK(f0.alloc(fb));
  HIPCHK(p0.alloc(pb));
  if (wb) HIPCHK(hipMemcpyAsync(w0.p, c->W[0].p, wb, hipMemcpyDeviceToDevice, c->stream));
  if (fb) HIPCHK(hipMemcpyAsync(f0.p, c->F[0].p, fb, hipMemcpyDeviceToDevice, c->stream));
  if (pb) HIPCHK(hipMemcpyAsync(p0.p, c->part.p, pb, hipMemcpyDeviceToDevice, c->stream));
  auto restore = [&]() -> int {
    if (wb) HIPCHK(hipMemcpyAsync(c->W[0].p, w0.p, wb, hipMemcpyDeviceToDevice, c->stream));
    if (fb) HIPCHK(hipMemcpyAsync(c->F[0].p, f0.p, fb, hipMemcpyDeviceToDevice, c->stream));
    if (pb) HIPCHK(hipMemcpyAsync(c->part.p, p0.p, pb, hipMemcpyDeviceToDevice, c->stream));
    HIPCHK(hipMemcpyAsync(c->sc.p, &s0, sizeof s0, hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return DGSWE_OK;
  };
  const int saved_prof = c->prof;
  const int saved_fused = c->fused, saved_tile = c->tile, saved_variant = c->variant;
  c->prof = 0;
  hipEvent_t ea, eb;
  HIPCHK(hipEventCreate(&ea));
  HIPCHK(hipEventCreate(&eb));
  // configurations: per-element kernel; per-edge kernel with the post pass
  // after every stage; per-edge kernel with the post-processing fused into
  // the next stage (limiter on, p <= 2, a halo built); per-edge kernel on
  // tiles of 512 (p = 1), 128 and 64 elements; per-edge kernel with the
  // area integrals on the matrix cores (p = 3, FP32)
  const int cfg_variant[NCFG] = {0, 1, 1, 1, 1, 1, 2}, cfg_fused[NCFG] = {0, 0, 1, 0, 0, 0, 0},
            cfg_tile[NCFG] = {TILE, TILE, TILE, 512, 128, 64, 64};
  double ms[NCFG] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const bool mf_ok = c->prm.p == 3 && c->prm.precision == DGSWE_FP32;
  int err = DGSWE_OK;
  for (int v = 0; v < NCFG && !err; ++v) {
    c->variant = cfg_variant[v];
    c->fused = cfg_fused[v];
    c->tile = cfg_tile[v];
    if (v == 2 && !c->use_fused()) continue;    // the same as configuration 1
    if (v == 6 && !mf_ok) continue;
    if (c->stage_tile() != cfg_tile[v]) continue;   // 512 at p > 1
    c->graph_dirty = true;
    err = dgswe_step(c, 2);                     // builds the step graph, warms caches
    if (!err) err = restore();
    if (err) break;
    if (hipEventRecord(ea, c->stream) != hipSuccess) { err = fail(DGSWE_EHIP, "hipEventRecord"); break; }
    err = dgswe_step(c, n_steps);
    if (err) break;
    if (hipEventRecord(eb, c->stream) != hipSuccess) { err = fail(DGSWE_EHIP, "hipEventRecord"); break; }
    if (hipEventSynchronize(eb) != hipSuccess) { err = fail(DGSWE_EHIP, "hipEventSynchronize"); break; }
    float f = 0.0f;
    (void)hipEventElapsedTime(&f, ea, eb);
    ms[v] = double(f) / n_steps;
    err = restore();
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  c->prof = saved_prof;
  if (err) {
    c->variant = saved_variant;
    c->fused = saved_fused;
    c->tile = saved_tile;
    (void)restore();
    return err;
  }
  int best = 0;
  for (int v = 1; v < NCFG; ++v)
    if (ms[v] > 0.0 && ms[v] <= ms[best]) best = v;
  c->variant = cfg_variant[best];
  c->fused = cfg_fused[best];
  c->tile = cfg_tile[best];
  c->graph_dirty = true;
  if (chosen) *chosen = c->variant;
  if (ms_per_step)
    for (int v = 0; v < NCFG; ++v) ms_per_step[v] = ms[v];
  return DGSWE_OK;
}

int dgswe_set_profiling(dgswe_ctx* c, int on) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (c->stream) HIPCHK(hipStreamSynchronize(c->stream));
  harvest(c);
  for (int k = 0; k < K_N; ++k) { c->k_launches[k] = 0; c->k_ms[k] = 0.0; }
  if (on < 0 || on > 2) return fail(DGSWE_EINVAL, "profiling mode must be 0, 1 or 2");
  c->prof = on;
  return DGSWE_OK;
}

int dgswe_kernel_stats(dgswe_ctx* c, const char* kernel, int64_t* launches, double* total_ms) {
  int rc = check_ctx(c, false);
  if (rc) return rc;
  if (!kernel) return fail(DGSWE_EINVAL, "null kernel name");
  harvest(c);
  for (int k = 0; k < K_N; ++k)
    if (std::strcmp(kernel, kname[k]) == 0) {
      if (launches) *launches = c->k_launches[k];
      if (total_ms) *total_ms = c->k_ms[k];
      return DGSWE_OK;
    }
  return fail(DGSWE_EINVAL, std::string("unknown kernel name ") + kernel);
}

}  // extern "C"

// ------------------------------------------------------------------ batches
namespace {

template <typename Real>
int batch_rebuild_t(dgswe_batch* b) {
  std::vector<Member<Real>> ms;
  std::map<std::tuple<int, int, int, int, int, int, int>, int> gi;
  b->groups.clear();
  b->member_slot.clear();
  for (size_t i = 0; i < b->slots.size(); ++i) {
    const auto& sl = b->slots[i];
    if (!sl.live) continue;
    const int idx = int(ms.size());
    ms.push_back(member_struct<Real>(sl.ctx));
    b->member_slot.push_back(int(i));
    const dgswe_params& p = sl.ctx->prm;
    auto key = std::make_tuple(p.p, p.flux, p.limiter, p.rk_stages, sl.ctx->variant, sl.ctx->use_fused() ? 1 : 0,
                               sl.ctx->stage_tile());
    auto it = gi.find(key);
    if (it == gi.end()) {
      dgswe_batch::Group g;
      g.p = p.p;
      g.flux = p.flux;
      g.limiter = p.limiter;
      g.variant = sl.ctx->variant;
      g.fused = sl.ctx->use_fused() ? 1 : 0;
      g.tile = sl.ctx->stage_tile();
      make_rk(p.rk_stages, g.rk);
      b->groups.push_back(std::move(g));
      it = gi.emplace(key, int(b->groups.size()) - 1).first;
    }
    b->groups[it->second].members.push_back(idx);
    if (sl.ctx->fo.rain_kind != RAIN_CONST || sl.ctx->fo.met_kind != MET_NONE)
      b->groups[it->second].node_forcing = true;
  }
  if (ms.empty()) ms.push_back(Member<Real>{});
  HIPCHK(upload(b->memb, ms));
  for (auto& g : b->groups) {
    std::vector<Tile> tl, ntl, ts;
    g.max_chunks = 1;
    for (int m : g.members) {
      const int nt = ms[m].n_tiles;
      g.max_chunks = std::max(g.max_chunks, red_chunks(nt));
      for (int t = 0; t < nt; ++t) tl.push_back({m, t});
      if (g.tile != TILE)
        for (int t = 0; t < (ms[m].E + g.tile - 1) / g.tile; ++t) ts.push_back({m, t});
      const int nnt = (ms[m].n_nodes + TILE - 1) / TILE;
      for (int t = 0; t < nnt; ++t) ntl.push_back({m, t});
    }
    g.n_tiles = int(tl.size());
    g.n_node_tiles = int(ntl.size());
    if (tl.empty()) tl.push_back({0, 0});
    if (ntl.empty()) ntl.push_back({0, 0});
    HIPCHK(upload(g.tiles, tl));
    HIPCHK(upload(g.node_tiles, ntl));
    HIPCHK(upload(g.ids, g.members));
    g.n_stage_tiles = int(ts.size());
    if (g.tile != TILE) {
      if (ts.empty()) ts.push_back({0, 0});
      HIPCHK(upload(g.stage_tiles, ts));
    }
  }
  b->dirty = false;
  return DGSWE_OK;
}

// New member tables (and so a new step graph) for the live slots.
int batch_rebuild(dgswe_batch* b) {
  HIPCHK(hipStreamSynchronize(b->stream));
  const int rc = b->prm.precision == DGSWE_FP32 ? batch_rebuild_t<float>(b) : batch_rebuild_t<double>(b);
  if (!rc) b->graph_dirty = true;
  return rc;
}

int64_t batch_footprint(const dgswe_batch* b) {
  int64_t f = 0;
  for (const auto& sl : b->slots)
    if (sl.live) f += footprint(&sl.ctx->prm, sl.ctx->E(), sl.ctx->mesh ? sl.ctx->mesh->host.n_nodes : 0);
  return f;
}

}  // namespace

extern "C" {

int dgswe_batch_create(const dgswe_params* params, void* hip_stream, int64_t budget_bytes, dgswe_batch** out) {
  if (!out) return fail(DGSWE_EINVAL, "null output pointer");
  *out = nullptr;
  int rc = check_params(params);
  if (rc) return rc;
  auto b = std::make_unique<dgswe_batch>();
  b->prm = *params;
  b->budget = budget_bytes;
  if (hip_stream) {
    b->stream = static_cast<hipStream_t>(hip_stream);
  } else {
    HIPCHK(hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking));
    b->own_stream = true;
  }
  *out = b.release();
  return DGSWE_OK;
}

int dgswe_batch_destroy(dgswe_batch* b) {
  if (!b) return DGSWE_OK;
  (void)hipStreamSynchronize(b->stream);
  for (auto& sl : b->slots)
    if (sl.live) {
      sl.ctx->in_batch = false;
      sl.ctx->batch_stream = nullptr;
    }
  delete b;
  return DGSWE_OK;
}

int dgswe_batch_add(dgswe_batch* b, dgswe_ctx* c, int64_t n_steps, int32_t* slot) {
  if (!b) return fail(DGSWE_EINVAL, "null batch");
  int rc = check_ctx(c, true, true);
  if (rc) return rc;
  if (c->in_batch) return fail(DGSWE_ESTATE, "context already belongs to a batch");
  if (n_steps < 0) return fail(DGSWE_EINVAL, "negative step count");
  if (c->prm.precision != b->prm.precision) return fail(DGSWE_EINVAL, "member precision differs from the batch");
  const int64_t need = footprint(&c->prm, c->E(), c->mesh->host.n_nodes);
  if (b->budget > 0 && batch_footprint(b) + need > b->budget)
    return fail(DGSWE_EBUDGET, "member footprint exceeds the remaining batch budget");
  Scalars s;
  rc = read_scalars(c, s);
  if (rc) return rc;
  if (s.error) return fail(DGSWE_ENONFINITE, "member has a latched error");
  s.target = s.steps + n_steps;
  s.active = n_steps > 0 ? 1 : 0;
  rc = write_scalars(c, s);
  if (rc) return rc;
  int id = -1;
  for (size_t i = 0; i < b->slots.size(); ++i)
    if (!b->slots[i].live) { id = int(i); break; }
  if (id < 0) {
    id = int(b->slots.size());
    b->slots.push_back({});
  }
  b->slots[id] = {c, s.target, true};
  c->in_batch = true;
  c->batch_stream = b->stream;
  b->dirty = true;
  if (slot) *slot = id;
  return DGSWE_OK;
}

static int batch_enqueue_step(dgswe_batch* b) {
  for (auto& g : b->groups) {
    int rc;
    if (b->prm.precision == DGSWE_FP32)
      rc = enqueue_step_group<float>(b->memb.as<Member<float>>(), g.tiles.as<Tile>(), g.n_tiles,
                                     g.node_tiles.as<Tile>(), g.n_node_tiles, g.ids.as<int>(),
                                     int(g.members.size()), g.max_chunks, g.p, g.flux, g.limiter, g.variant, g.rk,
                                     g.node_forcing, b->stream, nullptr, false, nullptr, g.fused != 0,
                                     g.stage_tiles.as<Tile>(), g.n_stage_tiles, g.tile);
    else
      rc = enqueue_step_group<double>(b->memb.as<Member<double>>(), g.tiles.as<Tile>(), g.n_tiles,
                                      g.node_tiles.as<Tile>(), g.n_node_tiles, g.ids.as<int>(),
                                      int(g.members.size()), g.max_chunks, g.p, g.flux, g.limiter, g.variant, g.rk,
                                      g.node_forcing, b->stream, nullptr, false, nullptr, g.fused != 0,
                                     g.stage_tiles.as<Tile>(), g.n_stage_tiles, g.tile);
    if (rc) return rc;
  }
  return DGSWE_OK;
}

// one step of every group captured once per membership and replayed
static int batch_build_graph(dgswe_batch* b) {
  if (b->graph) {
    (void)hipGraphExecDestroy(b->graph);
    b->graph = nullptr;
  }
  hipGraph_t g = nullptr;
  HIPCHK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  int rc = batch_enqueue_step(b);
  hipError_t e = hipStreamEndCapture(b->stream, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return fail(DGSWE_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(DGSWE_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  b->graph_dirty = false;
  return DGSWE_OK;
}

int dgswe_batch_step(dgswe_batch* b, int64_t max_steps) {
  if (!b) return fail(DGSWE_EINVAL, "null batch");
  if (max_steps < 0) return fail(DGSWE_EINVAL, "negative step count");
  if (b->dirty) {
    int rc = batch_rebuild(b);
    if (rc) return rc;
  }
  if (b->groups.empty()) return DGSWE_OK;
  const bool use_graph = max_steps >= 2;
  if (use_graph && b->graph_dirty) {
    int rc = batch_build_graph(b);
    if (rc) return rc;
  }
  for (int64_t i = 0; i < max_steps; ++i) {
    if (use_graph) {
      HIPCHK(hipGraphLaunch(b->graph, b->stream));
    } else {
      int rc = batch_enqueue_step(b);
      if (rc) return rc;
    }
  }
  return DGSWE_OK;
}

int dgswe_batch_poll(dgswe_batch* b, int32_t* done_slots, int32_t cap, int32_t* n_done) {
  if (!b || !n_done) return fail(DGSWE_EINVAL, "null argument");
  // the member table must list the live slots: rebuild it after a change
  if (b->dirty) {
    int rc = batch_rebuild(b);
    if (rc) return rc;
  }
  const size_t nm = b->member_slot.size();
  int32_t n = 0;
  if (nm > 0) {
    // every member's active flag in one small kernel and one copy
    if (nm > b->flags_cap) {
      if (b->flags_host) HIPCHK(hipHostFree(b->flags_host));
      b->flags_host = nullptr;
      b->flags_cap = 0;
      HIPCHK(b->flags.alloc(nm * sizeof(int)));
      HIPCHK(hipHostMalloc(reinterpret_cast<void**>(&b->flags_host), nm * sizeof(int), hipHostMallocDefault));
      b->flags_cap = nm;
    }
    if (b->prm.precision == DGSWE_FP32)
      HIPCHK(launch_active_flags<float>(b->memb.as<Member<float>>(), int(nm), b->flags.as<int>(), b->stream));
    else
      HIPCHK(launch_active_flags<double>(b->memb.as<Member<double>>(), int(nm), b->flags.as<int>(), b->stream));
    HIPCHK(hipMemcpyAsync(b->flags_host, b->flags.p, nm * sizeof(int), hipMemcpyDeviceToHost, b->stream));
  }
  HIPCHK(hipStreamSynchronize(b->stream));
  for (size_t m = 0; m < nm; ++m)
    if (!b->flags_host[m]) {
      if (done_slots && n < cap) done_slots[n] = int32_t(b->member_slot[m]);
      ++n;
    }
  *n_done = n;
  return DGSWE_OK;
}

int dgswe_batch_retire(dgswe_batch* b, int32_t slot) {
  if (!b) return fail(DGSWE_EINVAL, "null batch");
  if (slot < 0 || size_t(slot) >= b->slots.size() || !b->slots[slot].live) return fail(DGSWE_EINVAL, "no such slot");
  HIPCHK(hipStreamSynchronize(b->stream));
  dgswe_ctx* c = b->slots[slot].ctx;
  b->slots[slot] = {};
  c->in_batch = false;
  c->batch_stream = nullptr;
  Scalars s;
  int rc = read_scalars(c, s);
  if (rc) return rc;
  s.target = std::numeric_limits<long long>::max();
  s.active = s.error ? 0 : 1;
  rc = write_scalars(c, s);
  if (rc) return rc;
  b->dirty = true;
  return DGSWE_OK;
}

int dgswe_batch_read(dgswe_batch* b, int32_t slot, int layout, double* out, dgswe_mass* mass) {
  if (!b) return fail(DGSWE_EINVAL, "null batch");
  if (slot < 0 || size_t(slot) >= b->slots.size() || !b->slots[slot].live) return fail(DGSWE_EINVAL, "no such slot");
  dgswe_ctx* c = b->slots[slot].ctx;
  if (out) {
    const int rc = dgswe_read_state(c, layout, out);
    if (rc) return rc;
  }
  if (mass) return dgswe_mass_totals(c, mass);
  return DGSWE_OK;
}

int dgswe_batch_info(const dgswe_batch* b, int32_t* n_members, int64_t* fp) {
  if (!b) return fail(DGSWE_EINVAL, "null batch");
  int32_t n = 0;
  for (const auto& sl : b->slots) n += sl.live ? 1 : 0;
  if (n_members) *n_members = n;
  if (fp) *fp = batch_footprint(b);
  return DGSWE_OK;
}

}  // extern "C"
