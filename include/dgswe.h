/*
 * dgswe.h -- C ABI of the MI355X (gfx950) discontinuous Galerkin solver for
 * the rain-augmented shallow water equations.
 *
 * Model (Wichitrnithed et al., "A Discontinuous Galerkin Finite Element Model
 * for Compound Flood Simulations"):
 *   Sec. 2.1, Eq. SWE      d(zeta)/dt + div(H u) = R, momentum with bed slope
 *                          g zeta grad(hb) and bottom friction tau_b H u;
 *                          boundary partition ocean (specified elevation),
 *                          land (zero normal flow), river (Eq. river_bc:
 *                          specified normal flux in m^2/s).
 *   Sec. 2.2, Eq. elem_weak_form / Eq. dubiner / Eq. RKSSP
 *                          element weak form in an orthogonal Dubiner modal
 *                          basis (diagonal mass), SSP Runge-Kutta in time.
 *   Sec. 2.3               Roe or local Lax-Friedrichs flux, optional slope
 *                          limiter; Eq. rain: nodal rain averaged per element
 *                          and added in every element.
 *   Sec. 2.4               positive-depth operator (depth part, discharge
 *                          part) after every stage; wet/dry element flags.
 *   Sec. 2.5, Sec. 3.3     parametric storm rain and gridded rain lattices.
 *
 * Units are SI throughout: metres, seconds, m/s for rain, m^2/s for
 * discharge.  Bathymetry hb is positive downward, the free surface zeta
 * positive upward, the water depth is H = zeta + hb.
 *
 * Conventions shared by every call
 *   - Every function returns DGSWE_OK (0) or a negative DGSWE_E* code; the
 *     message of the last failure on the calling thread is returned by
 *     dgswe_last_error().  A failed call leaves the object as it was, except
 *     where stated.
 *   - Host arrays passed in are copied; the caller keeps ownership.  Host
 *     arrays passed out must be allocated by the caller with the documented
 *     size.  Device memory is owned by the context (or batch) and released by
 *     the matching destroy call.
 *   - dgswe_step / dgswe_batch_step enqueue work on the context's HIP stream
 *     and return without waiting; errors raised on the device (a non-finite
 *     volume) are latched and reported by dgswe_sync and every later call.
 *     Every read_* call and dgswe_mass_totals synchronise the stream.
 *   - A context is not thread-safe; distinct contexts may be used from
 *     distinct threads.
 */
#ifndef DGSWE_H
#define DGSWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ codes ---- */
#define DGSWE_OK          0
#define DGSWE_EINVAL     -1   /* bad argument, bad mesh, NaN input          */
#define DGSWE_ENOMEM     -2   /* device or host allocation failed           */
#define DGSWE_EHIP       -3   /* a HIP runtime call failed                  */
#define DGSWE_ESTATE     -4   /* call out of order (e.g. step before mesh)  */
#define DGSWE_ENONFINITE -5   /* latched: an element's state, the volume or
                                 the time step became NaN/Inf (the message
                                 and dgswe_mass.bad_element name the first
                                 element)                                   */
#define DGSWE_EBUDGET    -6   /* batch admission would exceed the budget    */

#define DGSWE_FP64 0          /* state, fluxes and reductions in FP64       */
#define DGSWE_FP32 1          /* state and fluxes in FP32; wet/dry tests,
                                 dt and mass/rain/boundary volumes in FP64  */

#define DGSWE_ROE 0           /* Roe flux (Sec. 3 default)                  */
#define DGSWE_LLF 1           /* local Lax-Friedrichs (Sec. 3.3)            */

#define DGSWE_MANNING   0     /* tau_b = g n^2 |u| / H^(4/3)               */
#define DGSWE_QUADRATIC 1     /* tau_b = C_f |u| / H                        */

#define DGSWE_LAND    0       /* zero normal flow: mirrored normal discharge */
#define DGSWE_OCEAN   1       /* specified elevation (tide of its slot)      */
#define DGSWE_RIVER   2       /* specified normal flux (series of its slot)  */
#define DGSWE_OUTFLOW 3       /* transmissive: ghost = interior state        */

#define DGSWE_MODAL  0        /* per element, per variable, per mode         */
#define DGSWE_VERTEX 1        /* per element, per variable, per vertex       */

#define DGSWE_MAX_SLOTS  16   /* forcing slots for ocean and river series    */

/* Solver settings (Sec. 2.3, Sec. 3).  p = 1 with rk_stages = 2 is the
 * paper's set-up; p = 2 needs rk_stages = 3 for linear stability;
 * rk_stages = 5 selects the optimal five-stage second-order SSP scheme. */
typedef struct dgswe_params {
  int32_t p;            /* polynomial degree: 1, 2 or 3                       */
  int32_t precision;    /* DGSWE_FP64 | DGSWE_FP32                            */
  int32_t flux;         /* DGSWE_ROE | DGSWE_LLF                              */
  int32_t rk_stages;    /* 2, 3 or 5                                          */
  int32_t limiter;      /* 0 = off, 1 = slope limiter on                      */
  int32_t friction;     /* DGSWE_MANNING | DGSWE_QUADRATIC                    */
  double  cfl;          /* dt = cfl * min_e d_e / lambda_e  (if dt_fixed <= 0) */
  double  dt_fixed;     /* > 0: fixed time step                               */
  double  dt_max;       /* upper bound of the CFL step                        */
  double  H0;           /* thin-layer depth of the positive-depth operator    */
  double  g;            /* gravity                                            */
} dgswe_params;

/* Time and mass bookkeeping (FP64 on the device). */
typedef struct dgswe_mass {
  double  t;            /* simulated time                                     */
  double  dt_last;      /* step just taken                                    */
  double  dt_next;      /* step that the next dgswe_step will take            */
  double  volume;       /* sum over elements of area * mean depth             */
  double  rain_in;      /* cumulative rain volume                             */
  double  bnd_in;       /* cumulative volume entering through the boundary    */
  double  bnd_out;      /* cumulative volume leaving through the boundary     */
  int64_t steps;        /* time steps taken                                   */
  int64_t n_dry;        /* elements flagged dry now                           */
  int64_t n_negative;   /* elements whose mean depth is negative now: the
                           positive-depth operator of Sec. 2.4 keeps each
                           element's water volume, so a negative mean is not
                           clamped; reported as a diagnostic (read only)     */
  int64_t bad_element;  /* caller's id of the first element whose mean depth
                           or wave speed became non-finite, -1 if none (read
                           only)                                            */
} dgswe_mass;

typedef struct dgswe_ctx dgswe_ctx;
typedef struct dgswe_batch dgswe_batch;

/* Fill *out with the defaults: p = 1, FP64, Roe, 2 stages, no limiter,
 * Manning, cfl 0.3, no fixed dt, dt_max 1e30, H0 1e-3, g 9.81. */
int dgswe_default_params(dgswe_params* out);

/* Create a solver context on the current HIP device.  hip_stream is a
 * hipStream_t to enqueue on (for example torch.cuda.current_stream()), or
 * NULL for a stream owned by the context.  EINVAL for unsupported settings. */
int dgswe_create(const dgswe_params* params, void* hip_stream, dgswe_ctx** out);
int dgswe_destroy(dgswe_ctx* ctx);

/* Hand the context device memory owned by the caller (for example the
 * storage of a torch tensor): from now on every device array of the context
 * (mesh arrays, states, flags, partials, forcing tables, the autotuner's
 * temporary copy) is placed in [dev_ptr, dev_ptr + bytes) by a first-fit
 * sub-allocator with 256-byte blocks, and the arrays made at creation move
 * there.  The library never frees dev_ptr; the caller keeps it valid until
 * the context, and every context that shares its mesh, is destroyed.
 * Sizing: dgswe_footprint_bytes(params, n_tri, n_nodes) bytes hold the
 * mesh, the state and everything made at creation; the forcing tables
 * (storm and wind records, rain lattice and its times, tide and river
 * series beyond one value each) need their own room, each rounded up to
 * 256 bytes, and so does dgswe_autotune (one more copy of the state, flags
 * and tile partials).  Must be called before
 * dgswe_upload_mesh / dgswe_share_mesh, once per context.  EINVAL for a null
 * or unaligned pointer, host memory or less than 64 KiB; ESTATE when a mesh
 * or a workspace is already there or the context is in a batch; a later
 * allocation that does not fit returns ENOMEM (nothing falls back to
 * hipMalloc).  Batches keep allocating their own small arrays. */
int dgswe_workspace_bind(dgswe_ctx* ctx, void* dev_ptr, size_t bytes);

/* Upload the mesh (Sec. 2.1 domain, Sec. 2.3 element-local operator).
 *   xy[2*n_nodes]            node coordinates (x0, y0, x1, y1, ...), m
 *   hb[n_nodes]              bathymetry, positive downward, m
 *   fric[n_nodes]            Manning n or quadratic C_f (element value =
 *                            mean of its three nodes)
 *   tri[3*n_tri]             0-based node ids; clockwise triangles are
 *                            reoriented (counted in dgswe_info)
 *   bedge_nodes[2*n_bedges]  node pairs of typed boundary edges
 *   bedge_type[n_bedges]     DGSWE_LAND/OCEAN/RIVER/OUTFLOW
 *   bedge_slot[n_bedges]     forcing slot (< DGSWE_MAX_SLOTS)
 * Boundary edges not listed are LAND.  EINVAL for node ids out of range,
 * zero-area triangles, edges shared by more than two triangles, listed
 * edges that are not on the boundary, bad types or slots, non-finite
 * coordinates, and for meshes too large for the kernels' 32-bit array
 * offsets: 3 Np n_tri bytes-per-value (the modal state) and 24 n_nodes must
 * stay below 2^32, i.e. at most 119M triangles at p = 1 in FP32, 59M in
 * FP64, 17.8M at p = 3 in FP64; an ensemble of separate contexts has no
 * such bound.  Elements are reordered along a Hilbert curve internally;
 * every array passed in or out uses the caller's element order.
 * Allowed once per context; n_tri = 0 is allowed (empty mesh). */
int dgswe_upload_mesh(dgswe_ctx* ctx, int64_t n_nodes, const double* xy, const double* hb,
                      const double* fric, int64_t n_tri, const int32_t* tri, int64_t n_bedges,
                      const int32_t* bedge_nodes, const int32_t* bedge_type,
                      const int32_t* bedge_slot);

/* Reuse the mesh already uploaded to src (read-only device arrays are
 * shared and kept alive while any context uses them).  Both contexts must
 * have the same precision, p and limiter setting. */
int dgswe_share_mesh(dgswe_ctx* dst, const dgswe_ctx* src);

/* Initial state from nodal values (zeta, qx, qy)[n_nodes]: each element
 * takes the linear interpolant of its vertices; the limiter (if on) and the
 * positive-depth operator are applied once (Sec. 2.4); t = 0 and the
 * budgets restart.  EINVAL on non-finite input. */
int dgswe_set_initial_nodal(dgswe_ctx* ctx, const double* zeta, const double* qx, const double* qy);

/* Set the state directly, for example to resume from a checkpoint taken
 * with dgswe_read_state and dgswe_mass_totals (Sec. 3.3 starts its storm run
 * from a tidal spin-up; Sec. 2.4 accounts for the water volume).
 *   layout DGSWE_MODAL:  w[n_tri][3][Np] with variables (zeta, qx, qy) and
 *                        Dubiner modes ordered (0,0),(1,0),(0,1),(2,0),
 *                        (1,1),(0,2),(3,0),(2,1),(1,2),(0,3) (Np = 3, 6, 10
 *                        for p = 1, 2, 3);
 *   layout DGSWE_VERTEX: w[n_tri][3][3], each variable's values at the three
 *                        vertices; the element takes their linear
 *                        interpolant (modes beyond the linear ones are zero).
 * The state is used as given (no limiter or positive-depth pass); flags, the
 * volume and (unless acc gives it) dt are derived from it.
 * acc == NULL: the budgets and the step count restart at time t.
 * acc != NULL: the run continues from these totals: rain_in, bnd_in, bnd_out,
 * steps, dt_last, and dt_next as the size of the next step (dt_next <= 0:
 * derived from the state); acc->t must equal t, the other fields are
 * ignored.  A state and totals read after step n and set again continue
 * bit for bit as the uninterrupted run.  EINVAL on non-finite input or a bad
 * layout; ESTATE inside a batch. */
int dgswe_set_state(dgswe_ctx* ctx, int layout, const double* w, double t, const dgswe_mass* acc);

/* Rain (Sec. 2.3 Eq. rain; Sec. 2.5; Sec. 3.3).  Each replaces the previous
 * rain source.  Like every forcing setter below, ESTATE while the context is
 * a member of a batch (retire it first).  Nodal rain r[n_nodes] (m/s) is held until replaced.
 * Parametric rain: rec[7*n_rec] rows (t, xc, yc, peak, T0, r_m, r_e) with
 * increasing t; parameters are interpolated linearly in time (held outside
 * the record span) and each node gets T0 + (peak - T0) r / r_m inside r_m
 * and peak exp(-(r - r_m)/r_e) outside, r its distance to (xc, yc).
 * Gridded rain: vals[n_rec][ny][nx] (m/s) on the lattice x0 + i dx,
 * y0 + j dy at times t_rec[n_rec]; bilinear in space (0 outside the
 * lattice), linear in time (held outside).  Rain is evaluated at the start
 * of each step and used for all its stages. */
int dgswe_set_rain_nodal(dgswe_ctx* ctx, const double* r);
int dgswe_set_rain_parametric(dgswe_ctx* ctx, int32_t n_rec, const double* rec);
int dgswe_set_rain_gridded(dgswe_ctx* ctx, double x0, double y0, double dx, double dy, int32_t nx,
                           int32_t ny, int32_t n_rec, const double* t_rec, const float* vals);
int dgswe_clear_rain(dgswe_ctx* ctx);

/* Wind stress and atmospheric pressure: the momentum sources F_x, F_y of
 * Sec. 2.1 (Eq. SWE) driven by a parametric storm, as Sec. 2.3 and Sec. 3.3
 * do with their hurricane wind and pressure model.  rec[9*n_rec] rows
 * (t, xc, yc, dp, rm, B, wf, wbx, wby) with increasing t, interpolated
 * linearly in time (held outside the record span): a symmetric vortex with
 * central pressure deficit dp >= 0 (Pa), radius of maximum wind rm > 0 (m)
 * and shape 0 < B <= 3, whose cyclostrophic wind
 * V = sqrt(B dp s exp(-s) / rho_a), s = (rm / r)^B, turns counter-clockwise
 * and is scaled by wf, plus a uniform background wind (wbx, wby) (m/s).
 * Pressure anomaly -dp (1 - exp(-s)).  Each node gets the kinematic stress
 * (rho_a / rho_w) C_d |W| W with C_d = min((0.75 + 0.067 |W|) 1e-3, 3.5e-3)
 * and the head psi = p_anomaly / (rho_w g) (rho_a = 1.15, rho_w = 1000
 * kg/m^3); inside an element both are linear and the momentum equations
 * take tau - g H grad psi at the area points.  Evaluated at the start of
 * each step and used for all its stages, like rain.  Replaces earlier
 * records; EINVAL on non-finite or out-of-range values.  dgswe_clear_wind
 * turns the forcing off. */
int dgswe_set_wind_vortex(dgswe_ctx* ctx, int32_t n_rec, const double* rec);
int dgswe_clear_wind(dgswe_ctx* ctx);

/* Ocean elevation of a slot (Sec. 2.1): mean + sum_k a_k sin(2 pi t/T_k +
 * phase_k), amp_period_phase[3*n_const].  River normal flux of a slot
 * (Eq. river_bc), outward positive, m^2/s, linear in time between samples
 * t[n], q[n] and held outside.  Both are evaluated at every stage time.
 * ESTATE while the context is a member of a batch. */
int dgswe_set_ocean_tide(dgswe_ctx* ctx, int32_t slot, double mean, int32_t n_const,
                         const double* amp_period_phase);
int dgswe_set_river_flux(dgswe_ctx* ctx, int32_t slot, int32_t n, const double* t, const double* q);

/* Advance n_steps time steps (asynchronous; see the conventions above). */
int dgswe_step(dgswe_ctx* ctx, int64_t n_steps);
/* The same steps as dgswe_step, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): nothing is allocated or freed, no graph is built and no
 * event is created; the steps are enqueued one launch at a time on the
 * context's stream.  The wavefront partials, reduction records and counter
 * that dgswe_step keeps in the context are placed in one static array of
 * 4 MiB per GPU instead, held until the process ends, which bounds the
 * mesh: EINVAL (with the limit in the message) above 2,094,848 triangles.  The
 * context's own arrays are updated at the end as after dgswe_step, so the
 * two calls can be mixed.  Calls that overlap on one GPU share the array
 * and race: keep them in one stream order.  ESTATE inside a batch or when
 * the context's device is not the current one; results are bit for bit
 * those of dgswe_step. */
int dgswe_step_noalloc(dgswe_ctx* ctx, int64_t n_steps);
/* Wait for queued work; returns the latched device error if any
 * (ENONFINITE, whose message names the first element whose state became
 * non-finite). */
int dgswe_sync(dgswe_ctx* ctx);

/* Read the state as FP64 in the caller's element order:
 * DGSWE_MODAL out[n_tri*3*Np], DGSWE_VERTEX out[n_tri*3*3]. */
int dgswe_read_state(dgswe_ctx* ctx, int layout, double* out);
/* Wet/dry flags (1 = dry) out[n_tri], caller's element order. */
int dgswe_read_flags(dgswe_ctx* ctx, uint8_t* out);
int dgswe_mass_totals(dgswe_ctx* ctx, dgswe_mass* out);

/* Mesh and bookkeeping sizes: any pointer may be NULL. */
int dgswe_info(const dgswe_ctx* ctx, int64_t* n_tri, int64_t* n_nodes, int64_t* n_edges,
               int64_t* n_flipped);
/* Device bytes of a context of this size with its own mesh: every array
 * made by dgswe_create, dgswe_upload_mesh and the state (mesh, three state
 * buffers and the staged initial state, flags, rain, nodal forcing, tile
 * lists and partials), each rounded up to 256 bytes; not the forcing tables
 * beyond one value per series.  A context that shares a mesh needs less.
 * Batch admission adds these numbers.  Returns DGSWE_EINVAL for bad
 * params or negative sizes. */
int64_t dgswe_footprint_bytes(const dgswe_params* params, int64_t n_tri, int64_t n_nodes);

/* Per-kernel timing with HIP events on the context's stream ("stage",
 * "post", "rain", "reduce").  The stage kernel's events are attached to its
 * own dispatch (start and end of the kernel itself); the others are marker
 * events recorded around the launch.  on: 0 = off (default; steps then
 * replay a HIP graph), 1 = every kernel, 2 = the stage kernel only (no
 * packets between launches).  Changing the mode resets the counters;
 * EINVAL for other values. */
int dgswe_set_profiling(dgswe_ctx* ctx, int on);
int dgswe_kernel_stats(dgswe_ctx* ctx, const char* kernel, int64_t* launches, double* total_ms);

/* Kernel choices (same arithmetic, different work layout; results differ
 * only by summation order).  DGSWE_TUNE_STAGE_VARIANT: 0 = every element
 * evaluates its three edges; 1 (default) = the tile's point values (p <= 2)
 * or edge traces (p = 3) are staged in LDS and each edge inside a tile is
 * evaluated once; 2 (p = 3, FP32 only, else EINVAL) = variant 1 on
 * 64-element tiles with the area integrals of Eq. elem_weak_form (modes to
 * the 16 area points, fluxes and sources back onto the 10 modes) computed
 * as 16x16x4 matrix products on the matrix cores.  DGSWE_TUNE_FUSED_POST (limiter on, variant 1, p <= 2):
 * 1 = every stage after the first applies the previous stage's limiter and
 * positive-depth operator (Sec. 2.3, Sec. 2.4) to its input itself, for its
 * tile and the ring of outside elements across the tile's edges, instead of
 * a separate pass over the whole state; 0 (default) = separate pass after
 * every stage.  The fused form needs a tile neighbourhood that fits the
 * kernel's LDS (built at upload; otherwise the key reads back 0).
 * DGSWE_TUNE_STAGE_TILE (variant 1): elements per workgroup of the
 * per-edge stage kernel, 64, 128, 256 (default) or, at p = 1, 512.  A
 * larger tile evaluates fewer cut edges twice; a smaller one lets more
 * independent workgroups share a CU, with fewer wavefronts waiting at each
 * barrier.  Results do not depend on it (partials are kept per wavefront).
 * It reads back 256 where it does not apply (variant 0, 512 at p > 1) and
 * 64 under variant 2; a tile other than 256 turns the fused form off.  dgswe_autotune times
 * every applicable choice.  EINVAL for unknown keys or values; ESTATE
 * while the context is in a batch. */
#define DGSWE_TUNE_STAGE_VARIANT 1
#define DGSWE_TUNE_FUSED_POST    2
#define DGSWE_TUNE_STAGE_TILE    3
int dgswe_set_tuning(dgswe_ctx* ctx, int key, int value);
int dgswe_get_tuning(const dgswe_ctx* ctx, int key, int* value);

/* Autotuner: times n_steps steps of this context in each configuration
 * (after two untimed steps each): per-element kernel, per-edge kernel with
 * a post pass after every stage, per-edge kernel with the post-processing
 * fused into the next stage (when available), per-edge kernel on tiles of
 * 512 (p = 1), 128 and 64 elements, stage variant 2 (p = 3, FP32); keeps
 * the fastest and restores the state, flags, partials and scalars, so the
 * context continues exactly where it was.  chosen (may be NULL) receives
 * the stage variant, ms_per_step[7] (may be NULL) the seven timings in that
 * order (0 where a configuration does not apply); the fused and tile
 * choices read back through dgswe_get_tuning.  Allocates a copy of the
 * state for the duration of the call.  EINVAL for n_steps < 1, ESTATE
 * without mesh or state or inside a batch, ENONFINITE if the context has a
 * latched error. */
int dgswe_autotune(dgswe_ctx* ctx, int n_steps, int* chosen, double* ms_per_step);

/* ---------------------------------------------------------------- batches
 * A batch advances many contexts (ensemble members or serving requests)
 * together: each stage is one launch over the element tiles of every active
 * member with the same (precision, p, flux, limiter, stages).  Members keep
 * their own dt, forcing and budgets; each member's result is bitwise the
 * same as when it runs alone.  The batch references (does not own) its
 * member contexts; a member must stay alive until it is retired. */
/* budget_bytes: admission limit on the summed dgswe_footprint_bytes of the
 * members (<= 0: no limit).  The params fix the precision of the batch. */
int dgswe_batch_create(const dgswe_params* params, void* hip_stream, int64_t budget_bytes,
                       dgswe_batch** out);
int dgswe_batch_destroy(dgswe_batch* b);
/* Add an initialised member that should run n_steps more steps.  *slot
 * receives its slot id.  EBUDGET if the footprint does not fit, EINVAL if
 * its precision differs from the batch. */
int dgswe_batch_add(dgswe_batch* b, dgswe_ctx* member, int64_t n_steps, int32_t* slot);
/* Advance every active member by up to max_steps steps (asynchronous). */
int dgswe_batch_step(dgswe_batch* b, int64_t max_steps);
/* Synchronise, then report members that reached their step count:
 * done_slots[cap] receives up to cap slot ids, *n_done their number. */
int dgswe_batch_poll(dgswe_batch* b, int32_t* done_slots, int32_t cap, int32_t* n_done);
/* Remove a member (done or not); its context stays valid. */
int dgswe_batch_retire(dgswe_batch* b, int32_t slot);
/* Synchronous read of a live member by slot: its state as dgswe_read_state
 * (layout, out; skipped when out is NULL) and its totals as
 * dgswe_mass_totals (skipped when mass is NULL), after the batch's queued
 * work.  EINVAL for an unknown slot or layout. */
int dgswe_batch_read(dgswe_batch* b, int32_t slot, int layout, double* out, dgswe_mass* mass);
/* Number of members, summed footprint. Either pointer may be NULL. */
int dgswe_batch_info(const dgswe_batch* b, int32_t* n_members, int64_t* footprint);

/* Bandwidth probe (measurement aid, not part of a step): a streaming
 * kernel that reads n_read arrays (1 to 3) and writes one, each `bytes`
 * long (>= 4096), reps times after one untimed launch, on the current
 * device; *gbs receives (n_read + 1) * bytes * reps / time in GB/s (1e9
 * bytes/s), timed with HIP events.  With n_read = 3 it has the stage
 * kernel's read:write mix, so its rate is the ceiling that kernel's HBM
 * rate is measured against beside the published peak.  Allocates and frees
 * its own arrays.  Returns EINVAL, ENOMEM or EHIP (no message is kept). */
int dgswe_stream_probe(int32_t n_read, int64_t bytes, int32_t reps, double* gbs);

/* Message of the last failed call on this thread ("" if none). */
const char* dgswe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DGSWE_H */
