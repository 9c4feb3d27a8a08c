#!/usr/bin/env python3
"""Benchmark: DG element-stage updates/s on the single-basin workload.

Workload (synthetic, seeded): 1,002,528-triangle jittered basin over
200 km x 200 km (708 x 708 quads cut along the shorter diagonal), -3000 m
ocean rising through a tanh shelf to +20 m land with 32 Gaussian bumps and
a dry land strip, ocean boundary at x = 0, parametric rain (peak 50 mm/h,
r_m 30 km, r_e 100 km, moving east at 5 m/s), p = 1, LLF flux, slope
limiter on, Manning 0.025, thin layer H0 = 0.05 m, SSP-RK2 at CFL 0.3.

One step = rain evaluation + 2 x (stage kernel + limiter/positive-depth
kernel) + the FP64 dt/budget reduction.  value = elements x stages x steps /
wall time of the timed steps (inputs resident in HBM), reported for the FP32
path (FP32 state and fluxes; FP64 wet/dry tests, dt and budgets); the FP64
path is reported beside it.  The dominant kernel's roofline uses the
algorithmic bytes of :func:`algorithmic_bytes` and its mean duration from
HIP events recorded by the library on its stream around every launch of
that kernel inside the timed region.  Then the 64-member FP32 ensemble and
the request loop (see :func:`run_ensemble`, :func:`run_serving`) and the
oracle on one host core.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "DG element-stage updates/s (FP64 vs FP32-batched); p50/p99 scenario latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def algorithmic_bytes(kernel, E, rs, p, a_nonzero, last, limiter, fused=False):
    """Bytes one launch must move from/to HBM (each array streamed once;
    neighbour gathers are cache traffic and not counted).

    stage: own state 3 Np rs, w^n 3 Np rs when the stage blends it, edge
           vectors 6 rs, vertex bathymetry 3 rs, friction rs, rain rs,
           neighbour ids 12, edge codes 1, flag 1; writes the new state
           3 Np rs and one flag byte; the last stage without limiter also
           reads d_in (rs).  A fused stage (it post-processes its input)
           also reads the limiter weights 6 rs, code 1 and wet byte 1, its
           neighbour slots 4 and the tile's halo lists (about 0.5 entries
           of 8 bytes per element), and reads no flag.
    post:  reads the unlimited state 3 Np rs, bathymetry 3 rs, neighbour
           ids 12, limiter weights 6 rs and code 1, wet byte 1; writes the
           state 3 Np rs and a flag; the last stage reads edge vectors and
           d_in (7 rs) for the volume and dt partials.
    """
    Np = (p + 1) * (p + 2) // 2
    st = 3 * Np * rs
    if kernel == "stage":
        b = st + (st if a_nonzero else 0) + 11 * rs + 14 + st + 1
        if last and not limiter:
            b += rs
        if fused:
            b += 6 * rs + 1 + 1 + 4 + 4 - 1
    else:
        b = st + 3 * rs + 12 + 6 * rs + 1 + 1 + st + 1 + (7 * rs if last else 0)
    return E * b


def step_bytes(E, n_nodes, rs, p, stages, limiter, fused, node_forcing=True):
    """Algorithmic bytes of one whole step (every launch): the stages (the
    first blends no w^n for the SSP schemes used), the post passes (after
    the last stage only when fused, else after every stage, when the limiter
    is on), the nodal forcing pass (16 B read and 8 B written per node) and
    the reduction (13 doubles per tile)."""
    b = 0
    for i in range(stages):
        last = i == stages - 1
        b += algorithmic_bytes("stage", E, rs, p, i > 0, last, limiter, fused and i > 0)
        if limiter and (last or not fused):
            b += algorithmic_bytes("post", E, rs, p, False, last, limiter)
    if node_forcing:
        b += 24 * n_nodes
    b += 13 * 8 * ((E + 255) // 256)
    return b


def run_precision(sc, precision, steps, warmup, variant=1, events=2, save_dir=None, fused=-1, tile=-1,
                  save_name="basin"):
    from paper_2307_14302_amd import Solver
    import torch

    t0 = time.perf_counter()
    s = Solver.from_scenario(sc, precision=precision)
    tuned = None
    if variant < 0:
        # the library's autotuner picks the stage kernel on this mesh (the
        # state is restored, so the run is the same as without it)
        variant, tuned = s.autotune(5)
    else:
        s.set_variant(variant)
    if fused >= 0:
        s.set_fused(fused)
    if tile > 0:
        s.set_tile(tile)
    fused, tile = s.fused(), s.tile()
    log(f"[{precision}] setup {time.perf_counter() - t0:.1f}s  E={s.n_tri}  stage variant {variant} fused {fused} "
        f"tile {tile}"
        + (f" (autotuned ms/step: per-element {tuned[0]:.3f}, per-edge {tuned[1]:.3f}, fused {tuned[2]:.3f}, "
           f"tiles 512/128/64 {tuned[3]:.3f}/{tuned[4]:.3f}/{tuned[5]:.3f}, matrix-core area {tuned[6]:.3f})"
           if tuned else ""))
    s.step(warmup)
    s.sync()
    # events on the stage kernel's own dispatches only: the dominant
    # kernel's duration for the roofline, with no packets between launches
    s.profiling(events)
    torch.cuda.synchronize()
    s.sync()
    t0 = time.perf_counter()
    s.step(steps)
    s.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    m = s.mass()
    stats = {k: s.kernel_stats(k) for k in ("stage", "post", "rain", "reduce")}
    s.profiling(False)
    E = s.n_tri
    stages = int(sc.params.get("rk_stages", 2))
    rate = E * stages * steps / el
    log(f"[{precision}] {steps} steps in {el:.3f}s -> {rate:.4e} element-stage/s; t={m['t']:.2f}s dt={m['dt_last']:.4f} "
        f"dry={m['n_dry']} kernels " + ", ".join(f"{k}:{n}x{(ms / max(n, 1)) * 1e3:.1f}us" for k, (n, ms) in stats.items()))
    graph = None
    if events:
        # the same workload continued without per-launch events, so that the
        # step replays one captured graph (the production path): reported
        # beside the timed region above, never as its value
        gsteps = min(steps, 2000)
        s.step(2)
        s.sync()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.step(gsteps)
        s.sync()
        torch.cuda.synchronize()
        gel = time.perf_counter() - t1
        graph = {"value": round(E * stages * gsteps / gel, 1), "ms_per_step": round(gel / gsteps * 1e3, 4),
                 "steps": gsteps}
        log(f"[{precision}] graph replay: {gsteps} steps in {gel:.3f}s -> {E * stages * gsteps / gel:.4e} element-stage/s")
    if save_dir:
        # the state after the run and after one more step, for the oracle's
        # one-step comparison in the CPU leg
        save_one_step(s, save_dir, f"{save_name}_{precision}")
    n_nodes = s.n_nodes
    s.close()
    return dict(rate=rate, elapsed=el, stats=stats, mass=m, E=E, stages=stages, variant=variant, graph=graph,
                fused=fused, tile=tile, tuned=tuned, steps=steps, n_nodes=n_nodes)


def save_one_step(s, save_dir, name):
    """A solver's state, time and next dt, then its state after one more
    step: the oracle's one-step comparison in the CPU leg starts from the
    first and is compared with the second."""
    m0 = s.mass()
    np.save(os.path.join(save_dir, f"{name}_w0.npy"), s.state())
    with open(os.path.join(save_dir, f"{name}_m0.json"), "w") as f:
        json.dump({"t": m0["t"], "dt_next": m0["dt_next"]}, f)
    s.step(1)
    np.save(os.path.join(save_dir, f"{name}_w1.npy"), s.state())


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "device_common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2307_14302_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


COUNTER_SUMMARIES = {"basin1M_p1": "stage_edge_kernel_basin1M_counters.md",
                     "graded3.6M_p1": "graded_coast3.6M_counters.md"}


def counted_traffic(kernel, precision, variant=1, tile=256, workload=None):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary of ``workload`` (FETCH_SIZE and WRITE_SIZE scaled by the copy
    calibration), or None when no summary covers this workload and kernel
    configuration or the kernel sources changed since it was taken.
    Summaries: the 1M-triangle p = 1 basin ("basin1M_p1") and the
    3.6M-triangle graded coast ("graded3.6M_p1")."""
    if workload not in COUNTER_SUMMARIES:
        return None
    path = os.path.join(ROOT, "profiles", COUNTER_SUMMARIES[workload])
    try:
        with open(path) as f:
            line = next(l for l in f if l.startswith("traffic-json:"))
        d = json.loads(line.split(":", 1)[1])
    except (OSError, StopIteration, ValueError):
        return None
    if d.get("sources") != kernel_sources_hash():
        return None
    if kernel == "stage":
        name = f"stage_edge_kernel/t{tile}" if variant == 1 else "stage_kernel"
    else:
        name = "post_kernel"
    return d["bytes"].get(f"{name}/{precision}")


def calib_copy():
    """A plain 1 GiB device copy, three times: the known byte count that the
    FETCH_SIZE and WRITE_SIZE counters are scaled by."""
    import torch
    a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    log("calibration copy: 3 x 1 GiB read + 1 GiB written")


def stream_ceiling():
    """Rate of the library's streaming probe (three arrays read, one written,
    the stage kernel's read:write mix): with 512 MiB arrays (HBM-resident)
    and with 32 MiB arrays (the four fit the 256 MB Infinity Cache)."""
    import ctypes as C
    from paper_2307_14302_amd import _native as N
    out = {}
    for label, nbytes in (("hbm_4x512MiB", 512 << 20), ("mall_4x32MiB", 32 << 20)):
        g = C.c_double()
        rc = N.lib.dgswe_stream_probe(3, nbytes, 20, C.byref(g))
        out[label] = round(g.value, 1) if rc == 0 else None
    log(f"stream probe (3 read : 1 write): {out} GB/s")
    return out


def roofline(res, precision, p, limiter, workload=None):
    rs = 4 if precision == "fp32" else 8
    stats = res["stats"]
    dom = max(("stage", "post"), key=lambda k: stats[k][1])
    n, ms = stats[dom]
    if n == 0:
        return None
    # SSP(2,2): stage 0 does not blend w^n, stage 1 does and is the last;
    # SSP(3,3): stages 1 and 2 blend, stage 2 is the last
    ns = res["stages"]
    fused = bool(res.get("fused"))
    per_launch = [algorithmic_bytes(dom, res["E"], rs, p, i > 0, i == ns - 1, limiter, fused and i > 0)
                  for i in range(ns)]
    byts = sum(per_launch) / len(per_launch)
    avg_s = ms / n * 1e-3
    ach = byts / avg_s / 1e9
    traffic = counted_traffic(dom, precision, res.get("variant", 1), res.get("tile", 256), workload)
    out = {"kernel": dom, "bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_source": ("FETCH_SIZE and WRITE_SIZE per launch from the committed rocprofv3 summary "
                              f"profiles/{COUNTER_SUMMARIES[workload]} (same kernel sources), scaled by "
                              "its copy calibration; not counted in this run") if traffic else
                             ("null: the committed counter summary has no figure for this kernel, stage tile and "
                              "precision, or the kernel sources changed since it was taken"
                              if workload in COUNTER_SUMMARIES else
                              "null: no committed counter summary for this workload"),
           "bytes_per_launch": int(byts),
           "avg_us": round(avg_s * 1e6, 2), "launches": n}
    # the whole step against the same peak: every launch's algorithmic bytes
    # over the measured time per step
    sb = step_bytes(res["E"], res.get("n_nodes", 0), rs, p, ns, limiter, fused)
    step_s = res["elapsed"] / res["steps"]
    out["step"] = {"bytes": int(sb), "ms": round(step_s * 1e3, 4), "achieved": round(sb / step_s / 1e9, 1),
                   "frac": round(sb / step_s / 1e9 / HBM_PEAK_GBS, 4)}
    if res.get("graph"):
        gs = res["graph"]["ms_per_step"] * 1e-3
        out["step"]["graph_replay_frac"] = round(sb / gs / 1e9 / HBM_PEAK_GBS, 4)
    return out


def _ensemble_members(n_members, t_sim, policy):
    """The ensemble's members, FP32, with their stage-kernel configuration
    chosen by ``policy``: "member" autotunes every member on its own mesh;
    "degree" autotunes the largest member of each degree and gives its
    choice to the others, so that each degree is one launch group."""
    import math
    import meshgen
    from paper_2307_14302_amd import Solver
    members = []
    for i, n_tri, p in meshgen.ensemble_plan(n_members):
        sc = meshgen.basin_member(4, i, n_tri, p=p)
        s = Solver.from_scenario(sc, precision="fp32")
        if policy == "member":
            s.autotune(3)
        dt0 = s.mass()["dt_next"]
        members.append((s, int(math.ceil(t_sim / dt0)), int(sc.params["rk_stages"]), p))
    if policy == "degree":
        for p in sorted({m[3] for m in members}):
            group = [m[0] for m in members if m[3] == p]
            ref = max(group, key=lambda s: s.n_tri)
            ref.autotune(3)
            for s in group:
                s.set_variant(ref.variant())
                s.set_fused(ref.fused())
                s.set_tile(ref.tile())
    return members


def _launch_groups(members):
    """Launch groups of a batch: members that share degree, scheme and kernel
    configuration run in the same launches."""
    return len({(p, st, s.variant(), s.fused(), s.tile()) for s, _, st, p in members})


def _run_batch(members, chunk):
    from paper_2307_14302_amd import Batch
    b = Batch({"precision": "fp32"})
    slots = {b.add(s, n): k for k, (s, n, _, _) in enumerate(members)}
    b.step(0)                                   # builds the member tables
    b.poll()
    # idle time before and after the timed loop sets the batch's kernels
    # apart from set-up and autotuning in a kernel trace
    time.sleep(0.2)
    done_at = {}
    t0 = time.perf_counter()
    while len(done_at) < len(slots):
        b.step(chunk)
        now = time.perf_counter() - t0
        for sl in b.poll():
            done_at.setdefault(sl, now)
    el = time.perf_counter() - t0
    time.sleep(0.2)
    lat = np.array([done_at[sl] for sl in slots])
    for sl in list(slots):
        b.retire(sl)
    b.close()
    return el, lat


def run_ensemble(n_members=64, t_sim=120.0, chunk=10, save_dir=None):
    """64 members (sizes log-uniform in [1e4, 5e5] triangles, even members
    p = 1, odd members p = 2, FP32), each simulating t_sim seconds, stepped
    together by one batch: every launch covers all active members of one
    launch group (degree, scheme, kernel configuration).  Latency =
    completion time of a member from the batch start.  Run twice: kernel
    configuration autotuned per degree (one launch group per degree: the
    reported value), and per member, which prices the extra launch groups."""
    t0 = time.perf_counter()
    members = _ensemble_members(n_members, t_sim, "degree")
    log(f"[ensemble] {len(members)} members, {sum(m[0].n_tri for m in members)} triangles, set-up "
        f"{time.perf_counter() - t0:.1f}s (one kernel configuration per degree)")
    groups = _launch_groups(members)
    el, lat = _run_batch(members, chunk)
    work = sum(s.n_tri * st * n for s, n, st, _ in members)
    # algorithmic bytes of every member's steps (each array streamed once
    # per launch, as for the single-mesh roofline), over the batch's time
    byts = sum(step_bytes(s.n_tri, s.n_nodes, 4, p, st, True, bool(s.fused())) * n for s, n, st, p in members)
    out = {"value": round(work / el, 1), "unit": "element-stage updates/s", "members": len(members),
           "n_tri_total": int(sum(s.n_tri for s, _, _, _ in members)),
           "p_mix": {"p1": sum(1 for m in members if m[3] == 1), "p2": sum(1 for m in members if m[3] == 2)},
           "t_sim_s": t_sim, "steps_min": int(min(m[1] for m in members)), "steps_max": int(max(m[1] for m in members)),
           "stage_variants": {"per_element": sum(1 for m in members if m[0].variant() == 0),
                              "per_edge": sum(1 for m in members if m[0].variant() == 1)},
           "stage_tiles": {str(t): sum(1 for m in members if m[0].tile() == t) for t in (64, 128, 256, 512)},
           "fused_members": sum(1 for m in members if m[0].fused()),
           "launch_groups": groups,
           "wall_s": round(el, 3), "p50_latency_s": round(float(np.percentile(lat, 50)), 4),
           "p99_latency_s": round(float(np.percentile(lat, 99)), 4), "dtype": "f32",
           "roofline": {"bound": "hbm", "achieved": round(byts / el / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(byts / el / 1e9 / HBM_PEAK_GBS, 4), "bytes": int(byts),
                        "basis": "algorithmic bytes of every launch of every member step (bench.step_bytes) "
                                 "over the batch's wall time"}}
    log(f"[ensemble] {work:.3e} element-stages in {el:.2f}s -> {work / el:.4e}/s with {groups} launch groups; "
        f"latency p50 {out['p50_latency_s']}s p99 {out['p99_latency_s']}s")
    if save_dir:
        # the p = 2 member of median size, as the batch left it, for the
        # oracle's one-step comparison in the CPU leg
        p2 = sorted((m[0].n_tri, k) for k, m in enumerate(members) if m[3] == 2)
        k = p2[len(p2) // 2][1]
        save_one_step(members[k][0], save_dir, "ensemble_fp32")
        with open(os.path.join(save_dir, "ensemble_member.json"), "w") as f:
            json.dump({"index": k, "n_members": n_members}, f)
        out["oracle_member"] = {"index": k, "n_tri": members[k][0].n_tri, "p": 2}
    for s, _, _, _ in members:
        s.close()
    # the same ensemble with the kernel configuration autotuned per member
    members = _ensemble_members(n_members, t_sim, "member")
    g2 = _launch_groups(members)
    el2, lat2 = _run_batch(members, chunk)
    work2 = sum(s.n_tri * st * n for s, n, st, _ in members)
    out["per_member_config"] = {"value": round(work2 / el2, 1), "launch_groups": g2, "wall_s": round(el2, 3),
                                "p50_latency_s": round(float(np.percentile(lat2, 50)), 4),
                                "p99_latency_s": round(float(np.percentile(lat2, 99)), 4),
                                "note": "every member autotuned on its own mesh; members whose choices differ "
                                        "run in separate launches"}
    log(f"[ensemble/per-member] {work2 / el2:.4e}/s with {g2} launch groups; latency p50 "
        f"{out['per_member_config']['p50_latency_s']}s p99 {out['per_member_config']['p99_latency_s']}s")
    for s, _, _, _ in members:
        s.close()
    return out


def run_serving(n_req=100, rate=20.0, budget_gib=24.0, chunk=20, light_rate=3.0, light_req=40):
    """Poisson arrivals of scenarios on a pool of 64 basin meshes (5e3..2e6
    triangles, FP32, p = 1, steps of at most 0.5 s), 500..5000 steps each,
    admitted by footprint under an HBM budget, continuous batching.
    Latency = arrival -> result (vertex state) on the host, split into queue
    delay (arrival -> admission) and service time (admission -> result).  Two
    traces: the first ``n_req`` requests at ``rate``/s (about three times
    what one GPU serves, so requests queue) and ``light_req`` requests of the
    same kind at ``light_rate``/s (below capacity)."""
    import meshgen
    from paper_2307_14302_amd import Request, Server, latency_summary
    sizes = meshgen.serving_pool_sizes()
    params = dict(precision="fp32", p=1, flux="llf", friction="manning", limiter=True, cfl=0.3, H0=0.05, dt_max=0.5)
    traces = {"overloaded": meshgen.request_trace(n_req=400, rate=rate, n_meshes=len(sizes))[:n_req],
              "below_capacity": meshgen.request_trace(n_req=light_req, rate=light_rate, n_meshes=len(sizes),
                                                      config_id=6)}
    t0 = time.perf_counter()
    pool = {}
    for k in sorted({r["mesh"] for tr in traces.values() for r in tr}):
        N = max(4, int(round(np.sqrt(sizes[k] / 2.0))))
        pool[k] = meshgen.basin(N, meshgen.seed_for(5, 1000 + k))
    log(f"[serving] {len(pool)} pool meshes generated in {time.perf_counter() - t0:.1f}s")
    out = {}
    for name, trace in traces.items():
        srv = Server(params, budget_bytes=int(budget_gib * (1 << 30)), chunk_steps=chunk, keep_results=False)
        for k in sorted({r["mesh"] for r in trace}):
            m = pool[k].mesh
            srv.register_mesh(k, m.xy, m.hb, m.fric, m.tri, m.bedges, m.btype, m.bslot)
        reqs = [Request(id=r["id"], arrival=r["arrival"], mesh=r["mesh"], n_steps=r["n_steps"],
                        initial=(pool[r["mesh"]].zeta0, pool[r["mesh"]].qx0, pool[r["mesh"]].qy0),
                        rain={"kind": "parametric", "records": r["track"]}, tides=dict(pool[r["mesh"]].tides))
                for r in trace]
        t0 = time.perf_counter()
        done = srv.run(reqs)
        el = time.perf_counter() - t0
        srv.close()
        work = sum(r.n_tri * 2 * r.n_steps for r in done)
        ls = latency_summary(done)
        rnd = lambda x: None if x is None else round(x, 4)  # noqa: E731
        out[name] = {"value": round(work / el, 1), "unit": "element-stage updates/s", "requests": len(done),
                     "arrival_rate_per_s": rate if name == "overloaded" else light_rate,
                     "makespan_s": round(el, 3),
                     "p50_latency_s": rnd(ls["p50_s"]), "p99_latency_s": rnd(ls["p99_s"]),
                     "mean_latency_s": rnd(ls["mean_s"]),
                     "queue_p50_s": rnd(ls["queue_p50_s"]), "queue_p99_s": rnd(ls["queue_p99_s"]),
                     "service_p50_s": rnd(ls["service_p50_s"]), "service_p99_s": rnd(ls["service_p99_s"]),
                     "failed": ls["failed"]}
        log(f"[serving/{name}] {len(done)} requests, {work:.3e} element-stages in {el:.2f}s -> {work / el:.4e}/s; "
            f"latency p50 {out[name]['p50_latency_s']}s p99 {out[name]['p99_latency_s']}s (queue p50 "
            f"{out[name]['queue_p50_s']}s, service p50 {out[name]['service_p50_s']}s)")
    res = dict(out["overloaded"])
    res.update({"budget_gib": budget_gib, "chunk_steps": chunk, "dtype": "f32",
                "trace": f"first {n_req} of a 400-request seeded trace", "below_capacity": out["below_capacity"]})
    return res


def run_graded(steps=1000, warmup=20, variant=-1, fused=-1, tile=-1, save_dir=None, fp64=True, main="fp32"):
    """The graded coastal workload at full size (3,596,698 triangles, FP32
    state, FP64 reductions, tidal boundary, river inflow, gridded rain);
    the stage kernel autotuned unless ``variant`` is given.  With ``fp64``
    the same steps also run on the plain FP64 path, its rate beside;
    ``main`` = "fp64" runs the FP64 path alone (for its counters)."""
    import meshgen
    t0 = time.perf_counter()
    sc = meshgen.graded_coast()
    log(f"[graded] {sc.mesh.n_tri} triangles generated in {time.perf_counter() - t0:.1f}s")
    if main == "fp64":
        f = run_precision(sc, "fp64", steps, warmup, variant, 2, fused=fused, tile=tile)
        return {"value": round(f["rate"], 1), "ms_per_step": round(f["elapsed"] / steps * 1e3, 4),
                "stage_variant": f["variant"], "stage_tile": f["tile"], "dtype": "f64",
                "roofline": roofline(f, "fp64", 1, True, "graded3.6M_p1")}
    r = run_precision(sc, "fp32", steps, warmup, variant, 2, fused=fused, tile=tile, save_dir=save_dir,
                      save_name="graded")
    n, ms = r["stats"]["stage"]
    out = {"value": round(r["rate"], 1), "unit": "element-stage updates/s", "n_tri": r["E"], "steps": steps,
           "ms_per_step": round(r["elapsed"] / steps * 1e3, 4), "stage_avg_us": round(ms / max(n, 1) * 1e3, 2),
           "dt_s": r["mass"]["dt_last"], "dtype": "f32", "stage_variant": r["variant"], "fused": r["fused"],
           "stage_tile": r["tile"],
           "roofline": roofline(r, "fp32", 1, True, "graded3.6M_p1"),
           "workload": "graded coast 30 m - 15.36 km, 1229 x 922 km, tides, 3 rivers, gridded rain, LLF, limiter"}
    if fp64:
        f = run_precision(sc, "fp64", steps, warmup, variant, 2, fused=fused, tile=tile)
        out["fp64"] = {"value": round(f["rate"], 1), "ms_per_step": round(f["elapsed"] / steps * 1e3, 4),
                       "stage_variant": f["variant"], "stage_tile": f["tile"], "dtype": "f64",
                       "roofline": roofline(f, "fp64", 1, True, "graded3.6M_p1"),
                       "fp32_over_fp64": round(r["rate"] / f["rate"], 3)}
    return out


def run_storm(N=708, steps=1000, warmup=20, save_dir=None):
    """The basin with the storm's wind stress and pressure on the rain track
    (FP32): the cost of the meteorological forcing."""
    import meshgen
    sc = meshgen.basin(N, wind=True)
    r = run_precision(sc, "fp32", steps, warmup, -1, 2, save_dir=save_dir, save_name="storm")
    n, ms = r["stats"]["stage"]
    return {"value": round(r["rate"], 1), "unit": "element-stage updates/s", "n_tri": r["E"], "steps": steps,
            "ms_per_step": round(r["elapsed"] / steps * 1e3, 4), "stage_avg_us": round(ms / max(n, 1) * 1e3, 2),
            "stage_variant": r["variant"], "dtype": "f32",
            "workload": "single basin as above plus the storm vortex (4,000 Pa, r_max 30 km, B 1.3) on the rain "
                        "track: wind stress and pressure gradient"}


def run_c1(outdir):
    """The 1,024-triangle rain-on-channel workload (1000 SSP-RK2 steps at
    CFL 0.3) on the GPU in FP64 and FP32: wall time of the 1000 steps, and
    the final states saved for the oracle comparison of the CPU leg."""
    import meshgen
    import torch
    from paper_2307_14302_amd import Solver
    sc = meshgen.channel_c1()
    out = {}
    for prec in ("fp64", "fp32"):
        s = Solver.from_scenario(sc, precision=prec)
        s.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(1000)
        s.sync()
        el = time.perf_counter() - t0
        np.save(os.path.join(outdir, f"c1_{prec}.npy"), s.state())
        out[prec] = {"seconds": round(el, 4), "value": round(sc.mesh.n_tri * 2 * 1000 / el, 1)}
        s.close()
    log(f"[c1] 1000 steps: FP64 {out['fp64']['seconds']} s, FP32 {out['fp32']['seconds']} s")
    return {"workload": "rain on a 100 m x 10 m channel, 1024 triangles, 1000 SSP-RK2 steps, Roe, CFL 0.3",
            "unit": "element-stage updates/s", **out}


def cpu_baseline(outdir, basin_state=None, timeout=900):
    """The FP64 oracle on one host core (OMP/OpenBLAS/MKL threads = 1):

    * the bench workload: 2 SSP-RK2 steps of the full basin, started from
      the GPU's FP32 state after the timed run (timed; the first step is also
      compared with the GPU's FP32 step from that state: the FP32 error);
    * the channel workload: all 1000 steps from its initial state, in CPU
      seconds, and the GPU's final FP64 and FP32 states against it;
    * the other FP32 legs (the storm basin, the graded coast and the median
      p = 2 ensemble member): one oracle step from the GPU's state after the
      leg, against the GPU's step (untimed: their FP32 error)."""
    code = r"""
import json, os, sys, time
import numpy as np
sys.path.insert(0, %r)
import meshgen
from oracle import basis
from oracle.solver import from_scenario
outdir = %r

def rel_l2(wg, o):
    # vertex values (p = 1) or values at the collapsed (p+1) x (p+1) Gauss
    # points (p >= 2); momentum as a vector; floors as in the parity tests
    if o.p >= 2:
        t, _ = np.polynomial.legendre.leggauss(o.p + 1)
        A, B = np.meshgrid(t, t)
        r, s_ = (0.5 * (1.0 + A) * (1.0 - B) - 1.0).ravel(), B.ravel()
        P = basis.eval_basis(o.p, r, s_)[0]
        a = np.einsum("evm,mq->evq", wg, P); b = np.einsum("evm,mq->evq", o.w, P)
        H = b[:, 0] + o.hbv @ np.array(basis.barycentric(r, s_))
    else:
        P = basis.Tables(1).phi_v
        a = np.einsum("evm,im->evi", wg[:, :, :3], P); b = np.einsum("evm,im->evi", o.w[:, :, :3], P)
        H = b[:, 0] + o.hbv
    D = max(np.sqrt(np.mean(H * H)), 1e-3); n = H.size
    fz = 1e-3 * np.sqrt(n) * D; fq = fz * np.sqrt(9.81 * D)
    ez = np.linalg.norm(a[:, 0] - b[:, 0]) / max(np.linalg.norm(b[:, 0]), fz)
    eq = np.linalg.norm(a[:, 1:] - b[:, 1:]) / max(np.linalg.norm(b[:, 1:]), fq)
    return [float(ez), float(eq)]

res = {}
sc = meshgen.channel_c1()
o = from_scenario(sc)
t0 = time.perf_counter()
o.step(1000)
res["c1_seconds"] = time.perf_counter() - t0
res["c1_E"] = o.E
for prec in ("fp64", "fp32"):
    f = os.path.join(outdir, "c1_%%s.npy" %% prec)
    if os.path.exists(f):
        res["c1_err_" + prec] = rel_l2(np.load(f), o)
sc = meshgen.basin(708)
s = from_scenario(sc)
f0 = os.path.join(outdir, "basin_fp32_w0.npy")
if os.path.exists(f0):
    m0 = json.load(open(os.path.join(outdir, "basin_fp32_m0.json")))
    s.set_state(np.load(f0), m0["t"], post=False)
    s.dt = m0["dt_next"]
    res["from_gpu_state"] = True
t0 = time.perf_counter()
s.step(1)
t1 = time.perf_counter()
if os.path.exists(f0):
    res["basin_err_fp32"] = rel_l2(np.load(os.path.join(outdir, "basin_fp32_w1.npy")), s)
t2 = time.perf_counter()
s.step(1)
res["E"] = s.E
res["elapsed"] = (t1 - t0) + (time.perf_counter() - t2)
del s

def one_step(name, scenario):
    # the oracle's step from the GPU's saved state, against the GPU's step
    f0 = os.path.join(outdir, name + "_w0.npy")
    if not os.path.exists(f0):
        return
    m0 = json.load(open(os.path.join(outdir, name + "_m0.json")))
    o = from_scenario(scenario())
    o.set_state(np.load(f0), m0["t"], post=False)
    o.dt = m0["dt_next"]
    o.step(1)
    res[name + "_err"] = rel_l2(np.load(os.path.join(outdir, name + "_w1.npy")), o)

one_step("storm_fp32", lambda: meshgen.basin(708, wind=True))
one_step("graded_fp32", meshgen.graded_coast)
fm = os.path.join(outdir, "ensemble_member.json")
if os.path.exists(fm):
    em = json.load(open(fm))
    i, n_tri, p = list(meshgen.ensemble_plan(em["n_members"]))[em["index"]]
    one_step("ensemble_fp32", lambda: meshgen.basin_member(4, i, n_tri, p=p))
print(json.dumps(res))
""" % (ROOT, outdir)
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1")
    try:
        out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=timeout)
        r = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as e:  # report, never fail the bench on the baseline leg
        return {"value": None, "unit": "element-stage updates/s", "cores": 1, "kind": "oracle", "error": str(e)[:200]}
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except Exception:
        pass
    out = {"value": round(r["E"] * 2 * 2 / r["elapsed"], 1), "unit": "element-stage updates/s", "cores": 1,
           "kind": "oracle", "sample": f"2 SSP-RK2 steps of the full {r['E']}-triangle basin"
           + (" from the GPU's state after the timed run" if r.get("from_gpu_state") else "")
           + f", FP64 NumPy oracle, 1 thread ({r['elapsed']:.1f}s)", "host_cpus": os.cpu_count(), "cpu_model": cpu_model,
           "c1": {"seconds": round(r["c1_seconds"], 3), "steps": 1000,
                  "value": round(r["c1_E"] * 2 * 1000 / r["c1_seconds"], 1),
                  "sample": "the whole 1000-step channel run, 1 thread"}}
    errs = {}
    if "basin_err_fp32" in r:
        errs["basin_fp32_one_step_rel_l2"] = r["basin_err_fp32"]
    for leg in ("storm", "graded", "ensemble"):
        if f"{leg}_fp32_err" in r:
            errs[f"{leg}_fp32_one_step_rel_l2"] = r[f"{leg}_fp32_err"]
    for prec in ("fp64", "fp32"):
        if "c1_err_" + prec in r:
            errs[f"c1_{prec}_1000_steps_rel_l2"] = r["c1_err_" + prec]
    if errs:
        out["gpu_error_vs_oracle"] = dict(errs, norm="relative L2 of (zeta, discharge vector) at the vertices "
                                                    "(p = 1) or the collapsed Gauss points (p = 2)")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", choices=["both", "fp32", "fp64"], default="both")
    ap.add_argument("--N", type=int, default=708, help="quads per side (708 -> 1,002,528 triangles)")
    ap.add_argument("--p", type=int, default=1, choices=[1, 2, 3], help="polynomial degree of the basin run")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-c1", action="store_true", help="skip the 1024-triangle channel run")
    ap.add_argument("--fused", type=int, default=-1, choices=[-1, 0, 1],
                    help="post-processing fused into the next stage: 0 off, 1 on, -1 as the autotuner picks")
    ap.add_argument("--tile", type=int, default=-1, choices=[-1, 64, 128, 256, 512],
                    help="elements per workgroup of the per-edge stage kernel: -1 as the autotuner picks")
    ap.add_argument("--variant", type=int, default=-1,
                    help="stage kernel: 0 per element, 1 per edge, 2 per edge with matrix-core area integrals (p = 3, "
                         "FP32), -1 autotuned on the workload (default)")
    ap.add_argument("--calib-copy", action="store_true", help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-events", action="store_true",
                    help="no HIP events in the timed region (steps replay a HIP graph; no roofline)")
    ap.add_argument("--events-all", action="store_true", help="HIP events around every kernel (per-kernel times)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the 64-member FP32 ensemble")
    ap.add_argument("--no-graded", action="store_true", help="skip the 3.6M-triangle graded coastal run")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-loop run")
    ap.add_argument("--no-storm", action="store_true", help="skip the basin run with storm wind and pressure")
    ap.add_argument("--serve-requests", type=int, default=100, help="requests of the 400-request trace to serve")
    ap.add_argument("--graded-only", action="store_true",
                    help="run only the 3.6M-triangle graded leg (--steps steps), FP32 unless --precision fp64, and "
                         "print its JSON (for profiling)")
    ap.add_argument("--ensemble-only", action="store_true",
                    help="run only the 64-member ensemble leg and print its JSON (for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the library drives one GPU per process and has no multi-GPU "
              "path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import meshgen
    torch.cuda.set_device(0)
    if args.graded_only:
        out = run_graded(steps=args.steps, warmup=args.warmup, variant=args.variant, fused=args.fused,
                         tile=args.tile, fp64=False, main="fp64" if args.precision == "fp64" else "fp32")
        if args.calib_copy:
            calib_copy()
        print(json.dumps(out), flush=True)
        return
    if args.ensemble_only:
        print(json.dumps(run_ensemble()), flush=True)
        return
    t0 = time.perf_counter()
    sc = meshgen.basin(args.N, p=args.p)
    log(f"workload generated in {time.perf_counter() - t0:.1f}s: {sc.mesh.n_tri} triangles")
    prm = sc.params
    res = {}
    import tempfile
    import shutil
    outdir = tempfile.mkdtemp(prefix="dgswe_bench_")
    for prec in (["fp32", "fp64"] if args.precision == "both" else [args.precision]):
        mode = 0 if args.no_events else (1 if args.events_all else 2)
        res[prec] = run_precision(sc, prec, args.steps, args.warmup, args.variant, mode,
                                  save_dir=outdir if (prec == "fp32" and not args.no_cpu and args.N == 708
                                                      and args.p == 1) else None, fused=args.fused,
                                  tile=args.tile)
    if args.calib_copy:
        calib_copy()
    ceiling = stream_ceiling()
    main_prec = "fp32" if "fp32" in res else "fp64"
    basin_key = "basin1M_p1" if args.N == 708 and args.p == 1 else None
    r = res[main_prec]
    out = {
        "metric": METRIC, "value": round(r["rate"], 1), "unit": "element-stage updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(r["elapsed"] / args.steps * 1e3, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if main_prec == "fp32" else "f64", "data": "synthetic",
        "config": {"workload": f"single basin, {r['E']} triangles (jittered {args.N}x{args.N} grid over 200 km), "
                               f"p={args.p}, LLF, limiter on, parametric moving rain, wet/dry front, "
                               + f"SSP-RK{r['stages']} CFL {prm['cfl']}",
                   "n_tri": r["E"], "p": prm["p"], "rk_stages": r["stages"], "precision": main_prec,
                   "stage_variant": r["variant"], "fused_post": r["fused"], "stage_tile": r["tile"],
                   "parallelism": "single GPU"},
        "roofline": roofline(r, main_prec, prm["p"], prm["limiter"], basin_key),
    }
    rl = out["roofline"]
    if rl and ceiling.get("hbm_4x512MiB"):
        # the measured streaming rate with the same read:write mix, beside the peak
        rl["ceiling_gbs"] = ceiling["hbm_4x512MiB"]
        rl["ceiling_mall_gbs"] = ceiling.get("mall_4x32MiB")
        rl["frac_of_ceiling"] = round(rl["achieved"] / ceiling["hbm_4x512MiB"], 4)
    if r.get("graph"):
        out["graph_replay"] = dict(r["graph"], note="the same run continued with one replayed HIP graph per step and "
                                                    "no per-launch events (not the timed region of value)")
    if "fp64" in res and main_prec != "fp64":
        f = res["fp64"]
        out["fp64"] = {"value": round(f["rate"], 1), "ms_per_step": round(f["elapsed"] / args.steps * 1e3, 4),
                       "stage_variant": f["variant"],
                       "dtype": "f64", "roofline": roofline(f, "fp64", prm["p"], prm["limiter"], basin_key),
                       "fp32_over_fp64": round(r["rate"] / f["rate"], 3)}
    # the FP32 legs also leave one step for the oracle to check in the CPU leg
    keep = outdir if (not args.no_cpu and args.N == 708 and args.p == 1) else None
    if not args.no_storm:
        out["storm"] = run_storm(args.N, save_dir=keep)
        out["storm"]["vs_no_wind"] = round(out["storm"]["value"] / r["rate"], 3)
    if not args.no_graded:
        out["graded"] = run_graded(save_dir=keep)
    if not args.no_ensemble:
        out["ensemble"] = run_ensemble(save_dir=keep)
        if "fp64" in res:
            out["ensemble"]["vs_fp64_single_mesh"] = round(out["ensemble"]["value"] / res["fp64"]["rate"], 3)
    if not args.no_serving:
        out["serving"] = run_serving(n_req=args.serve_requests)
    if not args.no_c1:
        out["c1"] = run_c1(outdir)
    if not args.no_cpu:
        log("timing the oracle on one host core ...")
        out["cpu_baseline"] = cpu_baseline(outdir)
    shutil.rmtree(outdir, ignore_errors=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
