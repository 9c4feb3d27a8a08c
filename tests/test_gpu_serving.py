"""The request loop: results are the same alone and in the mix, admission
respects the HBM budget, and requests arriving while others run share their
launches."""
import numpy as np
import pytest

import meshgen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2307_14302_amd as pkg
    return pkg


PARAMS = dict(precision="fp32", p=1, flux="llf", friction="manning", limiter=True, cfl=0.3, H0=0.05, dt_max=0.5)


def pool():
    sizes = [6000, 15000, 30000]
    return [meshgen.basin(int(round(np.sqrt(n / 2))), meshgen.seed_for(5, 900 + k)) for k, n in enumerate(sizes)]


def requests(dg, scs, arrivals):
    tr = meshgen.request_trace(n_req=len(arrivals), rate=50.0, n_meshes=len(scs), steps=(30, 90))
    out = []
    for k, r in enumerate(tr):
        sc = scs[r["mesh"]]
        out.append(dg.Request(id=k, arrival=arrivals[k], mesh=r["mesh"], n_steps=r["n_steps"],
                              initial=(sc.zeta0, sc.qx0, sc.qy0),
                              rain={"kind": "parametric", "records": r["track"]}, tides=dict(sc.tides)))
    return out


def alone(dg, sc, r):
    s = dg.Solver(PARAMS)
    m = sc.mesh
    s.upload_mesh(m.xy, m.hb, m.fric, m.tri, m.bedges, m.btype, m.bslot)
    for slot, (mean, rows) in r.tides.items():
        s.set_tide(slot, mean, rows)
    s.set_rain(r.rain)
    s.set_initial_nodal(*r.initial)
    s.step(r.n_steps)
    out = s.state("vertex"), s.mass()
    s.close()
    return out


def make_server(dg, scs, budget):
    srv = dg.Server(PARAMS, budget_bytes=budget, chunk_steps=7)
    for k, sc in enumerate(scs):
        m = sc.mesh
        srv.register_mesh(k, m.xy, m.hb, m.fric, m.tri, m.bedges, m.btype, m.bslot)
    return srv


def test_results_same_alone_and_in_the_mix(dg):
    scs = pool()
    reqs = requests(dg, scs, [0.0, 0.0, 0.002, 0.004, 0.03, 0.05, 0.05, 0.08])
    srv = make_server(dg, scs, budget=8 << 30)
    done = srv.run(reqs)
    srv.close()
    assert len(done) == len(reqs)
    for r in done:
        assert r.error is None, r.error
        w, m = alone(dg, scs[r.mesh], r)
        assert np.array_equal(r.result, w), r.id
        assert r.mass == m
        assert r.done >= r.admitted >= r.arrival
    # later arrivals joined while earlier requests were running
    first_done = min(r.done for r in done)
    assert any(r.admitted < first_done for r in done if r.arrival > 0.0)


def test_admission_waits_for_memory(dg):
    scs = pool()
    reqs = requests(dg, scs, [0.0] * 6)
    probe = make_server(dg, scs, budget=8 << 30)
    fp = {k: dg.Solver.footprint_of(PARAMS, probe.meshes[k]) for k in range(len(scs))}
    probe.close()
    # room for the largest request and a little more: requests must queue
    budget = int(1.2 * max(fp[r.mesh] for r in reqs))
    srv = make_server(dg, scs, budget)
    done = srv.run(reqs)
    srv.close()
    assert len(done) == len(reqs)
    events = sorted([(r.admitted, 1, r) for r in done] + [(r.done, -1, r) for r in done],
                    key=lambda e: (e[0], e[1]))
    resident, peak = {}, 0
    for _, kind, r in events:
        if kind == 1:
            resident[r.id] = fp[r.mesh]
        else:
            resident.pop(r.id, None)
        peak = max(peak, sum(resident.values()))
    assert peak <= budget
    assert max(r.admitted for r in done) > 0.0          # someone waited
    for r in done:
        w, _ = alone(dg, scs[r.mesh], r)
        assert np.array_equal(r.result, w)


def test_served_request_against_the_oracle(dg):
    """One request of a mix, its modal result against the FP64 oracle run of
    the same scenario (mesh, initial state, storm track, tide)."""
    from oracle.solver import OracleSolver
    from tests.parity import rel_l2
    scs = pool()
    reqs = requests(dg, scs, [0.0, 0.0, 0.001])
    srv = dg.Server(PARAMS, budget_bytes=8 << 30, chunk_steps=7, result_layout="modal")
    for k, sc in enumerate(scs):
        m = sc.mesh
        srv.register_mesh(k, m.xy, m.hb, m.fric, m.tri, m.bedges, m.btype, m.bslot)
    done = srv.run(reqs)
    srv.close()
    r = min(done, key=lambda q: scs[q.mesh].mesh.n_tri)
    m = scs[r.mesh].mesh
    prm = {k: v for k, v in PARAMS.items() if k != "precision"}
    orc = OracleSolver(m.xy, m.tri, m.hb, m.fric, m.bedges, m.btype, m.bslot, rain=r.rain, tides=r.tides, **prm)
    orc.set_initial_nodal(*r.initial)
    orc.step(r.n_steps)
    err = rel_l2(r.result, orc.w, orc)
    print(f"request {r.id} (E={m.n_tri}, {r.n_steps} steps): rel L2 {err}", flush=True)
    assert err.max() <= 1e-4, err
    assert r.mass["steps"] == r.n_steps and abs(r.mass["t"] - orc.t) <= 1e-6 * orc.t
