"""The bench line's accounting, on the host: algorithmic bytes per launch
and per step, the roofline fields built from them, and the counted-traffic
lookup in the committed counter summaries (read only while their recorded
kernel-source hash matches)."""
import json
import os

import pytest

import bench

E_BASIN = 1002528


def test_algorithmic_bytes_of_the_p1_stage_and_post():
    # stage 0: own state 36 B, edge vectors, bathymetry, friction and rain
    # 11 x 4 B, ids, codes and flag 14 B, writes 36 + 1 B
    assert bench.algorithmic_bytes("stage", 1, 4, 1, False, False, True) == 36 + 44 + 14 + 37
    # a blending stage also reads w^n
    assert bench.algorithmic_bytes("stage", 1, 4, 1, True, True, True) == 36 + 36 + 44 + 14 + 37
    # FP64 doubles every Real
    assert bench.algorithmic_bytes("stage", 1, 8, 1, True, True, True) == 72 + 72 + 88 + 14 + 73
    # the post pass: state, bathymetry, ids, limiter weights, code, wet byte,
    # state and flag written; the last stage adds edge vectors and d_in
    assert bench.algorithmic_bytes("post", 1, 4, 1, False, False, True) == 36 + 12 + 12 + 24 + 1 + 1 + 36 + 1
    assert bench.algorithmic_bytes("post", 1, 4, 1, True, True, True) == 123 + 28
    # p = 2 has six modes per variable
    assert bench.algorithmic_bytes("stage", 1, 4, 2, False, False, True) == 72 + 44 + 14 + 73
    # the per-launch mean of the two SSP(2,2) stages on the 1M basin
    mean = (bench.algorithmic_bytes("stage", E_BASIN, 4, 1, False, False, True)
            + bench.algorithmic_bytes("stage", E_BASIN, 4, 1, True, True, True)) / 2
    assert mean == 149 * E_BASIN


def test_roofline_fields_follow_from_bytes_and_time():
    res = {"stats": {"stage": (100, 100 * 0.0370), "post": (0, 0.0)}, "stages": 2, "fused": 0, "E": E_BASIN,
           "n_nodes": 502681, "elapsed": 0.148, "steps": 1000, "variant": 1, "tile": 64}
    r = bench.roofline(res, "fp32", 1, True, workload=None)
    assert r["kernel"] == "stage" and r["bound"] == "hbm" and r["peak"] == bench.HBM_PEAK_GBS
    assert r["bytes_per_launch"] == 149 * E_BASIN
    assert r["avg_us"] == pytest.approx(37.0)
    assert r["achieved"] == pytest.approx(149 * E_BASIN / 37.0e-6 / 1e9, rel=1e-3)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)
    assert r["traffic"] is None and "no committed counter summary" in r["traffic_source"]
    sb = bench.step_bytes(E_BASIN, 502681, 4, 1, 2, True, False)
    assert r["step"]["bytes"] == int(sb)
    assert r["step"]["frac"] == pytest.approx(sb / 0.148e-3 / 1e9 / bench.HBM_PEAK_GBS, rel=1e-3)


@pytest.mark.parametrize("workload,key", [("basin1M_p1", "stage_edge_kernel/t64/fp32"),
                                          ("graded3.6M_p1", "stage_edge_kernel/t128/fp32")])
def test_counted_traffic_is_read_only_for_matching_sources(monkeypatch, workload, key):
    path = os.path.join(bench.ROOT, "profiles", bench.COUNTER_SUMMARIES[workload])
    with open(path) as f:
        d = json.loads(next(l for l in f if l.startswith("traffic-json:")).split(":", 1)[1])
    tile = int(key.split("/t")[1].split("/")[0])
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: d["sources"])
    assert bench.counted_traffic("stage", "fp32", 1, tile, workload) == d["bytes"][key]
    assert bench.counted_traffic("post", "fp32", 1, tile, workload) == d["bytes"]["post_kernel/fp32"]
    # another stage tile, another kernel variant or another workload: no figure
    assert bench.counted_traffic("stage", "fp32", 1, 512, workload) is None
    assert bench.counted_traffic("stage", "fp32", 0, tile, workload) is None
    assert bench.counted_traffic("stage", "fp32", 1, tile, "basin1M_p2") is None
    # kernel sources changed since the counters were taken: no figure
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda: "0" * 16)
    assert bench.counted_traffic("stage", "fp32", 1, tile, workload) is None
