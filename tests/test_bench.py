"""Host logic of bench.py (no GPU): the algorithmic byte counts behind the
roofline, the counter-summary scaling, the stored-traffic lookup and its
staleness checks, the profile summaries, and the one-GPU contract."""
import csv
import os
import subprocess
import sys

import numpy as np
import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gather_bytes_structure():
    N, E, nnz, k, hubs = 1000, 700, 4000, 16, 7
    b4 = bench.gather_bytes(N, E, nnz, k, 4, covered=900, hubs=hubs)
    b8 = bench.gather_bytes(N, E, nnz, k, 8, covered=900, hubs=hubs)
    # the fused step streams F and R in and out and P in, where the apply
    # streams P in and Q out: three more row streams of the rows it finishes
    # (and it reads s of the hub rows too, to find the rows that iterate)
    assert b4["vertex_step"] - b4["vertex_gather"] == 4 * k * 3 * (N - hubs) + 4 * hubs
    # the value bytes scale with the element size, the index bytes do not
    for key in ("vertex_gather", "vertex_step", "edge_gather", "cg_iteration"):
        idx = 2 * b4[key] - b8[key]
        assert 0 < idx < b4[key]
    # each covered vertex adds its row of P and its entry of the covered list
    full = bench.gather_bytes(N, E, nnz, k, 4, covered=N, hubs=hubs)
    assert full["edge_gather"] - b4["edge_gather"] == (4 * k + 4) * (N - 900)
    # decoupled rows drop out of the fused step's and the direction's row
    # streams (five and three per row), not out of the iteration's definition
    d = bench.gather_bytes(N, E, nnz, k, 4, covered=900, hubs=hubs, decoupled=100)
    assert b4["vertex_step"] - d["vertex_step"] == 4 * k * 5 * 100
    assert b4["direction"] - d["direction"] == 4 * k * 3 * 100
    assert d["cg_iteration"] == b4["cg_iteration"]
    assert b4["cg_iteration_as_run"] - d["cg_iteration_as_run"] == 4 * k * 6 * 100


def test_decoupled_rows_count():
    import synth
    ep, ev = synth.explicit_hyperedges([[0, 1], [1, 2], [4, 5]])
    p = synth.Problem(7, 3, ep, ev, np.array([0.5, 0.5, 0.0]), 1.0, np.zeros((7, 1)))
    # vertex 3 and 6 are isolated, 4 and 5 only in a hyperedge of weight 0
    assert bench.decoupled_rows(p) == 4


def _write(path, rows, fields):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=fields)
        w.writeheader()
        for r in rows:
            w.writerow(r)


def test_summarize_counters_scales_by_the_copy(tmp_path):
    fields = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    # a 1 GiB copy that the counter reads as 512 MiB: factor 2 for FETCH,
    # read as 1 GiB for WRITE: factor 1
    fetch = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "FETCH_SIZE", "Counter_Value": 524288},
             {"Kernel_Name": "hgl::k_spmm_vertex<float, float, 64, 4, 3>(hgl::VertexArgs)",
              "Counter_Name": "FETCH_SIZE", "Counter_Value": 100},
             {"Kernel_Name": "hgl::k_spmm_vertex<float, float, 64, 4, 3>(hgl::VertexArgs)",
              "Counter_Name": "FETCH_SIZE", "Counter_Value": 300},
             {"Kernel_Name": "hgl::k_spmm_vertex<float, double, 64, 2, 2>(hgl::VertexArgs)",
              "Counter_Name": "FETCH_SIZE", "Counter_Value": 9999}]
    write = [{"Kernel_Name": "__amd_rocclr_copyBuffer", "Counter_Name": "WRITE_SIZE", "Counter_Value": 1048576},
             {"Kernel_Name": "hgl::k_spmm_vertex<float, float, 64, 4, 3>(hgl::VertexArgs)",
              "Counter_Name": "WRITE_SIZE", "Counter_Value": 50},
             {"Kernel_Name": "hgl::k_spmm_vertex<float, float, 64, 4, 3>(hgl::VertexArgs)",
              "Counter_Name": "WRITE_SIZE", "Counter_Value": 50}]
    _write(tmp_path / "f.csv", fetch, fields)
    _write(tmp_path / "w.csv", write, fields)
    rec = bench.summarize_counters(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), "k_spmm_vertex", "wl", "cmd")
    assert rec["instance"] == "hgl::k_spmm_vertex<float, float, 64, 4, 3>"  # the most-dispatched instance
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == round(200 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == round(50 * 1024 * 1.0)
    assert rec["dispatches"] == [2, 2]


def test_stored_traffic_checks_sources_and_instance(monkeypatch):
    path = os.path.join(bench.PROFILES, "multi_rhs_cg_k_spmm_vertex_traffic.json")
    if not os.path.exists(path):
        pytest.skip("no stored counter summary")
    import json
    rec = json.load(open(path))
    inst = rec["instance"].split("::")[-1]
    if rec["sources_sha256"] == bench.sources_digest():
        assert bench.stored_traffic("k_spmm_vertex", "multi_rhs_cg", inst) == rec["traffic_bytes_per_launch"]
    # another column shape, or changed kernel sources: no figure
    assert bench.stored_traffic("k_spmm_vertex", "multi_rhs_cg", inst.replace("64", "32", 1)) is None
    monkeypatch.setattr(bench, "sources_digest", lambda: "0" * 64)
    assert bench.stored_traffic("k_spmm_vertex", "multi_rhs_cg", inst) is None
    assert bench.stored_traffic("k_spmm_vertex", "no_such_workload", inst) is None


def test_summarize_stats_names(tmp_path):
    fields = ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"]
    rows = [{"Name": "hgl::(anonymous namespace)::k_cg_wg(hgl::(anonymous namespace)::WgArgs)", "Calls": "3",
             "AverageNs": "223400", "TotalDurationNs": "670200", "Percentage": "60.5"},
            {"Name": "void hgl::k_cg_direction<float, 64, 4>(int const*)", "Calls": "117",
             "AverageNs": "17750", "TotalDurationNs": "2076750", "Percentage": "39.5"}]
    _write(tmp_path / "s.csv", rows, fields)
    text = bench.summarize_stats(str(tmp_path / "s.csv"), "wl", "cmd")
    lines = text.splitlines()
    assert lines[0] == "# rocprofv3 kernel statistics: wl" and "command: cmd" in lines
    assert any(l.startswith("hgl::k_cg_wg ") and "223.40" in l for l in lines)
    assert any(l.startswith("hgl::k_cg_direction<float, 64, 4> ") and "17.75" in l for l in lines)


def test_roofline_fields():
    r = bench._roof("k", 4, 2.0, 4e9)  # 4 launches in 2 ms: 0.5 ms each, 4 GB per launch
    assert r["avg_launch_us"] == 500.0 and r["achieved"] == pytest.approx(8000.0)
    assert r["frac"] == pytest.approx(1.0) and r["peak"] == bench.HBM_PEAK_GBS
    m = bench._roof("g", 1, 1.0, 2.5e12, bound="mfma")  # 2.5 TFLOP in 1 ms
    assert m["achieved"] == pytest.approx(2500.0) and m["frac"] == pytest.approx(1.0)


def test_host_info_and_baseline_fields():
    info = bench._host_info()
    assert set(info) == {"cpu_model", "affinity_cores", "blas_threads"} and info["affinity_cores"] >= 1
    line = bench._line("m", 1.0, "u", 1, 0, 1.0, "f32", {}, None,
                       {"cpu_baseline": {"value": 1.0, "unit": "u", "cores": 1, "kind": "oracle", "sample": "s"}})
    assert line["cpu_baseline"]["host"] == info


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2 and "one GPU only" in r.stderr
