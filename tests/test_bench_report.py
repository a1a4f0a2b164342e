"""The bench line's arithmetic on the host: roofline bytes in the edge-visit
unit (with and without the update fused into the U-side gather), the stored
traffic lookup keyed by the kernel source, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

INFO = dict(n_edges=1000, n_u=100, n_v=200, isolated_u=10, isolated_v=20)


def stats(n, steps, vu, vv):
    return [dict(steps=steps, visits_u=vu, visits_v=vv, np_ss=vu, np_pi=vv, t=2, sparse_sweeps=1)
            for _ in range(n)]


def test_roofline_bytes_update_pass():
    # four kinds timed: gather A dominant
    prof = dict(ms=[4.0, 3.0, 1.0, 0.5], launches=[10, 10, 10, 10], live_sweeps=10)
    st = stats(3, 5, 100.0, 200.0)
    r = bench.roofline(prof, st, INFO, "no-such-workload")
    E, U1, V1, L, CS = 1000, 90, 180, 10, 15
    alg_a = L * (8 * E + 8 * V1) + 4 * 300.0 + 4 * V1 * CS
    assert r["kernel"].startswith("V-side gather")
    assert r["algorithmic_bytes_per_launch"] == int(alg_a / 10)
    assert r["achieved"] == pytest.approx(round(alg_a / 4e-3 / 1e9, 1))
    assert r["frac"] == pytest.approx(round(alg_a / 4e-3 / 1e9 / bench.HBM_PEAK_GBS, 4))
    assert r["traffic"] is None                       # no counters for this workload
    assert r["counts"]["edge_visits"] == 900.0
    assert r["counts"]["paper_work_units"] == 3 * (100 + 200 + 2 * E * 2)
    assert r["counts"]["column_use"] == round(CS / (64 * L), 4)
    assert set(r["kernels"]) == {"gather_a", "gather_b", "update", "select"}


def test_roofline_bytes_update_fused():
    # no update launches: the U-side gather carries the update's node terms without G
    prof = dict(ms=[3.0, 5.0, 0.0, 0.0], launches=[10, 10, 0, 0], live_sweeps=10)
    st = stats(2, 4, 50.0, 70.0)
    r = bench.roofline(prof, st, INFO, "no-such-workload")
    E, U1, L, CS = 1000, 90, 10, 8
    alg_b = L * (8 * E + 16 * U1) + 4 * 140.0 + 16 * U1 * CS
    assert r["kernel"].startswith("U-side gather with the update fused")
    assert r["algorithmic_bytes_per_launch"] == int(alg_b / 10)
    assert set(r["kernels"]) == {"gather_a", "gather_b"}   # kinds without launches are left out
    # compulsory: adjacency once per sweep, each dense row of both sides once per running column
    V1 = 180
    comp_b = L * (8 * E + 8 * U1) + 4 * (U1 + V1) * CS + L * 8 * U1 + 12 * U1 * CS
    assert r["compulsory"]["bytes_per_launch"] == int(comp_b / 10)
    assert r["compulsory"]["frac"] == pytest.approx(round(comp_b / 5e-3 / 1e9 / bench.HBM_PEAK_GBS, 4))


def test_traffic_rate_from_stored_counters(monkeypatch):
    prof = dict(ms=[3.0, 5.0, 0.0, 0.0], launches=[10, 10, 0, 0], live_sweeps=10)
    monkeypatch.setattr(bench, "stored_traffic", lambda wl, kind: 4_000_000_000 if kind == "gather_b" else None)
    r = bench.roofline(prof, stats(2, 4, 50.0, 70.0), INFO, "wl")
    assert r["traffic"] == 4_000_000_000
    assert r["traffic_gbs"] == pytest.approx(8000.0)   # 4 GB per launch in 0.5 ms


def test_stored_traffic_needs_the_profiled_source(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    src = tmp_path / "paper_2312_06724_amd" / "csrc"
    prof.mkdir()
    src.mkdir(parents=True)
    (src / "sweep.hip").write_text("kernel source v1\n")
    sha = bench.source_digest(str(src / "sweep.hip"))
    (prof / "pmc_traffic.json").write_text(json.dumps(
        {"wl": {"gather_b": {"sweep_hip_sha": sha, "bytes_per_launch": 1234}}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.stored_traffic("wl", "gather_b") == 1234
    assert bench.stored_traffic("wl", "gather_a") is None
    assert bench.stored_traffic("other", "gather_b") is None
    (src / "sweep.hip").write_text("kernel source v2\n")   # counters taken on another source
    assert bench.stored_traffic("wl", "gather_b") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
