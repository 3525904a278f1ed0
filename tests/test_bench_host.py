"""Host-side logic of bench.py (no GPU): the one-GPU guard, and that the
committed counter summaries are used only while the profiled kernel's
sources are unchanged."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    rec = json.loads(r.stdout.strip().splitlines()[-1])
    assert rec["n_gpus"] == 2 and "one GPU" in rec["error"]


def _summary(name):
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        pytest.skip(f"no committed summary {name}")
    with open(path) as f:
        return json.load(f)


def test_traffic_follows_the_source_hash(monkeypatch):
    rec = _summary("k_sweep_blocked_rmat20_k2_traffic.json")
    want = rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]
    assert rec["bytes_per_launch"] == pytest.approx(want)
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: rec["source_hash"])
    assert bench._traffic("rmat20_k2", "k_sweep_blocked") == rec["bytes_per_launch"]
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: "changed")
    assert bench._traffic("rmat20_k2", "k_sweep_blocked") is None
    assert bench._traffic("no_such_workload", "k_sweep_blocked") is None


def test_valu_issue_rate(monkeypatch):
    rec = _summary("k_sweep_blocked_rmat20_k2_valu.json")
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: rec["source_hash"])
    v = bench._valu_issue("rmat20_k2", "k_sweep_blocked", 20.0)
    insts = rec["counters_per_dispatch"]["SQ_INSTS_VALU"]
    assert v["achieved"] == pytest.approx(insts * 64 / 0.020)
    assert v["peak"] == pytest.approx(256 * 64 * 2.4e9)
    assert v["frac"] == pytest.approx(v["achieved"] / v["peak"])
    assert rec["valu_lane_slots_per_pair"] == pytest.approx(insts * 64 / rec["pairs_per_dispatch"])
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: "changed")
    assert bench._valu_issue("rmat20_k2", "k_sweep_blocked", 20.0) is None


@pytest.mark.parametrize("name,workload,kernel", [
    ("k_sweep_blocked_rmat20_k2_l2.json", "rmat20_k2", "k_sweep_blocked"),
    ("k_sweep_rmat20_k1_l2.json", "rmat20_k1", "k_sweep"),
])
def test_l2_hit_rate(monkeypatch, name, workload, kernel):
    rec = _summary(name)
    c = rec["counters_per_dispatch"]
    assert rec["l2_hit_rate"] == pytest.approx(c["TCC_HIT_sum"] / (c["TCC_HIT_sum"] + c["TCC_MISS_sum"]))
    assert 0.0 <= rec["l2_hit_rate"] <= 1.0
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: rec["source_hash"])
    assert bench._l2_hit_rate(workload, kernel) == rec["l2_hit_rate"]
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: "changed")
    assert bench._l2_hit_rate(workload, kernel) is None



def test_roofline_is_a_fraction_of_the_binding_roof(monkeypatch):
    """The blocked sweep is priced at its 15 VALU lane-instructions per stored
    pair against 256 CUs x 64 lanes x 2.4 GHz; the 16-bytes-per-pair
    convention is kept apart, since it exceeds the HBM peak by design.  A
    row-form sweep is priced against HBM with the algorithmic bytes."""
    monkeypatch.setattr(bench, "_kernel_source_hash", lambda k: "none")
    nnz, na, n, M = 23762699968, 646140, 1048576, 5
    r = bench.roofline("rmat20_k2", "k_sweep_blocked", 18.7, 500, nnz, na, n, M, 1, 4500.0)
    assert r["bound"] == "alu" and r["traffic"] is None
    assert r["achieved"] == pytest.approx(15 * nnz / 0.0187 / 1e12)
    assert r["peak"] == pytest.approx(256 * 64 * 2.4e9 / 1e12)
    assert 0.0 < r["frac"] < 1.0
    assert r["convention"]["frac_of_8TBs"] > 1.0
    r = bench.roofline("rmat20_k1", "k_sweep", 0.79, 500, 31_400_000, na, n, M, 1, 4500.0)
    assert r["bound"] == "hbm"
    want = (16.0 * 31_400_000 + 16.0 * M * na + 28.0 * n) / 0.00079 / 1e9
    assert r["achieved"] == pytest.approx(want) and r["frac"] == pytest.approx(want / 8000.0)
