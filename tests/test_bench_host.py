"""Host logic of bench.py, on the CPU: the one-GPU guard, the algorithmic
byte counts its roofline divides by, and the scaling of the rocprofv3
FETCH_SIZE / WRITE_SIZE counters into HBM bytes (written to a temporary
path, never over the committed summary)."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def tiny_batch():
    # DAG 0: 3 nodes, 2 edges; DAG 1: one node, no edge
    return W.from_dags([(3, [0, 1], [1, 2], [4, 5, 6], [1, 2, 3]), (1, [], [], [7], [2])])


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_by_hand():
    b = tiny_batch()
    K = 4
    # explicit: K bytes per node and candidate, 8 per bound, 17 per node, 4 per edge
    assert bench.algorithmic_bytes(b, K) == (K * 3 + 8 * K + 17 * 3 + 4 * 2) + (K * 1 + 8 * K + 17 * 1)
    # seeded candidates move no bytes of their own
    assert bench.algorithmic_bytes(b, K, explicit=False) == (8 * K + 17 * 3 + 4 * 2) + (8 * K + 17)
    # the large-DAG kernel reads its node records (34 B) and 2-byte successor ids
    assert bench.algorithmic_bytes(b, K, explicit=False, large=True) == (8 * K + 34 * 3 + 2 * 2) + (8 * K + 34)
    # comparison bounds: 12 B per node, 2 per edge, 40 per DAG
    assert bench.baselines_bytes(b) == 12 * 4 + 2 * 2 + 40 * 2


def test_algorithmic_bytes_empty_dag():
    b = W.from_dags([(0, [], [], [], [])])
    assert bench.algorithmic_bytes(b, 8) == 8 * 8
    assert bench.baselines_bytes(b) == 40


def _counter_csv(path, name, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": name, "Counter_Value": v})
        # a row of another counter is ignored
        w.writerow({"Kernel_Name": "k_eval<2, true, false, false>", "Counter_Name": "OTHER", "Counter_Value": 1e9})


def test_write_traffic_scaling(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(out))
    copy_kib_fetch = bench.COPY_PROBE_BYTES / 1024 / 2  # the counter reads half the copy's bytes: factor 2
    copy_kib_write = bench.COPY_PROBE_BYTES / 1024      # factor 1
    lib = "void dagbound::(anonymous namespace)::"
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    _counter_csv(fetch, "FETCH_SIZE", [
        ("void at::native::neg_kernel(...)", copy_kib_fetch),
        (lib + "k_eval<2, true, false, false>(dagbound::SweepArgs)", 100.0),
        (lib + "k_eval<2, true, false, false>(dagbound::SweepArgs)", 20.0),  # a second dispatch adds
        (lib + "k_eval_init(dagbound::SweepArgs)", 30.0),
        (lib + "k_prep<2>(dagbound::Tables)", 5000.0),                       # not an evaluation kernel
    ])
    _counter_csv(write, "WRITE_SIZE", [
        ("void at::native::neg_kernel(...)", copy_kib_write),
        (lib + "k_eval<1, true, false, false>(dagbound::SweepArgs)", 10.0),
    ])
    assert bench.write_traffic(str(fetch), str(write), wk=2) == 0
    rec = json.load(open(out))["batched-layered/100000x64"]
    assert rec["counters"]["FETCH_SIZE"]["bytes_per_kib"] == pytest.approx(2.0)
    assert rec["counters"]["FETCH_SIZE"]["kernels_kib"] == {"k_eval<2, true, false, false>": 120.0,
                                                            "k_eval_init": 30.0}
    assert rec["fetch_bytes"] == pytest.approx(150 * 1024 * 2.0)
    assert rec["write_bytes"] == pytest.approx(10 * 1024 * 1.0)
    assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
    assert rec["source_hash"] == bench.sweep_source_hash()
    # read back only for its own workload and kernel source
    assert bench.measured_traffic("batched-layered/100000x64") == pytest.approx(rec["bytes_per_launch"])
    assert bench.measured_traffic("batched-layered/1000x64") is None
    assert "--workload batched-layered" in rec["commands"][0]
    # a second workload's summary is kept beside the first
    assert bench.write_traffic(str(fetch), str(write), wk=3, dags=1000) == 0
    allrec = json.load(open(out))
    assert set(allrec) == {"batched-layered/100000x64", "persistent-mixed/1000x256"}
    assert bench.measured_traffic("persistent-mixed/1000x256") == pytest.approx(rec["bytes_per_launch"])
    allrec["batched-layered/100000x64"]["source_hash"] = "0" * 16
    json.dump(allrec, open(out, "w"))
    assert bench.measured_traffic("batched-layered/100000x64") is None


def test_write_traffic_needs_the_copy(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILE_TRAFFIC", str(tmp_path / "traffic.json"))
    fetch = tmp_path / "fetch.csv"
    _counter_csv(fetch, "FETCH_SIZE", [("dagbound k_eval<1, true, false, false>", 1.0)])
    with pytest.raises(SystemExit):
        bench.write_traffic(str(fetch), str(fetch), wk=2)
    assert not (tmp_path / "traffic.json").exists()


def test_committed_traffic_summary_is_consistent():
    # each committed summary's total is the sum of its scaled counters, and
    # the scale factors are those of a plain copy (2 for reads, 1 for writes)
    if not os.path.exists(bench.PROFILE_TRAFFIC):
        pytest.skip("no traffic summary committed")
    for key, rec in json.load(open(bench.PROFILE_TRAFFIC)).items():
        assert rec["workload"] == key
        for name, want in (("FETCH_SIZE", 2.0), ("WRITE_SIZE", 1.0)):
            c = rec["counters"][name]
            assert c["bytes_per_kib"] == pytest.approx(want, rel=0.01)
            assert c["bytes"] == pytest.approx(sum(c["kernels_kib"].values()) * 1024 * c["bytes_per_kib"])
        assert rec["bytes_per_launch"] == pytest.approx(rec["fetch_bytes"] + rec["write_bytes"])
        assert np.isfinite(rec["bytes_per_launch"]) and rec["bytes_per_launch"] > 0


def test_host_cpu_reports_counts():
    h = bench.host_cpu()
    assert h["os_cpu_count"] >= 1 and h["affinity"] >= 1
    assert isinstance(h["model"], str)


def test_describe_names_the_headline_workload():
    d = bench.describe(3, 1000000, 256, False)
    assert d.startswith("persistent-mixed: 1000000 DAGs") and "256 explicit candidates" in d
