"""Host logic of bench.py: request-weighted percentiles, the committed
counter record and its staleness checks, workload overrides and the one-GPU
rule.  No GPU needed."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def nearest_rank(values, weights, q):
    # the definition: expand every value by its weight, sort, take rank
    # ceil(q/100 N) (1-based, at least 1)
    e = np.sort(np.repeat(np.asarray(values, dtype=np.float64), weights), kind="stable")
    r = max(1, int(np.ceil(q / 100.0 * len(e))))
    return float(e[r - 1])


@pytest.mark.parametrize("seed", range(20))
def test_weighted_percentile_is_the_nearest_rank_of_the_expanded_list(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 60))
    a = rng.integers(0, 30, size=n).astype(np.float64)    # ties on purpose
    w = rng.integers(1, 9, size=n)
    for q in (0, 1, 25, 50, 90, 99, 100):
        assert bench.weighted_pct(a, w, q) == nearest_rank(a, w, q), (seed, q)
    assert bench.weighted_pct([], [], 50) is None
    # unit weights: the plain nearest-rank percentile
    assert bench.weighted_pct(a, np.ones(n, dtype=int), 50) == nearest_rank(a, np.ones(n, dtype=int), 50)


def test_counter_record_checks(tmp_path, monkeypatch):
    # a counter record of a made-up kernel source: traffic only while the
    # source and the table/codes modes match and a record has the tuning
    import hashlib
    (tmp_path / "profiles").mkdir()
    (tmp_path / "k.hip").write_bytes(b"kernel source")
    r1 = {"tuning": {"probes_per_lane": 8, "chunk": 16384}, "launches": 2,
          "fetch_kib_per_launch": [10.0, 30.0], "write_kib_per_launch": [1.0, 3.0]}
    r2 = {"tuning": {"probes_per_lane": 4, "chunk": 8192}, "launches": 2,
          "fetch_kib_per_launch": [5.0, 5.0], "write_kib_per_launch": [1.0, 1.0]}
    rec = {"sources": ["k.hip"],
           "source_sha256_16": hashlib.sha256(b"kernel source").hexdigest()[:16],
           "modes": ["heads", "inline"],
           "copy_calibration": {"fetch_factor": 2.0, "write_factor": 1.0},
           "random_line_calibration": {"fetch_factor": 1.01},
           "records": [r1, r2]}
    (tmp_path / "profiles" / "c.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    tuning = {"probes_per_lane": 8, "chunk": 16384, "sweep_bits": 18}
    traffic, got = bench.counter_traffic("c.json", tuning, ("heads", "inline"))
    # random reads scale by the random-line calibration, writes by the copy's
    assert traffic == (20.0 * 1.01 + 2.0 * 1.0) * 1024.0 and got == r1
    traffic, got = bench.counter_traffic("c.json", dict(tuning, probes_per_lane=4, chunk=8192),
                                         ("heads", "inline"))
    assert traffic == (5.0 * 1.01 + 1.0) * 1024.0 and got == r2
    assert bench.counter_traffic("c.json", dict(tuning, chunk=4096), ("heads", "inline"))[0] is None
    assert bench.counter_traffic("c.json", tuning, ("direct", "inline"))[0] is None
    (tmp_path / "k.hip").write_bytes(b"kernel source, changed")
    assert bench.counter_traffic("c.json", tuning, ("heads", "inline"))[0] is None
    assert bench.counter_traffic("missing.json", tuning, ("heads", "inline")) == (None, None)


def test_committed_counter_record_is_complete():
    path = os.path.join(ROOT, "profiles", "mih_search_1e9x64_m2_k100_counters.json")
    rec = json.load(open(path))
    for key in ("sources", "source_sha256_16", "modes", "copy_calibration", "random_line_calibration",
                "records", "commands"):
        assert key in rec, key
    for r in rec["records"]:
        assert len(r["fetch_kib_per_launch"]) == len(r["write_kib_per_launch"]) == r["launches"]
        assert r["tuning"]
    for src in rec["sources"]:
        assert os.path.exists(os.path.join(ROOT, src)), src


def test_search_roofline_counts_the_survey_bytes():
    # 8 B per probe, 4 B id + bits/8 B code per candidate, bits/8 B per
    # query and 8 B per output entry, over the rounds' event time
    st = {"probes": 1000, "candidates": 300, "search_kernel_ms": 2.0, "search_launches": 4}
    info = {"table_mode": "heads", "codes_mode": "inline"}
    k_list = np.full(10, 7, dtype=np.uint32)
    r = bench.search_roofline(st, info, 12345, 128, 4, 10, (7,), k_list, 2, {})
    alg = 1000 * 8 + 300 * (4 + 16) + 10 * 16 + 70 * 8
    assert r["alg_bytes_per_step"] == alg and r["alg_bytes_per_launch"] == alg // 4
    assert r["achieved"] == round(alg / 2e-3 / 1e9, 1) and r["frac"] == round(alg / 2e-3 / 1e9 / 8000.0, 4)
    assert r["traffic"] is None and r["random_lines"] is None
    r2 = bench.search_roofline(st, dict(info, table_mode="sorted"), 12345, 128, 4, 10, (7,), k_list, 2, {})
    assert r2["alg_bytes_per_step"] == alg + 1000 * 4


def test_workload_overrides():
    sys_argv = sys.argv
    try:
        sys.argv = ["bench.py", "--config", "3", "--n", "1000", "--nq", "7", "--k", "5", "--m", "4"]
        args = bench.parse()
    finally:
        sys.argv = sys_argv
    cfg = bench.workload(args)
    assert (cfg["n"], cfg["nq"], cfg["m"], tuple(cfg["ks"])) == (1000, 7, 4, (5,))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
