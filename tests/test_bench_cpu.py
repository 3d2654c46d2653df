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


def test_counter_record_and_its_checks():
    path = os.path.join(ROOT, "profiles", "mih_round_kernel_1e9x64_m2_k100_counters.json")
    rec = json.load(open(path))
    tuning = dict(rec["tuning"], sweep_bits=18)
    modes = tuple(rec["modes"])
    traffic, got = bench.counter_traffic(os.path.basename(path), tuning, modes)
    # the committed counters were taken from the committed kernel source
    assert traffic is not None and got["source_sha256_16"] == rec["source_sha256_16"]
    cal = rec["copy_calibration"]
    expect = (np.mean(rec["fetch_kib_per_launch"]) * cal["fetch_factor"] +
              np.mean(rec["write_kib_per_launch"]) * cal["write_factor"]) * 1024.0
    assert traffic == pytest.approx(expect, rel=1e-12)
    # another launch tuning, or other table/codes modes: no traffic figure
    other = dict(tuning, chunk=tuning["chunk"] * 2)
    assert bench.counter_traffic(os.path.basename(path), other, modes)[0] is None
    assert bench.counter_traffic(os.path.basename(path), tuning, ("direct", "inline"))[0] is None
    assert bench.counter_traffic("no_such_counters.json", tuning, modes) == (None, None)


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
