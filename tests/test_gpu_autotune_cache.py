"""The autotune cache of mih_build_opts: the first autotune of an index
shape and sample times the grid and stores the tuning in the file, a later
one (another index of the same shape) takes it from the file without
timing; another k is another entry; results do not depend on it."""
import json
import time

import numpy as np
import pytest

import datagen
import oracle
from gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def test_autotune_cache_stores_and_reuses(mih, tmp_path):
    path = str(tmp_path / "tuned.json")
    codes = datagen.uniform_codes(120_001, 64, 971)
    queries = datagen.uniform_codes(600, 64, 972)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, 3, autotune_cache=path)
    t0 = time.perf_counter()
    first = idx.autotune(dq, 10)
    t_first = time.perf_counter() - t0
    entries = json.load(open(path))
    assert len(entries) == 1
    (key, fields), = entries.items()
    assert "n=120001" in key and "queries=600" in key and "k=10" in key
    assert fields == list(first.values())
    idx.close()
    # another index of the same shape: the tuning comes from the file
    idx = mih.build(dc, 3, autotune_cache=path)
    idx.set_tuning(probes_per_lane=16, chunk=1024 * 16)
    t0 = time.perf_counter()
    second = idx.autotune(dq, 10)
    t_second = time.perf_counter() - t0
    assert idx.get_tuning() == json_tuning(fields, idx.get_tuning())
    assert t_second < t_first
    ids, dists = idx.knn(dq, 10)
    oi, od = oracle.knn(codes, queries, 10)
    assert_same(ids, dists, oi, od, "with the cached tuning")
    # per-query k: a second entry
    ks = datagen.choice_u32(600, [1, 10, 100], 973)
    idx.autotune(dq, ks.tolist())
    assert len(json.load(open(path))) == 2
    idx.close()


def json_tuning(fields, like):
    return dict(zip(like.keys(), fields))


def test_autotune_cache_unreadable_file_counts_as_empty(mih, tmp_path):
    path = tmp_path / "bad.json"
    path.write_text("not json at all\n[1, 2]\n")
    codes = datagen.uniform_codes(50_003, 64, 974)
    idx = mih.build(to_dev(codes), 3, autotune_cache=str(path))
    idx.autotune(to_dev(datagen.uniform_codes(100, 64, 975)), 5)
    assert len(json.load(open(path))) == 1
    idx.close()
