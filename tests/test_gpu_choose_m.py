"""Choosing m by timing on validation queries (mih_choose_m through the C
ABI): every candidate is built and timed, the fastest is returned, and an
index with the chosen m answers exactly."""
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


def test_choose_m_default_candidates(mih):
    n = 1_000_000
    codes = datagen.uniform_codes(n, 64, 81)
    dc = to_dev(codes)
    best, trials = mih.choose_m(dc, 10, validation=300, seed=5)
    ms = [t["m"] for t in trials]
    # 64 / log2(1e6) = 3.2: candidates 2, 3, 4 (the model's minimum is among them)
    assert ms == [2, 3, 4]
    assert all(t["status"] == "ok" and t["search_ms"] > 0 for t in trials)
    assert best == min(trials, key=lambda t: t["search_ms"])["m"]
    assert min(trials, key=lambda t: t["model_cost"])["m"] in ms
    # the chosen m answers exactly
    queries = datagen.uniform_codes(40, 64, 82)
    idx = mih.build(dc, best)
    ids, dists = idx.knn(to_dev(queries), 10)
    oi, od = oracle.knn(codes, queries, 10)
    assert_same(ids, dists, oi, od, f"m={best}")


def test_choose_m_given_candidates_and_queries(mih):
    codes = datagen.clustered_codes(200_000, 128, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(100, 128, datagen.SEED_Q_CLUSTERED)
    best, trials = mih.choose_m(to_dev(codes), 20, queries=to_dev(queries), candidates=[5, 6, 8],
                                table_mode="sorted")
    assert [t["m"] for t in trials] == [5, 6, 8]
    assert best in (5, 6, 8)
    assert all(t["status"] == "ok" for t in trials)
