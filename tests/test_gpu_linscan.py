"""GPU linear scan (linscan_knn through the C ABI) against the CPU oracle,
element by element, ids and distances bit-exact."""
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


@pytest.mark.parametrize("bits", [64, 128, 192, 256])
def test_linscan_uniform_all_word_counts(mih, bits):
    n, nq = 20_011, 37                       # several register blocks plus a ragged tail
    codes = datagen.uniform_codes(n, bits, 100 + bits)
    queries = datagen.uniform_codes(nq, bits, 200 + bits)
    dc, dq = to_dev(codes), to_dev(queries)
    for k in [1, 10, 100, 1000]:
        ids, dists = mih.linscan_knn(dc, dq, k)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"bits={bits} k={k}")


def test_linscan_clustered_128(mih):
    codes = datagen.clustered_codes(50_000, 128, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(64, 128, datagen.SEED_Q_CLUSTERED)
    ids, dists = mih.linscan_knn(to_dev(codes), to_dev(queries), 100)
    oi, od = oracle.knn(codes, queries, 100)
    assert_same(ids, dists, oi, od, "clustered")


def test_linscan_per_query_k_zero_and_beyond_n(mih):
    codes = datagen.uniform_codes(57, 64, 7)
    queries = datagen.uniform_codes(6, 64, 8)
    ks = [0, 1, 57, 60, 3, 0]
    ids, dists = mih.linscan_knn(to_dev(codes), to_dev(queries), ks)
    oi, od = oracle.knn(codes, queries, np.array(ks, dtype=np.uint32))
    assert_same(ids, dists, oi, od, "per-query k")


def test_linscan_ties_overflow_rerun(mih):
    # 9000 identical codes: every code ties, the candidate buffer (4096 for
    # k <= 256) overflows and the query is re-run with an exact capacity
    base = datagen.uniform_codes(3, 128, 9)
    codes = np.concatenate([np.repeat(base[:1], 9000, axis=0), base[1:]], axis=0)
    queries = np.concatenate([base[:1], base[1:2] ^ np.uint64(5)], axis=0)
    for k in [1, 100, 4096]:
        ids, dists = mih.linscan_knn(to_dev(codes), to_dev(queries), k)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"ties k={k}")


def test_linscan_empty_inputs(mih):
    import torch
    codes = datagen.uniform_codes(100, 64, 1)
    q = datagen.uniform_codes(3, 64, 2)
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    ids, dists = mih.linscan_knn(empty, to_dev(q), 5)
    assert (ids.cpu() == -1).all() and (dists.cpu() == -1).all()
    ids, dists = mih.linscan_knn(to_dev(codes), empty, 5)
    assert ids.numel() == 0


def test_linscan_rejects_large_k(mih):
    codes = datagen.uniform_codes(10, 64, 1)
    with pytest.raises(mih.MihError):
        mih.linscan_knn(to_dev(codes), to_dev(codes[:1]), 5000)
