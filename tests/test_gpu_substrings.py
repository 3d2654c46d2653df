"""Substring optimisation on the GPU: bit co-occurrence counts on the matrix
cores against the oracle's integer counts, and multi-index search over
tables built with an optimised bit order against the kNN and r-neighbour
oracles (results never depend on the order)."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import formulas
from oracle import substrings as S
from gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


@pytest.mark.parametrize("bits,n,kind", [(64, 70_001, "uniform"), (128, 70_001, "clustered"),
                                         (192, 1_000, "uniform"), (256, 131_075, "clustered"),
                                         (128, 0, "uniform"), (64, 15, "clustered")])
def test_cooccurrence_counts(mih, bits, n, kind):
    # several slices of 65536 samples and a ragged tail; empty and tiny sets
    codes = datagen.db_codes(kind, n, bits) if n else np.zeros((0, bits // 64), dtype=np.uint64)
    got = mih.bit_cooccurrence(to_dev(codes))
    want = S.cooccurrence(codes)
    assert np.array_equal(got.astype(np.int64), want), f"{bits}/{n}/{kind}"


@pytest.mark.parametrize("bits,m,tmode,cmode", [(128, 6, "direct", "inline"), (128, 6, "sorted", "indirect"),
                                                (256, 8, "sorted", "inline"), (64, 3, "grouped", "inline")])
def test_knn_with_optimised_substrings(mih, bits, m, tmode, cmode):
    n, nq = 120_000, 48
    kind = "uniform" if bits == 64 else "clustered"
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    dc, dq = to_dev(codes), to_dev(queries)
    order = mih.optimize_substrings(dc, m, sample=50_000, first_bit=1)
    assert order == S.greedy_bit_order(S.cooccurrence(codes[:50_000]), 50_000, bits, m, 1)
    idx = mih.build(dc, m, table_mode=tmode, codes_mode=cmode, bit_order=order)
    idx.set_tuning(lookahead=1, small_batch=0)   # one step per device round, for the probe count below
    assert idx.info()["bit_order"] == order
    for k in (1, 10, 100):
        ids, dists, st = idx.knn(dq, k, stats=True)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"{bits}/{m}/{tmode}/{cmode} k={k}")
        # the tables have the same lengths, so each step examines C(s_a, r') buckets
        lens, _ = formulas.partition(bits, m)
        dk = od.reshape(nq, k)[:, -1]
        assert st["probes"] == sum(sum(formulas.shell(lens[t % m], t // m) for t in range(int(d) + 1))
                                   for d in dk)
    r = bits // 8
    off, rid, rdist = idx.rnn(dq, r)
    for i in range(0, nq, 12):
        oi, od = oracle.rnn(codes, queries[i], r)
        a, b = int(off[i]), int(off[i + 1])
        assert np.array_equal(rid[a:b].cpu().numpy().view(np.uint32), oi)
        assert np.array_equal(rdist[a:b].cpu().numpy().view(np.uint32), od)


def test_bit_order_is_validated(mih):
    codes = to_dev(datagen.uniform_codes(100, 64, 92))
    bad = list(range(64))
    bad[5] = 4                      # not a permutation
    with pytest.raises(mih.MihError):
        mih.build(codes, 2, bit_order=bad)
