"""MIXED codes: the first tables keep their codes in table order, the others
read candidates through the ids.  Results equal the oracle's for every
split, the table views show which tables hold codes, and under a memory
budget the AUTO mode keeps as many inline tables as fit."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import as_u32, assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


@pytest.mark.parametrize("bits,m,kind,tmode", [(64, 4, "uniform", "direct"), (128, 6, "clustered", "sorted"),
                                               (256, 12, "clustered", "direct")])
def test_mixed_codes_knn_and_rnn(mih, bits, m, kind, tmode):
    n, nq = 80_003, 24
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    queries[0] = codes[5]
    dc, dq = to_dev(codes), to_dev(queries)
    ks = np.array([1, 10, 100, 0, 4096] * 5, dtype=np.uint32)[:nq]
    oi, od = oracle.knn(codes, queries, ks)
    r = bits // 8
    ref = [oracle.rnn(codes, queries[i], r) for i in range(nq)]
    for inl in (1, m // 2, m - 1):
        idx = mih.build(dc, m, table_mode=tmode, codes_mode="mixed", inline_tables=inl)
        inf = idx.info()
        assert inf["codes_mode"] == "mixed" and inf["inline_tables"] == inl
        for j in range(m):
            assert (idx.table(j).get("codes") is not None) == (j < inl), j
        for look in (1, 16):
            idx.set_tuning(lookahead=look)
            ids, dists = idx.knn(dq, ks.tolist())
            assert_same(ids, dists, oi, od, f"{bits}/{m}/{tmode} inline={inl} look={look}")
        off, rid, rdist = idx.rnn(dq, r)
        off = off.cpu().numpy()
        gi, gd = as_u32(rid), as_u32(rdist)
        for i in range(nq):
            a, b = int(off[i]), int(off[i + 1])
            assert np.array_equal(gi[a:b], ref[i][0]) and np.array_equal(gd[a:b], ref[i][1]), (inl, i)
        idx.close()


def test_mixed_codes_arguments(mih):
    codes = to_dev(datagen.uniform_codes(1000, 64, 31))
    for bad in (0, 4, 5):
        with pytest.raises(mih.MihError):
            mih.build(codes, 4, codes_mode="mixed", inline_tables=bad)
    for tmode in ("grouped", "heads"):
        with pytest.raises(mih.MihError):
            mih.build(codes, 4, table_mode=tmode, codes_mode="mixed", inline_tables=2)


def test_auto_codes_fill_the_budget(mih):
    # as the memory budget grows, AUTO keeps 0, then some, then all tables'
    # codes inline, and every split answers exactly
    n, m = 200_000, 4
    codes = datagen.uniform_codes(n, 64, 32)
    queries = datagen.uniform_codes(16, 64, 33)
    dc, dq = to_dev(codes), to_dev(queries)
    oi, od = oracle.knn(codes, queries, 20)
    seen = {}
    last = -1
    for mb in np.arange(4.0, 64.0, 0.5):
        try:
            idx = mih.build(dc, m, table_mode="sorted", mem_budget_bytes=int(mb * 2**20))
        except mih.MihError:
            continue
        k_in = idx.info()["inline_tables"]
        assert k_in >= last, (mb, k_in, last)
        last = k_in
        if k_in not in seen:
            seen[k_in] = mb
            ids, dists = idx.knn(dq, 20)
            assert_same(ids, dists, oi, od, f"budget {mb} MiB, {k_in} inline tables")
        idx.close()
    assert 0 in seen and m in seen and any(0 < k < m for k in seen), seen
