"""The one-launch search of small batches (a workgroup per query runs every
step of Algorithm 3 and writes the top-k rows, with no host round trip)
against the oracle, bit-exact, in every table and codes mode, and against
the device rounds on the same queries; queries whose buffer overflows are
re-run exactly by the rounds."""
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


# The one-launch path is taken when the expected probes per query (uniform
# codes, model radius of the largest k) are few; longer codes and clustered
# sets with few tables are left to the rounds (the last cases), whose
# result must be the same.
@pytest.mark.parametrize("bits,m,kind,tmode,cmode,one", [(64, 3, "uniform", "direct", "inline", True),
                                                         (64, 3, "uniform", "heads", "inline", True),
                                                         (64, 3, "uniform", "direct", "indirect", True),
                                                         (64, 4, "uniform", "grouped", "inline", True),
                                                         (64, 3, "clustered", "sorted", "inline", True),
                                                         (128, 8, "uniform", "direct", "mixed", True),
                                                         (128, 6, "clustered", "sorted", "inline", False),
                                                         (256, 11, "clustered", "sorted", "indirect", False)])
def test_small_batch_equals_oracle_and_rounds(mih, bits, m, kind, tmode, cmode, one):
    n, nq = 150_001, 97
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    queries[3] = codes[777]          # a query equal to a database code
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode=cmode, inline_tables=2)
    dq = to_dev(queries)
    ks = datagen.choice_u32(nq, [1, 10, 100], 31)
    ks[7] = 0
    oi, od = oracle.knn(codes, queries, ks)
    idx.set_tuning(small_batch=512)
    ids, dists, st = idx.knn(dq, ks.tolist(), stats=True)
    what = f"{bits}/{m}/{tmode}/{cmode}"
    assert_same(ids, dists, oi, od, what + " one launch")
    if one:
        assert st["rounds"] == 1 and st["search_launches"] == 1 and st["reruns"] == 0, st
    idx.set_tuning(small_batch=0)
    ri, rd, rst = idx.knn(dq, ks.tolist(), stats=True)
    assert_same(ri, rd, oi, od, what + " rounds")
    # the same steps: exact searches of both paths stop after step d_k
    assert st["steps"] <= rst["steps"]
    idx.close()


def test_small_batch_probe_count_is_the_shells(mih):
    # every step t <= d_k of every query probes C(s_a, t / m) buckets (Eq. 1);
    # the workgroups of a query may run a step or two past the stop step
    # before the flag reaches them, so those add probes but not steps
    from oracle import formulas
    n, nq, m, k = 80_021, 33, 3, 20
    codes = datagen.uniform_codes(n, 64, 611)
    queries = datagen.uniform_codes(nq, 64, 612)
    idx = mih.build(to_dev(codes), m)
    ids, dists, st = idx.knn(to_dev(queries), k, stats=True)
    oi, od = oracle.knn(codes, queries, k)
    assert_same(ids, dists, oi, od, "probe count")
    lens, _ = formulas.partition(64, m)
    dk = od.reshape(nq, k)[:, -1]
    assert st["probes"] >= sum(sum(formulas.shell(lens[t % m], t // m) for t in range(int(d) + 1)) for d in dk)
    assert st["steps"] == int(np.sum(dk.astype(np.int64) + 1))
    assert st["rounds"] == 1
    idx.close()


def test_small_batch_overflow_goes_to_the_rounds(mih):
    # 9000 copies of one code: queries near it overflow their buffers in the
    # one launch and are re-run exactly by the device rounds
    base = datagen.uniform_codes(2000, 64, 621)
    codes = np.concatenate([np.repeat(base[:1], 9000, axis=0), base[1:]], axis=0)
    queries = np.concatenate([base[:1], base[5:9], base[:1] ^ np.uint64(3)], axis=0)
    idx = mih.build(to_dev(codes), 4)
    dq = to_dev(queries)
    for k in (1, 100, 4096):
        ids, dists, st = idx.knn(dq, k, stats=True)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"ties k={k}")
        if k <= 256:
            # buffers of 2048 entries cannot hold 9000 codes at distance 0
            assert st["reruns"] >= 1 and st["rounds"] >= 2, (k, st)
    idx.close()


def test_small_batch_k_beyond_n_and_empty(mih):
    import torch
    codes = datagen.uniform_codes(57, 64, 631)
    queries = datagen.uniform_codes(6, 64, 632)
    idx = mih.build(to_dev(codes), 3)
    ks = [0, 1, 57, 60, 3, 0]
    ids, dists = idx.knn(to_dev(queries), ks)
    oi, od = oracle.knn(codes, queries, np.array(ks, dtype=np.uint32))
    assert_same(ids, dists, oi, od, "k beyond n")
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    ids, dists = idx.knn(empty, 5)
    assert ids.numel() == 0
    idx.close()


def test_small_batch_then_large_batch_share_the_index(mih):
    n = 200_003
    codes = datagen.uniform_codes(n, 64, 641)
    idx = mih.build(to_dev(codes), 3)
    for nq in (16, 700, 3, 2000, 40):
        queries = datagen.uniform_codes(nq, 64, 642, first_row=nq)
        ids, dists = idx.knn(to_dev(queries), 10)
        oi, od = oracle.knn(codes, queries, 10)
        assert np.array_equal(as_u32(ids), oi) and np.array_equal(as_u32(dists), od), nq
    idx.close()
