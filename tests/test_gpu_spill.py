"""Buckets holding more codes than the tuning's spill_codes are cut into
pieces of 1024 codes that any wave of the round kernel may walk (waves out
of work items take them first; the wave that met the bucket takes the rest).
Results must equal the oracle's with and without spilling, in every table
and codes mode, on codes with huge buckets."""
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


def heavy_codes(n, bits, seed):
    # clustered codes plus runs of repeated codes and of codes that share
    # all substrings but one: buckets of thousands of codes in every table
    codes = datagen.clustered_codes(n, bits, seed)
    base = datagen.uniform_codes(8, bits, seed + 1)
    reps = np.repeat(base, 1500, axis=0)
    flip = datagen.uniform_codes(len(reps), bits, seed + 2)
    # every other copy exact (a bucket of 750 codes in every table), the rest
    # with a few bits of the last word flipped
    reps[1::2, -1] ^= flip[1::2, -1] & np.uint64(0x0101010101010101)
    return np.concatenate([codes, reps], axis=0)


@pytest.mark.parametrize("bits,m,tmode,cmode,inl", [(64, 3, "direct", "inline", 0),
                                                    (64, 3, "heads", "inline", 0),
                                                    (64, 4, "grouped", "inline", 0),
                                                    (64, 3, "sorted", "indirect", 0),
                                                    (128, 4, "sorted", "inline", 0),
                                                    (128, 6, "direct", "indirect", 0),
                                                    (256, 8, "sorted", "mixed", 5)])
def test_spilled_buckets_equal_oracle(mih, bits, m, tmode, cmode, inl):
    codes = heavy_codes(60_001, bits, 700 + bits)
    n = len(codes)
    nq = 48
    queries = np.concatenate([codes[n - 12000:n:1000], datagen.clustered_codes(nq - 12, bits, 800 + bits)])
    ks = datagen.choice_u32(nq, [1, 10, 100, 1000], 33)
    oi, od = oracle.knn(codes, queries, ks)
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode=cmode, inline_tables=inl)
    dq = to_dev(queries)
    for spill in (0, 256, 4096):
        for look in (1, 16):
            idx.set_tuning(spill_codes=spill, small_batch=0, lookahead=look)
            ids, dists = idx.knn(dq, ks.tolist())
            assert_same(ids, dists, oi, od, f"{bits}/{m}/{tmode}/{cmode} spill={spill} lookahead={look}")
    idx.close()


def test_spill_with_r_neighbours_and_small_lookahead(mih):
    codes = heavy_codes(40_003, 64, 901)
    queries = np.concatenate([codes[-3000::600], datagen.clustered_codes(20, 64, 902)])
    idx = mih.build(to_dev(codes), 3)
    dq = to_dev(queries)
    for look in (1, 16):
        idx.set_tuning(spill_codes=256, small_batch=0, lookahead=look)
        ids, dists = idx.knn(dq, 50)
        oi, od = oracle.knn(codes, queries, 50)
        assert_same(ids, dists, oi, od, f"lookahead {look}")
        off, rid, rd = idx.rnn(dq, 9)
        from gpu_util import as_u32
        for i in range(len(queries)):
            a, b = int(off[i]), int(off[i + 1])
            ri, rdd = oracle.rnn(codes, queries[i], 9)
            assert np.array_equal(as_u32(rid[a:b]), ri) and np.array_equal(as_u32(rd[a:b]), rdd), i
    idx.close()


def test_spill_codes_is_validated(mih):
    codes = datagen.uniform_codes(1000, 64, 903)
    idx = mih.build(to_dev(codes), 2)
    with pytest.raises(Exception):
        idx.set_tuning(spill_codes=100)
    idx.set_tuning(spill_codes=0)
    idx.set_tuning(spill_codes=256)
    idx.close()


def test_round_tail_statistic_is_within_the_search_time(mih):
    # tail_ms: per round, first to last wave of the round kernel running out
    # of work items, summed; it cannot exceed the rounds' event time
    codes = heavy_codes(50_001, 64, 905)
    queries = datagen.clustered_codes(300, 64, 906)
    idx = mih.build(to_dev(codes), 3)
    for spill in (0, 1024):
        idx.set_tuning(spill_codes=spill, small_batch=0)
        _, _, st = idx.knn(to_dev(queries), 20, stats=True)
        assert 0.0 <= st["tail_ms"] <= st["search_kernel_ms"] + 0.05, st
    idx.close()
