"""GPU multi-index hashing (mih_build / mih_knn through the C ABI) against the
CPU oracle and against MIH-CPU's tables, bit-exact."""
import math

import numpy as np
import pytest

import datagen
import oracle
from oracle import formulas
from gpu_util import as_u32, assert_same, to_dev

pytestmark = pytest.mark.gpu

MODES = [("direct", "inline"), ("direct", "indirect"), ("sorted", "inline"), ("sorted", "indirect"),
         ("grouped", "inline"), ("heads", "inline")]


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def test_build_tables_match_algorithm1(mih):
    # Table j holds the ids ordered by (substring value, id), exactly as
    # MIH-CPU's literal Algorithm 1; offsets are the bucket starts.
    n = 30_001
    codes = datagen.uniform_codes(n, 128, 301)
    ref = oracle.MihCpu(codes, 6)
    for tmode in ["direct", "sorted", "grouped"]:
        idx = mih.build(to_dev(codes), 6, table_mode=tmode, codes_mode="inline")
        info = idx.info()
        assert info["sub_len"] == [22, 22, 21, 21, 21, 21]
        assert info["sub_start"] == [0, 22, 44, 65, 86, 107]
        for j in range(6):
            values, ids = ref.table(j)
            tab = idx.table(j)
            assert np.array_equal(tab["ids"].numpy().view(np.uint32), ids), (tmode, j)
            assert np.array_equal(tab["codes"].numpy().view(np.uint64), codes[ids])
            if tmode == "direct":
                expect = np.searchsorted(values, np.arange((1 << tab["len"]) + 1, dtype=np.uint64))
                assert np.array_equal(tab["offsets"].numpy().view(np.uint32), expect.astype(np.uint32))
                # occupancy map: one bit per bucket, set iff the bucket holds a code
                occupied = np.zeros(1 << tab["len"], dtype=bool)
                occupied[values] = True
                bits = np.unpackbits(tab["occupancy"].numpy().view(np.uint8), bitorder="little")
                assert np.array_equal(bits[: occupied.size].astype(bool), occupied), j
            elif tmode == "grouped":
                # record g: first position of a value >= 32 g, and one bit per
                # value of the group that holds codes
                ng = max((1 << tab["len"]) // 32, 1)
                rec = tab["groups"].numpy().view(np.uint64)
                first = np.searchsorted(values, np.arange(ng, dtype=np.uint64) * 32)
                assert np.array_equal(rec >> np.uint64(32), first.astype(np.uint64)), j
                occupied = np.zeros(ng * 32, dtype=bool)
                occupied[values] = True
                bits = np.unpackbits((rec & np.uint64(0xFFFFFFFF)).astype("<u4").view(np.uint8),
                                     bitorder="little")
                assert np.array_equal(bits.astype(bool), occupied), j
            else:
                assert np.array_equal(tab["keys"].numpy().view(np.uint32), values.astype(np.uint32))
                p = tab["dir_bits"]
                cells = np.arange((1 << p) + 1, dtype=np.uint64) << np.uint64(tab["len"] - p)
                expect = np.searchsorted(values, cells)
                assert np.array_equal(tab["dir"].numpy().view(np.uint32), expect.astype(np.uint32))
        idx.close()
    ref.close()


@pytest.mark.parametrize("tmode,cmode", MODES)
def test_mih_uniform_64_m3_all_modes(mih, tmode, cmode):
    n, nq = 200_003, 50
    codes = datagen.uniform_codes(n, 64, 0)
    queries = datagen.uniform_codes(nq, 64, 1)
    idx = mih.build(to_dev(codes), 3, table_mode=tmode, codes_mode=cmode)
    dq = to_dev(queries)
    for k in [1, 10, 100]:
        ids, dists = idx.knn(dq, k)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"{tmode}/{cmode} k={k}")


@pytest.mark.parametrize("tmode,occ,shift", [("direct", 0, 0), ("direct", 1, 0), ("grouped", 0, 0),
                                              ("direct", 1, 9), ("grouped", 0, 9), ("sorted", 0, 9),
                                              ("heads", 1, 0), ("heads", 1, 9)])
def test_mih_launch_tunings_agree(mih, tmode, occ, shift):
    # Every launch tuning (probes per lane, chunk, occupancy filter, swept
    # steps and their partition size) returns the same exact result and,
    # one step per round, examines the same buckets: a swept step
    # enumerates, per partition of the key space, the masks whose high part
    # the partition fixes.  Running ahead (lookahead) may examine more.
    n, nq, m, k = 150_001, 60, 3, 50
    codes = datagen.uniform_codes(n, 64, 51)
    queries = datagen.uniform_codes(nq, 64, 52)
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode="inline")
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, k)
    lens, _ = formulas.partition(64, m)
    dk = od.reshape(nq, k)[:, -1]
    probes = sum(sum(formulas.shell(lens[t % m], t // m) for t in range(int(d) + 1)) for d in dk)
    # tables with an occupancy map sweep in the partition kernel, whose
    # work items take sweep_queries queries each
    part = shift and occ and tmode in ("direct", "heads")
    for J in (4, 8, 16):
        for chunk in (64 * J * 2, 64 * J * 32):
            for sbits in ((12, 16, 20) if shift else (18,)):
                for look in (1, 16):
                    for sq in ((64, 192, 1024) if part else (256,)):
                        idx.set_tuning(probes_per_lane=J, chunk=chunk, blocks_per_cu=0, occupancy_filter=occ,
                                       sweep_shift=shift, sweep_bits=sbits, lookahead=look, sweep_queries=sq,
                                       small_batch=0)   # device rounds, not the one-launch path
                        ids, dists, st = idx.knn(dq, k, stats=True)
                        what = (f"{tmode} occ={occ} sweep={shift}/{sbits}/{sq} J={J} chunk={chunk} "
                                f"look={look}")
                        assert_same(ids, dists, oi, od, what)
                        if look == 1:
                            assert st["probes"] == probes, what
                        else:
                            assert st["probes"] >= probes, what
    idx.close()


def test_heads_tables_match_algorithm1(mih):
    # HEADS (64-bit codes): entry v holds the offset and size of bucket v
    # and, for a non-empty bucket, its first code in (value, id) order
    n = 40_003
    codes = datagen.uniform_codes(n, 64, 302)
    ref = oracle.MihCpu(codes, 3)
    idx = mih.build(to_dev(codes), 3, table_mode="heads")
    assert idx.info()["table_mode"] == "heads"
    for j in range(3):
        values, ids = ref.table(j)
        tab = idx.table(j)
        heads = tab["heads"].numpy()
        nb = 1 << tab["len"]
        start = np.searchsorted(values, np.arange(nb + 1, dtype=np.uint64)).astype(np.int64)
        assert np.array_equal(heads[:, 1] & 0xFFFFFFFF, start)
        size = np.append(start[1:] - start[:-1], 0)
        assert np.array_equal(heads[:, 1] >> 32, size)
        nonempty = start[1:] > start[:-1]
        first = np.zeros(nb, dtype=np.uint64)
        first[nonempty] = codes[ids[start[:-1][nonempty]], 0]
        assert np.array_equal(heads[:nb, 0].view(np.uint64), first)
    with pytest.raises(mih.MihError):
        mih.build(to_dev(datagen.uniform_codes(100, 128, 303)), 4, table_mode="heads")
    idx.close()
    ref.close()


def test_mih_probe_count_equals_closed_form(mih):
    # Every query examines, for each step t <= d_k, the C(s_a, r') buckets of
    # Eq. 1's shell: the device must enumerate each shell exactly once.
    n, nq, m, k = 100_000, 40, 3, 10
    codes = datagen.uniform_codes(n, 64, 11)
    queries = datagen.uniform_codes(nq, 64, 12)
    idx = mih.build(to_dev(codes), m)
    # one step per round in device rounds: no step runs early
    idx.set_tuning(lookahead=1, small_batch=0)
    ids, dists, st = idx.knn(to_dev(queries), k, stats=True)
    oi, od = oracle.knn(codes, queries, k)
    assert_same(ids, dists, oi, od, "probe count run")
    lens, _ = formulas.partition(64, m)
    dk = od.reshape(nq, k)[:, -1]
    expect = sum(sum(formulas.shell(lens[t % m], t // m) for t in range(int(d) + 1)) for d in dk)
    assert st["probes"] == expect
    assert st["steps"] == int(sum(int(d) + 1 for d in dk))


def test_mih_clustered_128_m6(mih):
    n, nq = 200_000, 64
    codes = datagen.clustered_codes(n, 128, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(nq, 128, datagen.SEED_Q_CLUSTERED)
    idx = mih.build(to_dev(codes), 6)
    dq = to_dev(queries)
    for k in [1, 10, 100]:
        ids, dists = idx.knn(dq, k)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"clustered k={k}")


@pytest.mark.parametrize("bits,m,kind", [(256, 8, "clustered"), (256, 16, "uniform"),
                                          (192, 12, "uniform"), (128, 4, "clustered")])
def test_mih_long_codes(mih, bits, m, kind):
    n, nq = 60_000, 24
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    for tmode, cmode in [("direct", "indirect"), ("sorted", "inline"), ("grouped", "inline")]:
        idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode=cmode)
        ids, dists = idx.knn(to_dev(queries), 10)
        oi, od = oracle.knn(codes, queries, 10)
        assert_same(ids, dists, oi, od, f"{bits}/{m}/{kind}/{tmode}/{cmode}")
        idx.close()


def test_mih_per_query_k_and_k_beyond_n(mih):
    codes = datagen.uniform_codes(300, 64, 21)
    queries = datagen.uniform_codes(7, 64, 22)
    ks = np.array([0, 1, 300, 310, 7, 0, 299], dtype=np.uint32)
    idx = mih.build(to_dev(codes), 4)
    ids, dists = idx.knn(to_dev(queries), ks.tolist())
    oi, od = oracle.knn(codes, queries, ks)
    assert_same(ids, dists, oi, od, "per-query k")


@pytest.mark.parametrize("tmode", ["auto", "grouped", "heads"])
def test_mih_duplicates_overflow_rerun(mih, tmode):
    # 5000 copies of one code: the query equal to it finds them all in one
    # bucket; the buffer (2048) overflows and the query is re-run exactly.
    # In a GROUPED table the group scan walks past long runs of equal values.
    base = datagen.uniform_codes(4, 64, 31)
    codes = np.concatenate([np.repeat(base[:1], 5000, axis=0), datagen.uniform_codes(3000, 64, 32),
                            np.repeat(base[2:3] ^ np.uint64(1), 37, axis=0)])
    queries = np.concatenate([base[:1], base[1:2], base[:1] ^ np.uint64(3), base[2:3]])
    idx = mih.build(to_dev(codes), 3, table_mode=tmode)
    reruns = 0
    for k in [1, 100, 4096]:
        ids, dists, st = idx.knn(to_dev(queries), k, stats=True)
        oi, od = oracle.knn(codes, queries, k)
        assert_same(ids, dists, oi, od, f"duplicates k={k}")
        reruns += st["reruns"]
    assert reruns >= 1


def test_mih_empty_database_and_no_queries(mih):
    import torch
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    idx = mih.build(empty, 2)
    q = to_dev(datagen.uniform_codes(3, 64, 2))
    ids, dists = idx.knn(q, 4)
    assert (ids.cpu() == -1).all() and (dists.cpu() == -1).all()
    idx2 = mih.build(to_dev(datagen.uniform_codes(50, 64, 3)), 2)
    ids, dists = idx2.knn(empty, 4)
    assert ids.numel() == 0


def test_mih_matches_linscan_mixed_k(mih):
    n, nq = 300_000, 200
    codes = datagen.uniform_codes(n, 64, 41)
    queries = datagen.uniform_codes(nq, 64, 42)
    ks = datagen.choice_u32(nq, (1, 10, 100, 1000), datagen.SEED_K)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, 3)
    ids, dists = idx.knn(dq, ks.tolist())
    li, ld = mih.linscan_knn(dc, dq, ks.tolist())
    assert np.array_equal(as_u32(ids), as_u32(li)) and np.array_equal(as_u32(dists), as_u32(ld))
    sel = np.arange(0, nq, 10)
    oi, od = oracle.knn(codes, queries[sel], ks[sel])
    off = np.concatenate([[0], np.cumsum(ks.astype(np.int64))])
    gi = np.concatenate([as_u32(ids)[off[i]:off[i + 1]] for i in sel])
    gd = np.concatenate([as_u32(dists)[off[i]:off[i + 1]] for i in sel])
    assert np.array_equal(gi, oi) and np.array_equal(gd, od)


def test_partition_sweep_of_a_group_larger_than_65536_queries(mih):
    # a swept step of more than 65,536 queries at once: the partition
    # kernel's work items index their queries within the item
    import torch
    n, nq = 300_007, 70_000
    codes = datagen.uniform_codes(n, 64, 961)
    queries = datagen.uniform_codes(nq, 64, 962)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, 3, table_mode="heads", codes_mode="inline")
    idx.set_tuning(probes_per_lane=4, chunk=256, occupancy_filter=1, sweep_shift=6, sweep_bits=16,
                   sweep_queries=4096, small_batch=0)
    ids, dists, st = idx.knn(dq, 3, stats=True)
    li, ld = mih.linscan_knn(dc, dq, 3)
    assert torch.equal(ids, li) and torch.equal(dists, ld)
    sel = np.arange(nq - 300, nq)
    oi, od = oracle.knn(codes, queries[sel], 3)
    assert_same(ids.reshape(nq, 3)[sel[0]:].reshape(-1), dists.reshape(nq, 3)[sel[0]:].reshape(-1), oi, od,
                "last queries of the group")
    idx.close()
