"""Pins for the CPU oracle (plain kNN definition, Section 1.1).

The oracle is checked against things other than itself: an independent
pure-Python brute force, numpy's popcount + lexsort, and closed-form cases
whose answers follow from the definition by hand.
"""
import numpy as np
import pytest

import datagen
import oracle

SENT = 0xFFFFFFFF


def rows(ids, dists, ks):
    off = 0
    out = []
    for k in ks:
        out.append((ids[off:off + k].tolist(), dists[off:off + k].tolist()))
        off += k
    return out


@pytest.mark.parametrize("bits", [64, 128, 192, 256])
@pytest.mark.parametrize("n", [0, 1, 7, 150])
def test_oracle_matches_python_brute_force(bits, n):
    codes = datagen.uniform_codes(n, bits, 11 + bits)
    queries = datagen.uniform_codes(4, bits, 12 + bits)
    ks = [0, 1, 5, n + 3]
    for k in ks:
        ids, dists = oracle.knn(codes, queries, k, threads=3)
        for qi, (ri, rd) in enumerate(rows(ids, dists, [k] * 4)):
            bi, bd = oracle.knn_brute(codes.tolist(), queries[qi].tolist(), k)
            assert ri == bi and rd == bd


def test_oracle_ties_resolve_to_lowest_id_with_duplicates():
    # a database with many exact duplicates: ties at every distance
    base = datagen.uniform_codes(5, 128, 3)
    codes = np.concatenate([base[np.arange(60) % 5], base[:2]], axis=0)
    q = base[1:2] ^ np.uint64(0b1011)
    for k in [1, 3, 12, 13, 30, 62, 70]:
        ids, dists = oracle.knn(codes, q, k)
        bi, bd = oracle.knn_brute(codes.tolist(), q[0].tolist(), k)
        assert ids.tolist() == bi and dists.tolist() == bd


def test_oracle_matches_numpy_lexsort():
    codes = datagen.clustered_codes(3000, 128, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(6, 128, datagen.SEED_Q_CLUSTERED)
    k = 3000
    ids, dists = oracle.knn(codes, queries, k, threads=4)
    for qi in range(6):
        d = np.bitwise_count(codes ^ queries[qi]).sum(axis=1).astype(np.int64)
        order = np.lexsort((np.arange(len(d)), d))
        assert np.array_equal(ids[qi * k:(qi + 1) * k], order.astype(np.uint32))
        assert np.array_equal(dists[qi * k:(qi + 1) * k], d[order].astype(np.uint32))


def test_closed_form_prefix_masks():
    # h_i = 2^i - 1 (i = 0..64) against query 0: d_i = i, so the kNN are 0..k-1
    codes = np.array([[(1 << i) - 1] for i in range(65)], dtype=np.uint64)
    q = np.zeros((1, 1), dtype=np.uint64)
    for k in [1, 17, 65, 70]:
        ids, dists = oracle.knn(codes, q, k)
        kk = min(k, 65)
        assert ids[:kk].tolist() == list(range(kk))
        assert dists[:kk].tolist() == list(range(kk))
        assert ids[kk:].tolist() == [SENT] * (k - kk)
        assert dists[kk:].tolist() == [SENT] * (k - kk)


def test_closed_form_all_equal_database():
    codes = np.tile(np.array([[0x0123456789ABCDEF, 0xFFFF]], dtype=np.uint64), (40, 1))
    q = np.array([[0x0123456789ABCDEE, 0xFFFE]], dtype=np.uint64)   # 2 bits away
    ids, dists = oracle.knn(codes, q, 25)
    assert ids.tolist() == list(range(25)) and dists.tolist() == [2] * 25


def test_closed_form_query_equals_code_and_single_bit_flips():
    g = np.uint64(0xDEADBEEFCAFEF00D)
    flips = [g ^ np.uint64(1 << p) for p in range(64)]
    codes = np.array([[x] for x in flips[:30] + [g] + flips[30:] + [g]], dtype=np.uint64)
    ids, dists = oracle.knn(codes, np.array([[g]], dtype=np.uint64), 66)
    assert ids[:2].tolist() == [30, 65] and dists[:2].tolist() == [0, 0]
    assert ids[2:].tolist() == [i for i in range(66) if i not in (30, 65)]
    assert dists[2:].tolist() == [1] * 64


def test_oracle_per_query_k_and_thread_count_invariance():
    codes = datagen.uniform_codes(5000, 64, 21)
    queries = datagen.uniform_codes(9, 64, 22)
    ks = np.array([0, 1, 2, 10, 100, 0, 7, 5000, 5003], dtype=np.uint32)
    a = oracle.knn(codes, queries, ks, threads=1)
    b = oracle.knn(codes, queries, ks, threads=8)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    off = 0
    for qi, k in enumerate(ks.tolist()):
        bi, bd = oracle.knn_brute(codes.tolist(), queries[qi].tolist(), k) if k <= 200 else (None, None)
        if bi is not None:
            assert a[0][off:off + k].tolist() == bi and a[1][off:off + k].tolist() == bd
        off += k


def test_uniform_distance_histogram_is_binomial():
    # Uniform codes: d ~ Binomial(q, 1/2) (the analysis regime of Section 3).
    n = 200_000
    codes = datagen.uniform_codes(n, 64, 0)
    q = datagen.uniform_codes(1, 64, 1)[0]
    d = oracle.distances(codes, q)
    hist = np.bincount(d, minlength=65)
    from math import comb
    expect = np.array([n * comb(64, i) / 2 ** 64 for i in range(65)])
    core = expect > 500
    z = (hist[core] - expect[core]) / np.sqrt(expect[core])
    assert np.all(np.abs(z) < 6)
    assert abs(d.mean() - 32) < 0.05


def test_rnn_oracle_matches_brute():
    codes = datagen.uniform_codes(400, 64, 5)
    q = datagen.uniform_codes(1, 64, 6)[0]
    for r in [0, 20, 26, 30, 64]:
        ids, dists = oracle.rnn(codes, q, r)
        bi, bd = oracle.rnn_brute(codes.tolist(), q.tolist(), r)
        assert ids.tolist() == bi and dists.tolist() == bd
