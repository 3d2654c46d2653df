"""MIH-CPU (Algorithms 1-3, bitstring de-duplication) against the oracle.

The search result must not depend on m, on the substring partition or on the
code distribution; MIH-CPU must also stop exactly after step d_k (the k-th
smallest distance), since step t completes the search of radius t
(Proposition 2) and the loop ends once radius t holds k codes.
"""
import numpy as np
import pytest

import datagen
import oracle
from oracle import formulas


def _check_against_oracle(codes, queries, m, ks):
    mih = oracle.MihCpu(codes, m)
    n = codes.shape[0]
    for k in ks:
        ids, dists = oracle.knn(codes, queries, k)
        for qi in range(queries.shape[0]):
            mi, md, st = mih.knn(queries[qi], k)
            assert mi.tolist() == ids[qi * k:(qi + 1) * k].tolist(), (m, k, qi)
            assert md.tolist() == dists[qi * k:(qi + 1) * k].tolist(), (m, k, qi)
            if 0 < k <= n:
                # the loop ends right after step t = d_k
                assert st["radius"] == int(md[k - 1]) + 1
                # lookups: one per bucket of each exact shell C(s_a, r') (Eq. 1)
                lens, _ = formulas.partition(codes.shape[1] * 64, m)
                expect = sum(formulas.shell(lens[t % m], t // m) for t in range(st["radius"]))
                assert st["lookups"] == expect
    mih.close()


@pytest.mark.parametrize("m", [3, 4, 5, 6, 7, 8])
def test_mih_cpu_equals_oracle_uniform_64(m):
    codes = datagen.uniform_codes(3000, 64, 31)
    queries = datagen.uniform_codes(3, 64, 32)
    _check_against_oracle(codes, queries, m, [1, 10, 100])


@pytest.mark.parametrize("m", [1, 2])
def test_mih_cpu_equals_oracle_planted_neighbours(m):
    # one or two tables only pay off when neighbours are near: plant 40 codes
    # within 3 bits of each query among 2000 uniform codes
    queries = datagen.uniform_codes(2, 64, 34)
    rng = np.random.default_rng(7)
    planted = []
    for q in queries[:, 0]:
        for _ in range(20):
            x = int(q)
            for b in rng.choice(64, size=int(rng.integers(0, 4)), replace=False):
                x ^= 1 << int(b)
            planted.append([x])
    codes = np.concatenate([datagen.uniform_codes(2000, 64, 33),
                            np.array(planted, dtype=np.uint64)], axis=0)
    _check_against_oracle(codes, queries, m, [1, 5, 20])


@pytest.mark.parametrize("m", [6, 9, 12])
def test_mih_cpu_equals_oracle_clustered_128(m):
    codes = datagen.clustered_codes(4000, 128, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(3, 128, datagen.SEED_Q_CLUSTERED)
    _check_against_oracle(codes, queries, m, [1, 10, 100])


@pytest.mark.parametrize("bits,m", [(64, 64), (64, 16), (192, 12), (256, 16), (256, 20)])
def test_mih_cpu_equals_oracle_many_tables(bits, m):
    codes = datagen.uniform_codes(300, bits, 41)
    queries = datagen.uniform_codes(2, bits, 42)
    _check_against_oracle(codes, queries, m, [1, 10])


def test_mih_cpu_k_beyond_n_and_zero():
    codes = datagen.uniform_codes(50, 64, 51)
    queries = datagen.uniform_codes(2, 64, 52)
    _check_against_oracle(codes, queries, 3, [0, 50, 55])


def test_mih_cpu_duplicates_and_ties():
    base = datagen.uniform_codes(4, 64, 53)
    codes = base[np.arange(200) % 4]
    queries = np.concatenate([base[:1], base[2:3] ^ np.uint64(0xF0)], axis=0)
    _check_against_oracle(codes, queries, 4, [1, 30, 51, 120, 200])


@pytest.mark.parametrize("m", [3, 4, 5])
def test_mih_cpu_rnn_equals_oracle(m):
    codes = datagen.uniform_codes(2000, 64, 61)
    q = datagen.uniform_codes(1, 64, 62)[0]
    mih = oracle.MihCpu(codes, m)
    lens, _ = formulas.partition(64, m)
    for r in [0, 3, 14, 20, 23]:
        ids, dists, st = mih.rnn(q, r)
        oi, od = oracle.rnn(codes, q, r)
        assert ids.tolist() == oi.tolist() and dists.tolist() == od.tolist()
        # Algorithm 2 examines, per table, the ball of Proposition 2's radius
        radii = formulas.prop2_radii(r, m)
        expect = sum(formulas.ball(lens[j], radii[j]) for j in range(m) if radii[j] >= 0)
        assert st["lookups"] == expect
    mih.close()
