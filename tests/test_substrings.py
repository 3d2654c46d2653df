"""Substring optimisation (Section 5.5): the oracle's greedy against a design
whose answer follows from the description by hand, its co-occurrence counts
against brute force, and the library's host-side greedy against the oracle.
No GPU."""
import numpy as np
import pytest

import datagen
from oracle import substrings as S


def paired_hadamard_codes():
    """64 codes of 64 bits: bits 2i and 2i+1 are equal, and the 32 pairs are
    columns 1..32 of a 64 x 64 Sylvester Hadamard matrix (balanced and
    pairwise orthogonal, so different pairs have correlation exactly 0)."""
    h = np.array([[1]])
    for _ in range(6):
        h = np.block([[h, h], [h, -h]])
    base = (h[:, 1:33] > 0).astype(np.uint64)
    codes = np.zeros((64, 1), dtype=np.uint64)
    for i in range(32):
        for b in (2 * i, 2 * i + 1):
            codes[:, 0] |= base[:, i] << np.uint64(b)
    return codes


def test_oracle_greedy_separates_correlated_pairs():
    # m = 2: substring 0 starts with bit 0, substring 1 with its twin bit 1;
    # every later pick has correlation 0 with what the substring holds, so
    # the lowest free bit goes to each substring in turn: evens and odds.
    codes = paired_hadamard_codes()
    counts = S.cooccurrence(codes)
    order = S.greedy_bit_order(counts, 64, 64, 2, 0)
    assert order == list(range(0, 64, 2)) + list(range(1, 64, 2))
    # m = 4: substring 2 starts with the lowest bit (2) since bit 1 is
    # uncorrelated with every free bit, substring 3 with its twin 3
    order = S.greedy_bit_order(counts, 64, 64, 4, 0)
    assert order == [b for r in range(4) for b in range(r, 64, 4)]
    # consecutive substrings hold twins (correlation 1); the greedy ones none
    assert S.max_within_correlation(counts, 64, list(range(64)), 2) == 1.0
    assert S.max_within_correlation(counts, 64, S.greedy_bit_order(counts, 64, 64, 2, 0), 2) == 0.0


def test_oracle_cooccurrence_is_pair_counts():
    codes = datagen.uniform_codes(50, 128, 91)
    counts = S.cooccurrence(codes)
    bit = lambda c, p: int(c[p // 64]) >> (p % 64) & 1
    for i in range(0, 128, 7):
        for j in range(0, 128, 5):
            assert counts[i, j] == sum(bit(c, i) & bit(c, j) for c in codes)


def test_oracle_greedy_is_a_partition_of_the_bits():
    codes = datagen.clustered_codes(3000, 128, datagen.SEED_DB_CLUSTERED)
    counts = S.cooccurrence(codes)
    for m in (3, 6):
        order = S.greedy_bit_order(counts, 3000, 128, m, 17)
        assert sorted(order) == list(range(128)) and order[0] == 17


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


@pytest.mark.parametrize("bits,m,first", [(64, 2, 0), (64, 3, 5), (128, 6, 0), (128, 5, 99), (256, 8, 3)])
def test_library_greedy_equals_oracle(mih, bits, m, first):
    codes = datagen.clustered_codes(2000, bits, datagen.SEED_DB_CLUSTERED)
    counts = S.cooccurrence(codes)
    assert mih.greedy_bit_order(counts, 2000, m, first) == S.greedy_bit_order(counts, 2000, bits, m, first)


def test_library_greedy_on_the_paired_design(mih):
    counts = S.cooccurrence(paired_hadamard_codes())
    assert mih.greedy_bit_order(counts, 64, 2, 0) == list(range(0, 64, 2)) + list(range(1, 64, 2))
