"""Pure-Python brute force for tiny inputs: an oracle independent of the C one.

TEST INFRASTRUCTURE ONLY.  Implements the definitions of Section 1.1 with
Python integers: the Hamming distance of two codes is the number of set bits
of their XOR; kNN returns the first min(k, n) pairs (d, id) in ascending
lexicographic order; the r-neighbours are all ids with d <= r in that order.
"""
from __future__ import annotations


def _as_int(row) -> int:
    v = 0
    for w, word in enumerate(row):
        v |= (int(word) & 0xFFFFFFFFFFFFFFFF) << (64 * w)
    return v


def hamming(a, b) -> int:
    return (_as_int(a) ^ _as_int(b)).bit_count()


def knn_brute(codes, query, k: int):
    g = _as_int(query)
    pairs = sorted(((_as_int(h) ^ g).bit_count(), i) for i, h in enumerate(codes))
    top = pairs[:k]
    ids = [i for _, i in top] + [0xFFFFFFFF] * (k - len(top))
    dists = [d for d, _ in top] + [0xFFFFFFFF] * (k - len(top))
    return ids, dists


def rnn_brute(codes, query, r: int):
    g = _as_int(query)
    pairs = sorted(((_as_int(h) ^ g).bit_count(), i) for i, h in enumerate(codes))
    pairs = [p for p in pairs if p[0] <= r]
    return [i for _, i in pairs], [d for d, _ in pairs]
