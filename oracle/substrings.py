"""Substring optimisation of Section 5.5, written out (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by the tests alone.  Shares no code with
the GPU library.

* ``cooccurrence(codes)``: counts[i, j] = number of codes whose bits i and j
  are both set, from the unpacked 0/1 matrix X as X^T X in integers.
* ``correlation(counts, n)``: |Pearson correlation| of every pair of bits,
  from the counts (a constant bit has correlation 0 with every bit).  The
  numerator N c_ij - c_i c_j is exact in integers; the quotient is taken in
  double precision.
* ``greedy_bit_order(counts, n, bits, m, first_bit)``: the paper's greedy
  assignment.  Substring 0 starts with a given bit; substring j starts with
  the unused bit most correlated with the bit of substring j - 1; then the
  substrings, one after another in turn, each take the unused bit whose
  largest correlation with the bits already in that substring is smallest.
  Ties go to the lowest bit index.  Returns the bit order: substring j is
  positions [start_j, start_j + s_j) of it, with the substring lengths of
  Section 2.1 (floor or ceil of bits / m, longer ones first).
"""
from __future__ import annotations

import math

import numpy as np


def unpack_bits(codes: np.ndarray) -> np.ndarray:
    """0/1 matrix [n, bits]: column p is bit p (bit p % 64 of word p // 64)."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    n, words = codes.shape
    cols = [((codes[:, p // 64] >> np.uint64(p % 64)) & np.uint64(1)).astype(np.int64)
            for p in range(64 * words)]
    return np.stack(cols, axis=1) if cols else np.zeros((n, 0), dtype=np.int64)


def cooccurrence(codes: np.ndarray) -> np.ndarray:
    x = unpack_bits(codes)
    return x.T @ x


def correlation(counts: np.ndarray, n: int) -> list[list[float]]:
    bits = counts.shape[0]
    c = [[int(counts[u, v]) for v in range(bits)] for u in range(bits)]
    out = [[0.0] * bits for _ in range(bits)]
    for u in range(bits):
        for v in range(bits):
            vu = c[u][u] * (n - c[u][u])
            vv = c[v][v] * (n - c[v][v])
            if vu == 0 or vv == 0:
                continue
            num = n * c[u][v] - c[u][u] * c[v][v]
            out[u][v] = abs(float(num) / math.sqrt(float(vu) * float(vv)))
    return out


def substring_lengths(bits: int, m: int) -> list[int]:
    return [bits // m + (1 if j < bits % m else 0) for j in range(m)]


def greedy_bit_order(counts: np.ndarray, n: int, bits: int, m: int, first_bit: int) -> list[int]:
    corr = correlation(counts, n)
    lens = substring_lengths(bits, m)
    used = [False] * bits
    subs = [[first_bit]]
    used[first_bit] = True
    for j in range(1, m):
        prev = subs[j - 1][0]
        best = None
        for u in range(bits):
            if not used[u] and (best is None or corr[prev][u] > corr[prev][best]):
                best = u
        subs.append([best])
        used[best] = True
    assigned = m
    while assigned < bits:
        for j in range(m):
            if assigned == bits:
                break
            if len(subs[j]) >= lens[j]:
                continue
            best, best_v = None, 0.0
            for u in range(bits):
                if used[u]:
                    continue
                worst = max(corr[u][v] for v in subs[j])
                if best is None or worst < best_v:
                    best, best_v = u, worst
            subs[j].append(best)
            used[best] = True
            assigned += 1
    return [b for s in subs for b in s]


def max_within_correlation(counts: np.ndarray, n: int, order: list[int], m: int) -> float:
    """Largest |correlation| between two bits of the same substring."""
    corr = correlation(counts, n)
    lens = substring_lengths(len(order), m)
    worst, p = 0.0, 0
    for ln in lens:
        sub = order[p:p + ln]
        p += ln
        for i in range(len(sub)):
            for j in range(i + 1, len(sub)):
                worst = max(worst, corr[sub[i]][sub[j]])
    return worst
