"""Closed forms from the paper, written out (test infrastructure).

* ``ball(q, r)``: L(q, r) = sum_{z=0}^{r} C(q, z), the number of buckets within
  Hamming radius r of a q-bit key (Section 1.1, Eq. 1).
* ``lookups(q, s, r)``: (q/s) sum_{z=0}^{floor(s r / q)} C(s, z), the lookups of
  r-neighbour search with m = q/s tables (Section 3, Eq. 5).
* ``lookups_bound(q, s, r)``: (q/s) 2^{H(r/q) s} (right side of Eq. 5).
* ``cost(n, q, s, r)``: (1 + n / 2^s) lookups(s) (Eq. 6) and its bound (Eq. 7).
* ``memory_bytes(n, q, m)``: m 2^{s-5} 24 + m min(n, 2^s) 4 + 4 m n + n m s / 8
  with s = q/m (Section 6, "Memory Requirements").
* ``m_heuristic(n, q)``: q / log2 n (Section 3.1 and Table 4).
* ``shell(s, rho)``: C(s, rho), the buckets one kNN step examines
  (Algorithm 3 looks up buckets that differ in exactly r' bits).
* ``partition(q, m)``: substring lengths floor(q/m) or ceil(q/m) (Section 2.1
  footnote), longer ones first, contiguous.
"""
from __future__ import annotations

import math


def ball(q: int, r: int) -> int:
    return sum(math.comb(q, z) for z in range(0, min(r, q) + 1))


def shell(s: int, rho: int) -> int:
    return math.comb(s, rho) if 0 <= rho <= s else 0


def entropy(eps: float) -> float:
    if eps <= 0.0 or eps >= 1.0:
        return 0.0
    return -eps * math.log2(eps) - (1.0 - eps) * math.log2(1.0 - eps)


def lookups(q: int, s: int, r: int) -> float:
    return (q / s) * sum(math.comb(s, z) for z in range(0, (s * r) // q + 1))


def lookups_bound(q: int, s: int, r: int) -> float:
    return (q / s) * 2.0 ** (entropy(r / q) * s)


def cost(n: int, q: int, s: int, r: int) -> float:
    return (1.0 + n / 2.0 ** s) * lookups(q, s, r)


def cost_bound(n: int, q: int, s: int, r: int) -> float:
    return (1.0 + n / 2.0 ** s) * lookups_bound(q, s, r)


def memory_bytes(n: int, q: int, m: int) -> float:
    s = q // m
    return m * 2 ** (s - 5) * 24 + m * min(n, 2 ** s) * 4 + 4 * m * n + n * m * s / 8


def m_heuristic(n: int, q: int) -> float:
    return q / math.log2(n)


def partition(q: int, m: int):
    base, extra = divmod(q, m)
    lens = [base + (1 if j < extra else 0) for j in range(m)]
    starts, s = [], 0
    for ln in lens:
        starts.append(s)
        s += ln
    return lens, starts


def step_of(t: int, m: int):
    """Algorithm 3's step t uses table a = t mod m at substring radius floor(t/m)."""
    return t // m, t % m


def prop2_radii(r: int, m: int):
    """Proposition 2: with r = m r' + a, tables 1..a+1 at r', the rest at r'-1."""
    rp, a = divmod(r, m)
    return [rp if j <= a else rp - 1 for j in range(m)]
