"""Which codes Algorithm 3 has met after a given step, computed from the
definition by brute force; the reference of its early-stopped (approximate)
variants of Section 7.

TEST INFRASTRUCTURE ONLY: used by the tests to pin MIH-CPU's early stops and
the GPU's approximate search.  It shares no code with the GPU library and
none with MIH-CPU (it builds no table and probes no bucket).

Algorithm 3 runs steps t = 0, 1, 2, ...; step t looks up, in table
a = t mod m, every bucket whose substring differs from the query's in exactly
r' = floor(t / m) bits.  A code h whose substring distances to the query g
are d_0 .. d_{m-1} (d_j = Hamming distance of substring j of h and of g)
lies in such a bucket at exactly the steps m d_j + j, so it is met for the
first time at step

    t_h = min_j (m d_j + j)

and after steps 0 .. T the distinct codes met are {h : t_h <= T}.  Every code
within full distance T has some d_j <= floor(T / m) with the right table
order (Proposition 2), so after step T every code with d_h <= T is among
them.

The loop of Algorithm 3 ends after the first step T at which any of these
holds:
  * exact stop: the codes met within distance T number at least k (the sets
    N_0 .. N_T of Algorithm 3), i.e. |{h : d_h <= T}| >= k;
  * radius stop (Section 7): T reaches the given radius;
  * budget stop (Section 7): the distinct codes met number at least the
    budget, |{h : t_h <= T}| >= budget;
  * guard: every table has been searched over its whole length, which only
    matters when k exceeds n.  The guard step depends on the implementation
    (MIH-CPU: T = m (max_j s_j + 1) - 1; the device library: the first step
    at which every code is surely met, min_j (m s_j + j)), so it is an
    argument.
The answer is the k best codes met, in (distance, id) order, padded with
0xFFFFFFFF.

Substrings (Section 2.1 and its footnote): contiguous bit runs, the first
(bits mod m) of them one bit longer; bit p of a code is bit p mod 64 of
64-bit word floor(p / 64).
"""
from __future__ import annotations

import numpy as np

SENTINEL = 0xFFFFFFFF


def partition(bits: int, m: int):
    """Substring lengths and first bits: floor or ceil of bits / m, the
    longer ones first, each starting where the previous one ends."""
    base, extra = divmod(bits, m)
    lens = [base + 1 if j < extra else base for j in range(m)]
    starts = [sum(lens[:j]) for j in range(m)]
    return lens, starts


def _bit_mask(words: int, start: int, length: int) -> np.ndarray:
    """Per-word masks of code bits [start, start + length)."""
    mask = np.zeros(words, dtype=np.uint64)
    for p in range(start, start + length):
        mask[p // 64] |= np.uint64(1) << np.uint64(p % 64)
    return mask


def substring_distances(codes: np.ndarray, query: np.ndarray, m: int) -> np.ndarray:
    """[m, n] array: d_j of every code to the query."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
    n, words = codes.shape
    x = codes ^ q[None, :]
    lens, starts = partition(64 * words, m)
    out = np.zeros((m, n), dtype=np.int64)
    for j in range(m):
        mk = _bit_mask(words, starts[j], lens[j])
        out[j] = np.bitwise_count(x & mk[None, :]).sum(axis=1)
    return out


def first_steps(codes: np.ndarray, query: np.ndarray, m: int):
    """(t_h, d_h) for every code: the step of its first encounter and its
    full Hamming distance to the query."""
    dj = substring_distances(codes, query, m)
    steps = m * dj + np.arange(m, dtype=np.int64)[:, None]
    return steps.min(axis=0), dj.sum(axis=0)


def mihcpu_guard(bits: int, m: int) -> int:
    """The step after which MIH-CPU ends a query whose k was not reached."""
    lens, _ = partition(bits, m)
    return m * (max(lens) + 1) - 1


def device_guard(bits: int, m: int) -> int:
    """The step after which the device library ends such a query."""
    lens, _ = partition(bits, m)
    return min(m * s + j for j, s in enumerate(lens))


def stop_step(th: np.ndarray, dh: np.ndarray, k: int, max_step: int | None, max_found: int,
              guard: int) -> int:
    """The step after which Algorithm 3 ends (k >= 1)."""
    last = guard
    if k <= len(dh):
        # exact stop: the k-th smallest full distance
        last = min(last, int(np.partition(dh, k - 1)[k - 1]))
    if max_step is not None:
        last = min(last, int(max_step))
    if max_found:
        if max_found <= len(th):
            last = min(last, int(np.partition(th, max_found - 1)[max_found - 1]))
    return last


def early_stop(codes: np.ndarray, query: np.ndarray, m: int, k: int, max_step: int | None = None,
               max_found: int = 0, guard: int | None = None, steps_and_dists=None):
    """(ids, dists, steps): the k best codes met by Algorithm 3 stopped as
    above, and the number of steps it ran (last step + 1).
    steps_and_dists: first_steps(codes, query, m), if already computed."""
    codes = np.ascontiguousarray(codes, dtype=np.uint64)
    bits = 64 * codes.shape[1]
    if guard is None:
        guard = mihcpu_guard(bits, m)
    ids = np.full(k, SENTINEL, dtype=np.uint32)
    dists = np.full(k, SENTINEL, dtype=np.uint32)
    if k == 0:
        return ids, dists, 0
    th, dh = steps_and_dists if steps_and_dists is not None else first_steps(codes, query, m)
    last = stop_step(th, dh, k, max_step, max_found, guard)
    met = np.nonzero(th <= last)[0]
    order = np.lexsort((met, dh[met]))[:k]
    ids[:len(order)] = met[order]
    dists[:len(order)] = dh[met][order]
    return ids, dists, last + 1
