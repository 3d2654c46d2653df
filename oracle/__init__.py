"""CPU oracle for exact Hamming kNN by multi-index hashing.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's CPU-baseline leg may import anything from this package.  It
shares no code with the GPU library in ``paper_1307_2982_amd``; the two meet
only through the seeded input generators in ``datagen``.

Contents:

* ``knn`` / ``rnn``: the plain definition of kNN and r-neighbour search
  (Section 1.1) as a threaded C linear scan (``knn_oracle.c``), ordered by
  (distance, id) with the lowest id winning ties.
* ``brute``: an independent pure-Python brute force for tiny inputs.
* ``MihCpu``: a literal single-threaded multi-index hashing (Algorithms 1, 2
  and 3 with the paper's bitstring de-duplication, ``mih_cpu.c``), a second
  test subject used to check the reading of the algorithm; with early
  stopping (``knn_approx``) it is the reference of the approximate variants
  of Section 7.
* ``substrings``: the substring optimisation of Section 5.5 (bit
  co-occurrence counts and the greedy bit order).
* ``first_encounter``: which codes Algorithm 3 has met after each step, from
  the substring distances (brute force); the reference of the early stops
  of Section 7.
* ``formulas``: the paper's closed forms (Eq. 1, 5, 6, 7, the memory formula
  of Section 6 and the q / log2 n heuristic of Section 3.1).

Parity status: the kNN oracle is pinned by the Python brute force, by closed
forms and by library routines (numpy popcount + lexsort); MIH-CPU is pinned
by agreement with the oracle for every m, and its early stops by agreement
with ``first_encounter`` (answers and step counts).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from . import first_encounter  # noqa: F401
from . import formulas  # noqa: F401
from .brute import knn_brute, rnn_brute  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_L = None
SENTINEL = 0xFFFFFFFF


def build(force: bool = True) -> str:
    """Compile the C oracle and MIH-CPU into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-mpopcnt", "-std=c11", "-fPIC", "-shared", "-pthread",
               os.path.join(_HERE, "knn_oracle.c"), os.path.join(_HERE, "mih_cpu.c"),
               "-o", _SO + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    return _SO


class _Stats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("lookups", ctypes.c_uint64),
                ("candidates", ctypes.c_uint64), ("unique", ctypes.c_uint64),
                ("radius", ctypes.c_uint64)]


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        L.oracle_knn.argtypes = [vp, u64, u32, vp, u32, vp, vp, vp, vp, i32]
        L.oracle_knn.restype = i32
        L.oracle_rnn.argtypes = [vp, u64, u32, vp, u32, vp, vp, u64]
        L.oracle_rnn.restype = u64
        L.oracle_distances.argtypes = [vp, u64, u32, vp, vp]
        L.oracle_distances.restype = None
        L.mihcpu_build.argtypes = [vp, u64, u32, u32]
        L.mihcpu_build.restype = vp
        L.mihcpu_free.argtypes = [vp]
        L.mihcpu_free.restype = None
        L.mihcpu_knn.argtypes = [vp, vp, u32, vp, vp, ctypes.POINTER(_Stats)]
        L.mihcpu_knn.restype = i32
        L.mihcpu_knn_approx.argtypes = [vp, vp, u32, u32, ctypes.c_uint64, vp, vp, ctypes.POINTER(_Stats)]
        L.mihcpu_knn_approx.restype = i32
        L.mihcpu_rnn.argtypes = [vp, vp, u32, vp, vp, u64, ctypes.POINTER(_Stats)]
        L.mihcpu_rnn.restype = ctypes.c_int64
        L.mihcpu_partition.argtypes = [u32, u32, vp, vp]
        L.mihcpu_partition.restype = None
        L.mihcpu_substring.argtypes = [vp, u32, u32]
        L.mihcpu_substring.restype = u64
        L.mihcpu_table.argtypes = [vp, u32, vp, vp]
        L.mihcpu_table.restype = None
        _L = L
    return _L


def _codes(a) -> np.ndarray:
    a = np.ascontiguousarray(a)
    if a.dtype == np.int64:
        a = a.view(np.uint64)
    if a.dtype != np.uint64 or a.ndim != 2:
        raise TypeError("codes must be a 2-D uint64 array [n, bits/64]")
    return a


def row_offsets(k_per_query) -> np.ndarray:
    k = np.asarray(k_per_query, dtype=np.uint64)
    off = np.zeros(len(k), dtype=np.uint64)
    if len(k) > 1:
        off[1:] = np.cumsum(k[:-1])
    return off


def knn(codes, queries, k, threads: int | None = None):
    """Exact kNN of every query.

    ``k`` is an int or a per-query sequence.  Returns flat (ids, dists) uint32
    arrays with row i at offset sum(k[:i]), padded with 0xFFFFFFFF.
    """
    codes, queries = _codes(codes), _codes(queries)
    n, words = codes.shape
    nq = queries.shape[0]
    if queries.shape[1] != words:
        raise ValueError("queries and codes differ in length")
    ks = np.full(nq, k, dtype=np.uint32) if np.isscalar(k) else np.ascontiguousarray(k, dtype=np.uint32)
    off = row_offsets(ks)
    total = int(ks.sum(dtype=np.uint64))
    ids = np.empty(total, dtype=np.uint32)
    dists = np.empty(total, dtype=np.uint32)
    used = _lib().oracle_knn(codes.ctypes.data, n, words, queries.ctypes.data, nq,
                             ks.ctypes.data, off.ctypes.data, ids.ctypes.data,
                             dists.ctypes.data, threads or (os.cpu_count() or 1))
    knn.last_threads = int(used)
    return ids, dists


knn.last_threads = 0


def rnn(codes, query, r: int):
    """All codes within distance r of one query, in (d, id) order."""
    codes = _codes(codes)
    q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
    n, words = codes.shape
    cap = 1 << 16
    while True:
        ids = np.empty(cap, dtype=np.uint32)
        dists = np.empty(cap, dtype=np.uint32)
        tot = int(_lib().oracle_rnn(codes.ctypes.data, n, words, q.ctypes.data, r,
                                    ids.ctypes.data, dists.ctypes.data, cap))
        if tot <= cap:
            return ids[:tot].copy(), dists[:tot].copy()
        cap = tot


def distances(codes, query) -> np.ndarray:
    codes = _codes(codes)
    q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
    n, words = codes.shape
    out = np.empty(n, dtype=np.uint32)
    _lib().oracle_distances(codes.ctypes.data, n, words, q.ctypes.data, out.ctypes.data)
    return out


def partition(bits: int, m: int):
    """Substring lengths and start bits used by MIH-CPU (Section 2.1 footnote)."""
    ln = np.empty(m, dtype=np.uint32)
    st = np.empty(m, dtype=np.uint32)
    _lib().mihcpu_partition(bits, m, ln.ctypes.data, st.ctypes.data)
    return ln.tolist(), st.tolist()


def substring(code, start: int, length: int) -> int:
    c = np.ascontiguousarray(code, dtype=np.uint64).reshape(-1)
    return int(_lib().mihcpu_substring(c.ctypes.data, start, length))


class MihCpu:
    """Literal multi-index hashing on the CPU (Algorithms 1-3); a test subject."""

    def __init__(self, codes, m: int):
        self.codes = _codes(codes)
        self.n, self.words = self.codes.shape
        self.m = m
        self._ix = _lib().mihcpu_build(self.codes.ctypes.data, self.n, self.words, m)
        if not self._ix:
            raise ValueError("bad arguments for MIH-CPU build")

    def close(self):
        if self._ix:
            _lib().mihcpu_free(self._ix)
            self._ix = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def table(self, j: int):
        """Table j of Algorithm 1 as (values, ids) sorted by value, then id."""
        values = np.empty(self.n, dtype=np.uint64)
        ids = np.empty(self.n, dtype=np.uint32)
        _lib().mihcpu_table(self._ix, j, values.ctypes.data, ids.ctypes.data)
        return values, ids

    def knn(self, query, k: int):
        q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
        ids = np.empty(max(k, 1), dtype=np.uint32)
        dists = np.empty(max(k, 1), dtype=np.uint32)
        st = _Stats()
        rc = _lib().mihcpu_knn(self._ix, q.ctypes.data, k, ids.ctypes.data, dists.ctypes.data,
                               ctypes.byref(st))
        if rc != 0:
            raise MemoryError("MIH-CPU out of memory")
        stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
        return ids[:k].copy(), dists[:k].copy(), stats

    def knn_approx(self, query, k: int, max_step: int | None = None, max_found: int = 0,
                   stats: bool = False):
        """Algorithm 3 stopped after the step covering radius max_step, or
        after the step in which max_found distinct codes have been met
        (Section 7); the k best codes met (and, with stats, the counters of
        the search: ``radius`` is the number of steps run)."""
        q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
        ids = np.empty(max(k, 1), dtype=np.uint32)
        dists = np.empty(max(k, 1), dtype=np.uint32)
        st = _Stats()
        rc = _lib().mihcpu_knn_approx(self._ix, q.ctypes.data, k,
                                      0xFFFFFFFF if max_step is None else max_step, max_found,
                                      ids.ctypes.data, dists.ctypes.data, ctypes.byref(st))
        if rc != 0:
            raise MemoryError("MIH-CPU out of memory")
        if stats:
            return ids[:k].copy(), dists[:k].copy(), {f: getattr(st, f) for f, _ in _Stats._fields_}
        return ids[:k].copy(), dists[:k].copy()

    def rnn(self, query, r: int):
        q = np.ascontiguousarray(query, dtype=np.uint64).reshape(-1)
        cap = max(1, self.n)
        ids = np.empty(cap, dtype=np.uint32)
        dists = np.empty(cap, dtype=np.uint32)
        st = _Stats()
        tot = _lib().mihcpu_rnn(self._ix, q.ctypes.data, r, ids.ctypes.data, dists.ctypes.data,
                                cap, ctypes.byref(st))
        if tot < 0:
            raise MemoryError("MIH-CPU out of memory")
        stats = {f: getattr(st, f) for f, _ in _Stats._fields_}
        return ids[:tot].copy(), dists[:tot].copy(), stats
