"""Exact Hamming kNN by multi-index hashing on AMD MI355X (gfx950).

A thin ctypes binding over ``libmih.so`` (C ABI declared in
``include/mih.h``).  PyTorch supplies device memory and the current HIP
stream; every step of the search runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing, loading fails with an error.

    import paper_1307_2982_amd as mih
    idx = mih.build(codes, m=2)              # codes: int64/uint64 [n, bits/64] on cuda
    ids, dists = idx.knn(queries, k=100)     # int32 tensors, row-major [nq, k]
    ids, dists = mih.linscan_knn(codes, queries, 100)
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmih.so")

SENTINEL = 0xFFFFFFFF
K_MAX = 4096
TABLE_MODES = {"auto": 0, "direct": 1, "sorted": 2, "grouped": 3, "heads": 4}
CODES_MODES = {"auto": 0, "inline": 1, "indirect": 2, "mixed": 3}
STATUS = {0: "ok", 1: "invalid argument", 2: "out of device memory", 3: "device error",
          4: "unsupported", 5: "no capacity"}


class MihError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {STATUS.get(status, status)} (status {status})")
        self.status = status


class BuildOpts(ctypes.Structure):
    _fields_ = [("table_mode", ctypes.c_int), ("codes_mode", ctypes.c_int),
                ("mem_budget_bytes", ctypes.c_uint64), ("bit_order", ctypes.c_void_p),
                ("inline_tables", ctypes.c_uint32), ("autotune_cache", ctypes.c_char_p)]


class IndexInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("bits", ctypes.c_uint32), ("m", ctypes.c_uint32),
                ("table_mode", ctypes.c_uint32), ("codes_mode", ctypes.c_uint32),
                ("sub_len", ctypes.c_uint32 * 64), ("sub_start", ctypes.c_uint32 * 64),
                ("dir_bits", ctypes.c_uint32 * 64), ("device_bytes", ctypes.c_uint64),
                ("build_ms", ctypes.c_double), ("bit_order", ctypes.c_uint16 * 256),
                ("inline_tables", ctypes.c_uint32), ("autotune_cache", ctypes.c_char_p)]


class TableView(ctypes.Structure):
    _fields_ = [("offsets", ctypes.c_void_p), ("keys", ctypes.c_void_p), ("dir", ctypes.c_void_p),
                ("ids", ctypes.c_void_p), ("codes", ctypes.c_void_p), ("len", ctypes.c_uint32),
                ("start", ctypes.c_uint32), ("dir_bits", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("occupancy", ctypes.c_void_p), ("groups", ctypes.c_void_p), ("heads", ctypes.c_void_p)]


class QueryStats(ctypes.Structure):
    _fields_ = [("probes", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("appended", ctypes.c_uint64), ("steps", ctypes.c_uint64),
                ("rounds", ctypes.c_uint32), ("reruns", ctypes.c_uint32),
                ("elapsed_ms", ctypes.c_double), ("search_kernel_ms", ctypes.c_double),
                ("search_launches", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("tail_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class ScanStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_uint64), ("appended", ctypes.c_uint64),
                ("reruns", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("elapsed_ms", ctypes.c_double), ("scan_kernel_ms", ctypes.c_double),
                ("sample_kernel_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad"}


class Tuning(ctypes.Structure):
    _fields_ = [("probes_per_lane", ctypes.c_uint32), ("chunk", ctypes.c_uint32),
                ("blocks_per_cu", ctypes.c_uint32), ("occupancy_filter", ctypes.c_uint32),
                ("sweep_shift", ctypes.c_uint32), ("sweep_bits", ctypes.c_uint32),
                ("lookahead", ctypes.c_uint32), ("sweep_queries", ctypes.c_uint32),
                ("buffer_mult", ctypes.c_uint32), ("small_batch", ctypes.c_uint32),
                ("round_masks", ctypes.c_uint32), ("spill_codes", ctypes.c_uint32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MTrial(ctypes.Structure):
    _fields_ = [("m", ctypes.c_uint32), ("status", ctypes.c_int), ("model_cost", ctypes.c_double),
                ("search_ms", ctypes.c_double), ("build_ms", ctypes.c_double),
                ("device_bytes", ctypes.c_uint64)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["status"] = STATUS.get(d["status"], d["status"])
        return d


M_TRIALS_MAX = 16


class RnnView(ctypes.Structure):
    _fields_ = [("total", ctypes.c_uint64), ("nq", ctypes.c_uint32), ("pad", ctypes.c_uint32),
                ("offsets", ctypes.c_void_p), ("ids", ctypes.c_void_p), ("dists", ctypes.c_void_p)]


EXPORTED = ["mih_build", "mih_knn", "mih_knn_ex", "linscan_knn", "linscan_knn_ex", "linscan_knn_noalloc",
            "mih_free",
            "mih_rnn", "mih_rnn_ex", "linscan_rnn", "mih_rnn_result_view", "mih_rnn_result_free",
            "mih_knn_approx", "mih_model_cost", "mih_model_radius", "mih_choose_m", "mih_bit_cooccurrence",
            "mih_greedy_bit_order",
            "mih_status_str", "mih_index_get_info", "mih_index_table", "mih_get_tuning",
            "mih_set_tuning", "mih_autotune", "mih_server_create", "mih_server_submit", "mih_server_step",
            "mih_server_poll", "mih_server_get_stats", "mih_server_destroy", "mih_random_read_rate"]

_lib = None


def lib_path() -> str:
    return LIB_PATH


def load():
    """Load libmih.so (built by ``paper_1307_2982_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1307_2982_amd.buildlib` "
                          "(the search has no CPU fallback)")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
    L.mih_build.argtypes = [vp, u64, u32, u32, ctypes.POINTER(BuildOpts), vp, ctypes.POINTER(vp)]
    L.mih_build.restype = i32
    L.mih_knn.argtypes = [vp, vp, u32, u32, vp, vp, vp, vp]
    L.mih_knn.restype = i32
    L.mih_knn_ex.argtypes = [vp, vp, u32, u32, vp, vp, vp, vp, ctypes.POINTER(QueryStats)]
    L.mih_knn_ex.restype = i32
    L.mih_knn_approx.argtypes = [vp, vp, u32, u32, vp, u32, u32, vp, vp, vp, ctypes.POINTER(QueryStats)]
    L.mih_knn_approx.restype = i32
    L.linscan_knn.argtypes = [vp, u64, u32, vp, u32, u32, vp, vp, vp, vp]
    L.linscan_knn.restype = i32
    L.linscan_knn_ex.argtypes = [vp, u64, u32, vp, u32, u32, vp, vp, vp, vp, ctypes.POINTER(ScanStats)]
    L.linscan_knn_ex.restype = i32
    L.linscan_knn_noalloc.argtypes = [vp, u64, u32, vp, u32, u32, vp, vp, vp, vp]
    L.linscan_knn_noalloc.restype = i32
    L.mih_free.argtypes = [vp]
    L.mih_free.restype = None
    L.mih_rnn.argtypes = [vp, vp, u32, u32, vp, vp, ctypes.POINTER(vp)]
    L.mih_rnn.restype = i32
    L.mih_rnn_ex.argtypes = [vp, vp, u32, u32, vp, vp, ctypes.POINTER(vp), ctypes.POINTER(QueryStats)]
    L.mih_rnn_ex.restype = i32
    L.linscan_rnn.argtypes = [vp, u64, u32, vp, u32, u32, vp, vp, ctypes.POINTER(vp)]
    L.linscan_rnn.restype = i32
    L.mih_rnn_result_view.argtypes = [vp, ctypes.POINTER(RnnView)]
    L.mih_rnn_result_view.restype = i32
    L.mih_rnn_result_free.argtypes = [vp]
    L.mih_rnn_result_free.restype = None
    L.mih_model_cost.argtypes = [u64, u32, u32, u32]
    L.mih_model_cost.restype = ctypes.c_double
    L.mih_model_radius.argtypes = [u64, u32, u32]
    L.mih_model_radius.restype = u32
    L.mih_choose_m.argtypes = [vp, u64, u32, vp, u32, u32, vp, u32, ctypes.POINTER(BuildOpts), vp,
                               ctypes.POINTER(u32), ctypes.POINTER(MTrial), ctypes.POINTER(u32)]
    L.mih_choose_m.restype = i32
    L.mih_bit_cooccurrence.argtypes = [vp, u64, u32, vp, vp]
    L.mih_bit_cooccurrence.restype = i32
    L.mih_greedy_bit_order.argtypes = [vp, u64, u32, u32, u32, vp]
    L.mih_greedy_bit_order.restype = i32
    L.mih_status_str.argtypes = [i32]
    L.mih_status_str.restype = ctypes.c_char_p
    L.mih_index_get_info.argtypes = [vp, ctypes.POINTER(IndexInfo)]
    L.mih_index_get_info.restype = i32
    L.mih_index_table.argtypes = [vp, u32, ctypes.POINTER(TableView)]
    L.mih_index_table.restype = i32
    L.mih_get_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.mih_get_tuning.restype = i32
    L.mih_set_tuning.argtypes = [vp, ctypes.POINTER(Tuning)]
    L.mih_set_tuning.restype = i32
    L.mih_autotune.argtypes = [vp, vp, u32, u32, vp, vp, ctypes.POINTER(Tuning)]
    L.mih_autotune.restype = i32
    L.mih_server_create.argtypes = [vp, ctypes.POINTER(ServerOpts), vp, ctypes.POINTER(vp)]
    L.mih_server_create.restype = i32
    L.mih_server_submit.argtypes = [vp, vp, u32, u32, vp, vp, vp, ctypes.POINTER(u64)]
    L.mih_server_submit.restype = i32
    L.mih_server_step.argtypes = [vp, vp, u32, ctypes.POINTER(u32)]
    L.mih_server_step.restype = i32
    L.mih_server_poll.argtypes = [vp, u64, ctypes.POINTER(ctypes.c_int)]
    L.mih_server_poll.restype = i32
    L.mih_server_get_stats.argtypes = [vp, ctypes.POINTER(ServerStats)]
    L.mih_server_get_stats.restype = i32
    L.mih_server_destroy.argtypes = [vp]
    L.mih_server_destroy.restype = None
    L.mih_random_read_rate.argtypes = [vp, u64, u64, u32, vp, vp, ctypes.POINTER(ctypes.c_double)]
    L.mih_random_read_rate.restype = i32
    _lib = L
    return L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _codes_arg(t: torch.Tensor, what: str):
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{what} must be int64 or uint64 words, got {t.dtype}")
    if t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous [rows, bits/64] tensor")
    return t


def _k_arg(k, nq: int, device):
    """Returns (scalar k, device k tensor or None, per-query k list)."""
    if isinstance(k, int):
        return k, None, None
    kt = torch.as_tensor(k, dtype=torch.int32)
    if kt.numel() != nq:
        raise ValueError("k_per_query must have one entry per query")
    kl = kt.cpu().tolist()
    return 0, kt.to(device).contiguous(), kl


def _outputs(nq: int, k: int, kl, device):
    total = sum(kl) if kl is not None else nq * k
    ids = torch.empty(max(total, 1), dtype=torch.int32, device=device)
    dists = torch.empty(max(total, 1), dtype=torch.int32, device=device)
    return ids, dists, total


def _shape(ids, dists, total, nq, k, kl):
    ids, dists = ids[:total], dists[:total]
    if kl is None:
        return ids.view(nq, k), dists.view(nq, k)
    return ids, dists


def _check(status: int, what: str):
    if status != 0:
        raise MihError(status, what)


class Index:
    """A multi-index hashing index over device codes (borrowed, kept alive here)."""

    def __init__(self, handle, codes: torch.Tensor):
        self._h = handle
        self.codes = codes

    def close(self):
        if self._h:
            load().mih_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def info(self) -> dict:
        inf = IndexInfo()
        _check(load().mih_index_get_info(self._h, ctypes.byref(inf)), "mih_index_get_info")
        m = inf.m
        return {"n": inf.n, "bits": inf.bits, "m": m,
                "table_mode": {1: "direct", 2: "sorted", 3: "grouped", 4: "heads"}.get(inf.table_mode,
                                                                                      inf.table_mode),
                "codes_mode": {1: "inline", 2: "indirect", 3: "mixed"}.get(inf.codes_mode, inf.codes_mode),
                "inline_tables": inf.inline_tables,
                "sub_len": list(inf.sub_len[:m]), "sub_start": list(inf.sub_start[:m]),
                "dir_bits": list(inf.dir_bits[:m]), "device_bytes": inf.device_bytes,
                "build_ms": inf.build_ms, "bit_order": list(inf.bit_order[:inf.bits])}

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(load().mih_get_tuning(self._h, ctypes.byref(t)), "mih_get_tuning")
        return t.as_dict()

    def set_tuning(self, **fields):
        """Launch tuning (speed only): any fields of mih_tuning (probes_per_lane,
        chunk, blocks_per_cu, occupancy_filter, sweep_shift, sweep_bits,
        lookahead, sweep_queries, buffer_mult, small_batch, round_masks,
        spill_codes); the others keep their value."""
        cur = self.get_tuning()
        for f, v in fields.items():
            if f not in cur:
                raise TypeError(f"unknown tuning field {f!r}")
            if v is not None:
                cur[f] = int(v)
        t = Tuning(**cur)
        _check(load().mih_set_tuning(self._h, ctypes.byref(t)), "mih_set_tuning")

    def autotune(self, queries: torch.Tensor, k) -> dict:
        """Pick the fastest launch tuning on a sample of queries (mih_autotune)."""
        queries = _codes_arg(queries, "queries")
        nq = queries.shape[0]
        kk, kt, _ = _k_arg(k, nq, queries.device)
        t = Tuning()
        _check(load().mih_autotune(self._h, queries.data_ptr(), nq, kk,
                                   kt.data_ptr() if kt is not None else None, _stream(),
                                   ctypes.byref(t)), "mih_autotune")
        return t.as_dict()

    def table(self, j: int) -> dict:
        """Copies of table j's device arrays (as CPU tensors), for inspection."""
        v = TableView()
        _check(load().mih_index_table(self._h, j, ctypes.byref(v)), "mih_index_table")
        n = self.codes.shape[0]
        W = self.codes.shape[1]
        out = {"len": v.len, "start": v.start, "dir_bits": v.dir_bits}
        out["ids"] = _copy_device(v.ids, n, torch.int32)
        if v.offsets:
            out["offsets"] = _copy_device(v.offsets, (1 << v.len) + 1, torch.int32)
        if v.keys:
            out["keys"] = _copy_device(v.keys, n, torch.int32)
        if v.dir:
            out["dir"] = _copy_device(v.dir, (1 << v.dir_bits) + 1, torch.int32)
        if v.codes:
            out["codes"] = _copy_device(v.codes, n * W, torch.int64).view(n, W)
        if v.occupancy:
            out["occupancy"] = _copy_device(v.occupancy, max((1 << v.len) // 32, 1), torch.int32)
        if v.groups:
            out["groups"] = _copy_device(v.groups, max((1 << v.len) // 32, 1), torch.int64)
        if v.heads:
            out["heads"] = _copy_device(v.heads, 2 * ((1 << v.len) + 1), torch.int64).view(-1, 2)
        return out

    def rnn(self, queries: torch.Tensor, r, stats: bool = False):
        """Every code within distance r (an int or one radius per query) of
        each query.  Returns (offsets, ids, dists) as device tensors: query
        i's results are ids[offsets[i]:offsets[i+1]] in ascending (distance,
        id) order; with stats=True a dict of search counters is appended."""
        queries = _codes_arg(queries, "queries")
        if queries.shape[1] != self.codes.shape[1]:
            raise ValueError("queries and codes differ in length")
        nq = queries.shape[0]
        rr, rt = _r_arg(r, nq, queries.device)
        st = QueryStats()
        h = ctypes.c_void_p()
        rc = load().mih_rnn_ex(self._h, queries.data_ptr() if nq else None, nq, rr,
                               rt.data_ptr() if rt is not None else None, _stream(),
                               ctypes.byref(h), ctypes.byref(st))
        _check(rc, "mih_rnn")
        out = _take_rnn(h, queries.device)
        return (*out, st.as_dict()) if stats else out

    def knn_approx(self, queries: torch.Tensor, k, max_radius: int | None = None,
                   max_candidates: int = 0, stats: bool = False):
        """Approximate kNN (Section 7): stop after the step covering
        max_radius, or once max_candidates distinct codes were met."""
        queries = _codes_arg(queries, "queries")
        if queries.shape[1] != self.codes.shape[1]:
            raise ValueError("queries and codes differ in length")
        nq = queries.shape[0]
        kk, kt, kl = _k_arg(k, nq, queries.device)
        ids, dists, total = _outputs(nq, kk, kl, queries.device)
        st = QueryStats()
        rc = load().mih_knn_approx(self._h, queries.data_ptr(), nq, kk,
                                   kt.data_ptr() if kt is not None else None,
                                   0xFFFFFFFF if max_radius is None else max_radius, max_candidates,
                                   ids.data_ptr(), dists.data_ptr(), _stream(), ctypes.byref(st))
        _check(rc, "mih_knn_approx")
        out = _shape(ids, dists, total, nq, kk, kl)
        return (*out, st.as_dict()) if stats else out

    def knn(self, queries: torch.Tensor, k, stats: bool = False):
        """Exact kNN; k is an int or a per-query sequence (then rows are flat)."""
        queries = _codes_arg(queries, "queries")
        if queries.shape[1] != self.codes.shape[1]:
            raise ValueError("queries and codes differ in length")
        nq = queries.shape[0]
        kk, kt, kl = _k_arg(k, nq, queries.device)
        ids, dists, total = _outputs(nq, kk, kl, queries.device)
        st = QueryStats()
        rc = load().mih_knn_ex(self._h, queries.data_ptr(), nq, kk,
                               kt.data_ptr() if kt is not None else None,
                               ids.data_ptr(), dists.data_ptr(), _stream(), ctypes.byref(st))
        _check(rc, "mih_knn")
        ids, dists = _shape(ids, dists, total, nq, kk, kl)
        return (ids, dists, st.as_dict()) if stats else (ids, dists)


def build(codes: torch.Tensor, m: int, table_mode: str = "auto", codes_mode: str = "auto",
          mem_budget_bytes: int = 0, bit_order=None, inline_tables: int = 0,
          autotune_cache: str | None = None) -> Index:
    """Build the m substring tables (Algorithm 1) on the device; bit_order
    (a permutation of the code bits, Section 5.5) places the substrings;
    codes_mode "mixed" keeps inline codes in the first inline_tables tables;
    autotune_cache: a file where autotune() keeps and looks up its results."""
    codes = _codes_arg(codes, "codes")
    n, W = codes.shape
    order = None
    if bit_order is not None:
        if len(bit_order) != 64 * W:
            raise ValueError("bit_order must list every code bit once")
        order = (ctypes.c_uint16 * (64 * W))(*[int(b) for b in bit_order])
    opts = BuildOpts(TABLE_MODES[table_mode], CODES_MODES[codes_mode], mem_budget_bytes,
                     ctypes.cast(order, ctypes.c_void_p) if order is not None else None, inline_tables,
                     autotune_cache.encode() if autotune_cache else None)
    h = ctypes.c_void_p()
    rc = load().mih_build(codes.data_ptr() if n else None, n, 64 * W, m, ctypes.byref(opts),
                          _stream(), ctypes.byref(h))
    _check(rc, "mih_build")
    return Index(h, codes)


def bit_cooccurrence(codes: torch.Tensor):
    """counts[i, j] = number of codes with bits i and j set (numpy uint32 [bits, bits])."""
    import numpy as np
    codes = _codes_arg(codes, "codes")
    n, W = codes.shape
    bits = 64 * W
    out = np.zeros((bits, bits), dtype=np.uint32)
    _check(load().mih_bit_cooccurrence(codes.data_ptr() if n else None, n, bits, _stream(),
                                       out.ctypes.data), "mih_bit_cooccurrence")
    return out


def greedy_bit_order(counts, n: int, m: int, first_bit: int = 0):
    """The Section 5.5 greedy bit order from co-occurrence counts of n codes."""
    import numpy as np
    counts = np.ascontiguousarray(counts, dtype=np.uint32)
    bits = counts.shape[0]
    order = np.zeros(bits, dtype=np.uint16)
    _check(load().mih_greedy_bit_order(counts.ctypes.data, n, bits, m, first_bit, order.ctypes.data),
           "mih_greedy_bit_order")
    return order.tolist()


def optimize_substrings(codes: torch.Tensor, m: int, sample: int = 1_000_000, first_bit: int = 0):
    """Bit order for build(): counts over the first `sample` codes, then the greedy order."""
    n = min(sample, codes.shape[0])
    counts = bit_cooccurrence(codes[:n])
    return greedy_bit_order(counts, n, m, first_bit)


def model_cost(n: int, bits: int, m: int, r: int) -> float:
    """Eq. 6 cost (in lookups) of searching radius r with m tables over n uniform codes."""
    return load().mih_model_cost(n, bits, m, r)


def model_radius(n: int, bits: int, k: int) -> int:
    """Smallest r with at least k expected uniform codes within distance r."""
    return load().mih_model_radius(n, bits, k)


def choose_m(codes: torch.Tensor, k: int, queries: torch.Tensor | None = None,
             validation: int = 1000, candidates=None, table_mode: str = "auto",
             codes_mode: str = "auto", seed: int = 0):
    """Pick m by building and timing each candidate (Section 6).  Without
    `queries`, `validation` database rows chosen with a seeded permutation
    serve as the validation queries.  Returns (best m, list of trial dicts)."""
    codes = _codes_arg(codes, "codes")
    n, W = codes.shape
    if queries is None:
        g = torch.Generator(device="cpu").manual_seed(seed)
        rows = torch.randperm(n, generator=g)[:min(validation, n)].to(codes.device)
        queries = codes.index_select(0, rows).contiguous()
    queries = _codes_arg(queries, "queries")
    cand = None
    nc = 0
    if candidates is not None:
        nc = len(candidates)
        cand = (ctypes.c_uint32 * max(nc, 1))(*candidates)
    opts = BuildOpts(TABLE_MODES[table_mode], CODES_MODES[codes_mode], 0)
    best = ctypes.c_uint32()
    ntr = ctypes.c_uint32()
    trials = (MTrial * M_TRIALS_MAX)()
    rc = load().mih_choose_m(codes.data_ptr() if n else None, n, 64 * W, queries.data_ptr(),
                             queries.shape[0], k, cand, nc, ctypes.byref(opts), _stream(),
                             ctypes.byref(best), trials, ctypes.byref(ntr))
    _check(rc, "mih_choose_m")
    return best.value, [trials[i].as_dict() for i in range(ntr.value)]


def _r_arg(r, nq: int, device):
    """Returns (scalar r, device radius tensor or None)."""
    if isinstance(r, int):
        if r < 0:
            raise ValueError("r must be non-negative")
        return r, None
    rt = torch.as_tensor(r, dtype=torch.int64)
    if rt.numel() != nq:
        raise ValueError("r_per_query must have one entry per query")
    if (rt < 0).any():
        raise ValueError("radii must be non-negative")
    return 0, rt.clamp(max=0xFFFFFFFF).to(torch.int32).to(device).contiguous()


def _take_rnn(handle, device):
    """Device copies (offsets int64 [nq+1], ids int32, dists int32) of a
    library-owned r-neighbour result, which is then released."""
    L = load()
    try:
        v = RnnView()
        _check(L.mih_rnn_result_view(handle, ctypes.byref(v)), "mih_rnn_result_view")
        offsets = torch.empty(v.nq + 1, dtype=torch.int64, device=device)
        ids = torch.empty(v.total, dtype=torch.int32, device=device)
        dists = torch.empty(v.total, dtype=torch.int32, device=device)
        torch.cuda.synchronize(device)
        for dst, src, nbytes in ((offsets, v.offsets, 8 * (v.nq + 1)), (ids, v.ids, 4 * v.total),
                                 (dists, v.dists, 4 * v.total)):
            if nbytes:
                rc = _hip_runtime().hipMemcpy(dst.data_ptr(), src, nbytes, 3)   # device to device
                if rc != 0:
                    raise RuntimeError(f"hipMemcpy failed ({rc})")
        return offsets, ids, dists
    finally:
        L.mih_rnn_result_free(handle)


def linscan_rnn(codes: torch.Tensor, queries: torch.Tensor, r):
    """Every code within distance r of each query, by the GPU linear scan.
    Returns (offsets, ids, dists): query i's results are ids[offsets[i]:offsets[i+1]]
    in ascending (distance, id) order."""
    codes = _codes_arg(codes, "codes")
    queries = _codes_arg(queries, "queries")
    if queries.shape[1] != codes.shape[1]:
        raise ValueError("queries and codes differ in length")
    n, W = codes.shape
    nq = queries.shape[0]
    rr, rt = _r_arg(r, nq, queries.device)
    h = ctypes.c_void_p()
    rc = load().linscan_rnn(codes.data_ptr() if n else None, n, 64 * W,
                            queries.data_ptr() if nq else None, nq, rr,
                            rt.data_ptr() if rt is not None else None, _stream(), ctypes.byref(h))
    _check(rc, "linscan_rnn")
    return _take_rnn(h, queries.device)


def linscan_knn(codes: torch.Tensor, queries: torch.Tensor, k, stats: bool = False):
    """Exact kNN by the GPU linear scan."""
    codes = _codes_arg(codes, "codes")
    queries = _codes_arg(queries, "queries")
    if queries.shape[1] != codes.shape[1]:
        raise ValueError("queries and codes differ in length")
    n, W = codes.shape
    nq = queries.shape[0]
    kk, kt, kl = _k_arg(k, nq, queries.device)
    ids, dists, total = _outputs(nq, kk, kl, queries.device)
    st = ScanStats()
    rc = load().linscan_knn_ex(codes.data_ptr() if n else None, n, 64 * W, queries.data_ptr(), nq,
                               kk, kt.data_ptr() if kt is not None else None, ids.data_ptr(),
                               dists.data_ptr(), _stream(), ctypes.byref(st))
    _check(rc, "linscan_knn")
    ids, dists = _shape(ids, dists, total, nq, kk, kl)
    return (ids, dists, st.as_dict()) if stats else (ids, dists)


def linscan_knn_noalloc(codes: torch.Tensor, queries: torch.Tensor, k, out=None):
    """linscan_knn through the entry point that allocates no device memory
    (its buffers sit in a fixed array of the library).  ``out``: optional
    preallocated (ids, dists) int32 tensors of the right size, so that the
    call itself allocates nothing anywhere."""
    codes = _codes_arg(codes, "codes")
    queries = _codes_arg(queries, "queries")
    if queries.shape[1] != codes.shape[1]:
        raise ValueError("queries and codes differ in length")
    n, W = codes.shape
    nq = queries.shape[0]
    kk, kt, kl = _k_arg(k, nq, queries.device)
    if out is None:
        ids, dists, total = _outputs(nq, kk, kl, queries.device)
    else:
        ids, dists = out
        total = ids.numel()
    rc = load().linscan_knn_noalloc(codes.data_ptr() if n else None, n, 64 * W, queries.data_ptr(), nq,
                                    kk, kt.data_ptr() if kt is not None else None, ids.data_ptr(),
                                    dists.data_ptr(), _stream())
    _check(rc, "linscan_knn_noalloc")
    return _shape(ids, dists, total, nq, kk, kl)


def random_read_rate(array: torch.Tensor, reads: int, depth: int = 8) -> dict:
    """The device's rate of independent random 64-byte line reads from
    ``array`` (a device tensor; a measurement helper, mih_random_read_rate)."""
    if not array.is_cuda or not array.is_contiguous() or array.element_size() * array.numel() < 64:
        raise ValueError("array must be a contiguous device tensor of at least 64 bytes")
    sink = torch.zeros(1, dtype=torch.int64, device=array.device)
    ms = ctypes.c_double()
    words = array.numel() * array.element_size() // 8
    _check(load().mih_random_read_rate(array.data_ptr(), words, reads, depth, sink.data_ptr(), _stream(),
                                       ctypes.byref(ms)), "mih_random_read_rate")
    threads = torch.cuda.get_device_properties(array.device).multi_processor_count * 8 * 256
    per_lane = -(-reads // threads)
    per_lane = -(-per_lane // depth) * depth
    done = per_lane * threads
    return {"reads": done, "ms": ms.value, "reads_per_s": done / (ms.value / 1e3), "depth": depth}


# ------------------------------------------------------------------ serving

class ServerOpts(ctypes.Structure):
    _fields_ = [("max_queries", ctypes.c_uint32), ("use_graph", ctypes.c_uint32),
                ("buffer_entries", ctypes.c_uint64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("probes", ctypes.c_uint64), ("candidates", ctypes.c_uint64),
                ("completed_requests", ctypes.c_uint64), ("rounds", ctypes.c_uint32),
                ("in_flight", ctypes.c_uint32), ("pending_queries", ctypes.c_uint32),
                ("reruns", ctypes.c_uint32), ("search_kernel_ms", ctypes.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class Server:
    """Continuous-batching server over an index (mih_server_* in the C ABI).

    submit() queues a request and returns its ticket; step() admits what fits,
    runs one device round and returns the tickets completed in it.  Each
    request's (ids, dists) tensors are available from result(ticket) once
    completed.
    """

    def __init__(self, index: Index, max_queries: int = 4096, buffer_entries: int = 0,
                 use_graph: bool = True):
        L = load()
        self.index = index
        self._h = ctypes.c_void_p()
        opts = ServerOpts(max_queries, 1 if use_graph else 0, buffer_entries)
        _check(L.mih_server_create(index._h, ctypes.byref(opts), _stream(), ctypes.byref(self._h)),
               "mih_server_create")
        self._live = {}      # ticket -> (queries, ids, dists, shape)
        self._done = {}

    def close(self):
        if self._h:
            load().mih_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, queries: torch.Tensor, k) -> int:
        queries = _codes_arg(queries, "queries")
        nq = queries.shape[0]
        if isinstance(k, int):
            kk, karr, kl = k, None, None
        else:
            kl = [int(x) for x in k]
            kk, karr = 0, (ctypes.c_uint32 * nq)(*kl)
        ids, dists, total = _outputs(nq, kk, kl, queries.device)
        t = ctypes.c_uint64()
        _check(load().mih_server_submit(self._h, queries.data_ptr(), nq, kk, karr, ids.data_ptr(),
                                        dists.data_ptr(), ctypes.byref(t)), "mih_server_submit")
        self._live[t.value] = (queries, ids, dists, (total, nq, kk, kl))
        return t.value

    def step(self, max_completed: int = 4096):
        buf = (ctypes.c_uint64 * max_completed)()
        n = ctypes.c_uint32()
        _check(load().mih_server_step(self._h, buf, max_completed, ctypes.byref(n)), "mih_server_step")
        out = [buf[i] for i in range(n.value)]
        for t in out:
            q, ids, dists, shape = self._live.pop(t)
            self._done[t] = _shape(ids, dists, *shape)
        return out

    def result(self, ticket: int):
        return self._done.pop(ticket)

    def done(self, ticket: int) -> bool:
        d = ctypes.c_int()
        _check(load().mih_server_poll(self._h, ticket, ctypes.byref(d)), "mih_server_poll")
        return bool(d.value)

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().mih_server_get_stats(self._h, ctypes.byref(st)), "mih_server_get_stats")
        return st.as_dict()

    def drain(self):
        """Step until every submitted request has completed."""
        done = []
        while self._live:
            done += self.step()
        return done


# ------------------------------------------------------------------ plumbing

_hip = None


def _hip_runtime():
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so.7")   # the runtime torch has loaded
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    return _hip


def _copy_device(ptr, count: int, dtype) -> torch.Tensor:
    """Copy `count` elements at a device pointer owned by the library to CPU."""
    out = torch.empty(max(count, 1), dtype=dtype, device="cuda")
    nbytes = count * out.element_size()
    if nbytes:
        torch.cuda.synchronize()
        rc = _hip_runtime().hipMemcpy(out.data_ptr(), ptr, nbytes, 3)   # device to device
        if rc != 0:
            raise RuntimeError(f"hipMemcpy failed ({rc})")
    return out[:count].cpu()
