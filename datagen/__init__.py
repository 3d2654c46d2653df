"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Only input generation lives here (SplitMix64 streams, uniform and clustered
codes, per-query k draws, request streams); none of the search method's
arithmetic does.  The generator definitions are in ``gen.c``.

Workloads (the paper's datasets, SIFT 1B and Gist 80M, are not available, so
these synthetic sets stand in for them, Section 5.1):

* uniform: every bit i.i.d. Bernoulli(1/2), the regime of the analysis in
  Section 3 (expected N / 2^s items per bucket);
* clustered: sign-of-random-projection codes of points drawn from a
  1000-component isotropic Gaussian mixture in 128-D (sigma 0.3), the
  construction of LSH codes described in Section 5.1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libdatagen.so")
_lib_handle = None

SEED_DB_UNIFORM = 0
SEED_Q_UNIFORM = 1
SEED_DB_CLUSTERED = 4
SEED_Q_CLUSTERED = 5
SEED_K = 6
SEED_ARRIVALS = 7
SEED_SIZES = 8


_DEV_SO = os.path.join(_HERE, "libdatagen_dev.so")
_dev_handle = None


def build(force: bool = True) -> str:
    """Compile ``gen.c`` into ``libdatagen.so`` (gcc) and ``gen_device.hip``
    into ``libdatagen_dev.so`` (hipcc, gfx950)."""
    if force or not os.path.exists(_SO):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
               os.path.join(_HERE, "gen.c"), "-o", _SO + ".tmp"]
        subprocess.run(cmd, check=True)
        os.replace(_SO + ".tmp", _SO)
    if force or not os.path.exists(_DEV_SO):
        hipcc = "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc"
        cmd = [hipcc, "--offload-arch=gfx950", "-O3", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               os.path.join(_HERE, "gen_device.hip"), "-o", _DEV_SO + ".tmp"]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(_DEV_SO + ".tmp", _DEV_SO)
    return _SO


def _dev_lib():
    """The device generators (load after torch, which owns the HIP runtime)."""
    global _dev_handle
    if _dev_handle is None:
        import torch  # noqa: F401  (the HIP runtime torch has loaded is shared)
        if not os.path.exists(_DEV_SO):
            build(force=False)
        L = ctypes.CDLL(_DEV_SO)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.dg_dev_uniform.argtypes = [vp, u64, u32, u64, u64, vp]
        L.dg_dev_points.argtypes = [vp, u64, u64, u64, vp, vp]
        L.dg_dev_pack.argtypes = [vp, vp, u64, u32, vp]
        for f in (L.dg_dev_uniform, L.dg_dev_points, L.dg_dev_pack):
            f.restype = ctypes.c_int
        _dev_handle = L
    return _dev_handle


def codes_device(kind: str, n: int, bits: int, seed: int, first_row: int = 0,
                 chunk: int = 1 << 22):
    """The same rows as uniform_codes / clustered_codes, generated on cuda:0
    into an int64 tensor [n, bits/64].  Clustered rows go through an exact
    fp64 matrix product (see gen_device.hip)."""
    import torch
    words = _check_bits(bits)
    L = _dev_lib()
    out = torch.empty((n, words), dtype=torch.int64, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if n == 0:
        return out
    if kind == "uniform":
        rc = L.dg_dev_uniform(out.data_ptr(), n, words, seed, first_row, stream)
        if rc:
            raise RuntimeError(f"dg_dev_uniform failed ({rc})")
        return out
    if kind != "clustered":
        raise ValueError(kind)
    mu, w = clustered_params(bits)
    mu_d = torch.from_numpy(mu).cuda()
    wt_d = torch.from_numpy(w.T.astype(np.float64)).cuda().contiguous()   # [128, bits]
    for p0 in range(0, n, chunk):
        m = min(chunk, n - p0)
        x = torch.empty((m, 128), dtype=torch.float64, device="cuda")
        rc = L.dg_dev_points(x.data_ptr(), m, seed, first_row + p0, mu_d.data_ptr(), stream)
        if rc:
            raise RuntimeError(f"dg_dev_points failed ({rc})")
        dots = torch.matmul(x, wt_d)
        rc = L.dg_dev_pack(out[p0:p0 + m].data_ptr(), dots.data_ptr(), m, bits, stream)
        if rc:
            raise RuntimeError(f"dg_dev_pack failed ({rc})")
        del x, dots
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build(force=True)
        L = ctypes.CDLL(_SO)
        u64, u32, i32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p
        L.dg_splitmix.argtypes = [u64, u64]
        L.dg_splitmix.restype = u64
        L.dg_gauss_public.argtypes = [u64, u64]
        L.dg_gauss_public.restype = ctypes.c_int64
        L.dg_uniform.argtypes = [vp, u64, u32, u64, u64, i32]
        L.dg_uniform.restype = None
        L.dg_clustered.argtypes = [vp, u64, u32, u64, u64, i32]
        L.dg_clustered.restype = i32
        L.dg_clustered_params.argtypes = [vp, vp, u32]
        L.dg_clustered_params.restype = None
        L.dg_choice_u32.argtypes = [vp, u64, vp, u32, u64, u64]
        L.dg_choice_u32.restype = None
        L.dg_uniform_f64.argtypes = [vp, u64, u64, u64]
        L.dg_uniform_f64.restype = None
        _lib_handle = L
    return _lib_handle


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def splitmix(seed: int, counter: int) -> int:
    return int(_lib().dg_splitmix(seed, counter))


def gauss(seed: int, counter: int) -> int:
    return int(_lib().dg_gauss_public(seed, counter))


def _check_bits(bits: int) -> int:
    if bits <= 0 or bits % 64 != 0 or bits > 256:
        raise ValueError(f"bits must be 64, 128, 192 or 256, got {bits}")
    return bits // 64


def uniform_codes(n: int, bits: int, seed: int, first_row: int = 0,
                  threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Rows [first_row, first_row+n) of the uniform code stream, as uint64 [n, bits/64]."""
    words = _check_bits(bits)
    if out is None:
        out = np.empty((n, words), dtype=np.uint64)
    assert out.dtype == np.uint64 and out.flags.c_contiguous and out.shape == (n, words)
    if n:
        _lib().dg_uniform(out.ctypes.data, n, words, seed, first_row,
                          threads or default_threads())
    return out


def clustered_codes(n: int, bits: int, seed: int, first_row: int = 0,
                    threads: int | None = None, out: np.ndarray | None = None) -> np.ndarray:
    """Rows of the clustered (Gaussian-mixture sign-projection) code stream."""
    words = _check_bits(bits)
    if out is None:
        out = np.empty((n, words), dtype=np.uint64)
    assert out.dtype == np.uint64 and out.flags.c_contiguous and out.shape == (n, words)
    if n:
        rc = _lib().dg_clustered(out.ctypes.data, n, bits, seed, first_row,
                                 threads or default_threads())
        if rc != 0:
            raise MemoryError("dg_clustered failed")
    return out


def clustered_params(bits: int):
    """The mixture means [1000,128] and hyperplanes [bits,128] (int64, scaled)."""
    _check_bits(bits)
    mu = np.empty((1000, 128), dtype=np.int64)
    w = np.empty((bits, 128), dtype=np.int64)
    _lib().dg_clustered_params(mu.ctypes.data, w.ctypes.data, bits)
    return mu, w


def choice_u32(n: int, choices, seed: int, first: int = 0) -> np.ndarray:
    ch = np.ascontiguousarray(np.asarray(choices, dtype=np.uint32))
    out = np.empty(n, dtype=np.uint32)
    if n:
        _lib().dg_choice_u32(out.ctypes.data, n, ch.ctypes.data, len(ch), seed, first)
    return out


def uniform_f64(n: int, seed: int, first: int = 0) -> np.ndarray:
    out = np.empty(n, dtype=np.float64)
    if n:
        _lib().dg_uniform_f64(out.ctypes.data, n, seed, first)
    return out


def request_stream(n_requests: int, rate_per_s: float, k_choices, max_size: int = 4096,
                   seed_arrivals: int = SEED_ARRIVALS, seed_sizes: int = SEED_SIZES,
                   seed_k: int = SEED_K):
    """Poisson arrivals with log-uniform request sizes in [1, max_size].

    Returns (arrival_times_s, sizes, ks) as numpy arrays.  Inter-arrival gaps
    are exponential with the given rate; size = floor(exp(U * ln(max_size+1)))
    clipped to [1, max_size]; each request carries one k drawn from k_choices.
    """
    u = uniform_f64(n_requests, seed_arrivals)
    gaps = -np.log(u) / float(rate_per_s)
    arrivals = np.cumsum(gaps)
    v = uniform_f64(n_requests, seed_sizes)
    sizes = np.floor(np.exp(v * np.log(max_size + 1.0))).astype(np.int64)
    sizes = np.clip(sizes, 1, max_size)
    ks = choice_u32(n_requests, k_choices, seed_k)
    return arrivals, sizes, ks


# The five workloads, with the seeds that define them.
CONFIGS = {
    1: dict(name="C1 uniform 1e6 x 64b, m=3", n=1_000_000, bits=64, m=3, kind="uniform",
            nq=100, ks=(1, 10, 100)),
    2: dict(name="C2 clustered 1e7 x 128b, m=6", n=10_000_000, bits=128, m=6, kind="clustered",
            nq=10_000, ks=(1, 10, 100)),
    3: dict(name="C3 uniform 1e8 x 64b, m=3, mixed k", n=100_000_000, bits=64, m=3, kind="uniform",
            nq=100_000, ks=(1, 10, 100, 1000)),
    4: dict(name="C4 uniform 1e9 x 64b, m=2", n=1_000_000_000, bits=64, m=2, kind="uniform",
            nq=10_000, ks=(100,)),
    5: dict(name="C5 clustered 1e9 x 256b, m=8", n=1_000_000_000, bits=256, m=8, kind="clustered",
            nq=10_000, ks=(1, 10, 100)),
}


def db_codes(kind: str, n: int, bits: int, first_row: int = 0, threads: int | None = None,
             out: np.ndarray | None = None) -> np.ndarray:
    if kind == "uniform":
        return uniform_codes(n, bits, SEED_DB_UNIFORM, first_row, threads, out)
    if kind == "clustered":
        return clustered_codes(n, bits, SEED_DB_CLUSTERED, first_row, threads, out)
    raise ValueError(kind)


def query_codes(kind: str, n: int, bits: int, first_row: int = 0, threads: int | None = None) -> np.ndarray:
    if kind == "uniform":
        return uniform_codes(n, bits, SEED_Q_UNIFORM, first_row, threads)
    if kind == "clustered":
        return clustered_codes(n, bits, SEED_Q_CLUSTERED, first_row, threads)
    raise ValueError(kind)
