"""Parity at the full sizes of the benchmark workloads, in the launch
configuration bench.py times (autotuned tuning, the whole query batch in one
call): every query against the oracle where it finishes in seconds (1e6 x
64-bit, 1e7 x 128-bit clustered), sampled queries against the oracle
elsewhere, and the whole batch against the GPU linear scan (a second,
independent kernel) at every size."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import as_u32, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def check_rows(ids, dists, ks, sel, codes, queries, what):
    ks = np.asarray(ks, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(ks)])
    gi, gd = as_u32(ids), as_u32(dists)
    oi, od = oracle.knn(codes, queries[sel], ks[sel], threads=16)
    o = 0
    for q in sel:
        k = int(ks[q])
        assert np.array_equal(gi[off[q]:off[q] + k], oi[o:o + k]), f"{what}: query {q} ids"
        assert np.array_equal(gd[off[q]:off[q] + k], od[o:o + k]), f"{what}: query {q} distances"
        o += k


def sample(nq, count, seed):
    return np.sort(np.argsort(datagen.uniform_f64(nq, seed), kind="stable")[:count])


def same_as_linscan(mih, dc, dq, k, ids, dists, what):
    import torch
    li, ld = mih.linscan_knn(dc, dq, k)
    assert torch.equal(li, ids) and torch.equal(ld, dists), f"{what}: MIH differs from the linear scan"


def test_fullsize_1e6_uniform_64bit_m3_every_query(mih):
    cfg = datagen.CONFIGS[1]
    n, nq = cfg["n"], cfg["nq"]
    codes = datagen.uniform_codes(n, 64, datagen.SEED_DB_UNIFORM, threads=16)
    queries = datagen.uniform_codes(nq, 64, datagen.SEED_Q_UNIFORM)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, cfg["m"])
    ks = datagen.choice_u32(nq, cfg["ks"], datagen.SEED_K)
    idx.autotune(to_dev(datagen.uniform_codes(nq, 64, datagen.SEED_Q_UNIFORM, first_row=nq)), ks.tolist())
    for k in list(cfg["ks"]) + [ks.tolist()]:
        ids, dists = idx.knn(dq, k)
        kk = np.full(nq, k, dtype=np.uint32) if isinstance(k, int) else ks
        check_rows(ids, dists, kk, np.arange(nq), codes, queries, f"1e6 k={k if isinstance(k, int) else 'mixed'}")
        same_as_linscan(mih, dc, dq, k, ids, dists, "1e6")
    idx.close()


def test_fullsize_1e7_clustered_128bit_m6_every_query(mih):
    import torch
    cfg = datagen.CONFIGS[2]
    n, nq = cfg["n"], cfg["nq"]
    codes = datagen.db_codes("clustered", n, 128, threads=16)
    queries = datagen.query_codes("clustered", nq, 128, threads=16)
    ks = datagen.choice_u32(nq, cfg["ks"], datagen.SEED_K)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, cfg["m"])
    idx.autotune(to_dev(datagen.query_codes("clustered", 2000, 128, first_row=nq)), ks[:2000].tolist())
    ids, dists = idx.knn(dq, ks.tolist())
    # every query against the oracle (1e11 distances on the host)
    gi, gd = as_u32(ids), as_u32(dists)
    oi, od = oracle.knn(codes, queries, ks, threads=16)
    bad = np.nonzero((gi != oi) | (gd != od))[0]
    assert len(bad) == 0, f"1e7 clustered: {len(bad)} entries differ from the oracle, first at {bad[:1]}"
    same_as_linscan(mih, dc, dq, ks.tolist(), ids, dists, "1e7 clustered")
    idx.close()
    del dc
    torch.cuda.empty_cache()


def test_fullsize_1e9_uniform_64bit_m2(mih):
    import torch
    cfg = datagen.CONFIGS[4]
    n, nq = cfg["n"], cfg["nq"]
    codes = datagen.uniform_codes(n, 64, datagen.SEED_DB_UNIFORM, threads=16)
    queries = datagen.uniform_codes(nq, 64, datagen.SEED_Q_UNIFORM)
    queries[7] = codes[123_456_789]          # a query equal to a database code
    dc = datagen.codes_device("uniform", n, 64, datagen.SEED_DB_UNIFORM)
    dq = to_dev(queries)
    idx = mih.build(dc, cfg["m"])
    idx.autotune(dq[:2000], 100)
    ids, dists = idx.knn(dq, 100)
    same_as_linscan(mih, dc, dq, 100, ids, dists, "1e9 k=100")
    sel = np.concatenate([[7], sample(nq, 200, 101)])
    check_rows(ids, dists, [100] * nq, sel, codes, queries, "1e9 k=100")
    assert int(as_u32(dists)[700]) == 0 and int(as_u32(ids)[700]) <= 123_456_789
    # the largest k on a few queries; r-neighbours of two
    few = dq[sel[:3]].contiguous()
    ids, dists = idx.knn(few, 4096)
    check_rows(ids, dists, [4096] * 3, np.arange(3), codes, queries[sel[:3]], "1e9 k=4096")
    off, rid, rd = idx.rnn(few, 11)
    for i in range(2):
        oi, od = oracle.rnn(codes, queries[sel[i]], 11)
        a, b = int(off[i]), int(off[i + 1])
        assert np.array_equal(as_u32(rid[a:b]), oi) and np.array_equal(as_u32(rd[a:b]), od)
    idx.close()
    del dc
    torch.cuda.empty_cache()


def test_fullsize_1e8_uniform_mixed_k(mih):
    import torch
    cfg = datagen.CONFIGS[3]
    n, nq = cfg["n"], cfg["nq"]
    codes = datagen.uniform_codes(n, 64, datagen.SEED_DB_UNIFORM, threads=16)
    queries = datagen.uniform_codes(nq, 64, datagen.SEED_Q_UNIFORM)
    ks = datagen.choice_u32(nq, cfg["ks"], datagen.SEED_K)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, cfg["m"])
    idx.autotune(dq[:2000], ks[:2000].tolist())
    ids, dists = idx.knn(dq, ks.tolist())
    same_as_linscan(mih, dc, dq, ks.tolist(), ids, dists, "1e8 mixed k")
    check_rows(ids, dists, ks, sample(nq, 1000, 102), codes, queries, "1e8 mixed k")
    idx.close()
    torch.cuda.empty_cache()


def test_fullsize_1e9_clustered_256bit_m8(mih):
    import torch
    cfg = datagen.CONFIGS[5]
    n, nq = cfg["n"], cfg["nq"]
    dc = datagen.codes_device("clustered", n, 256, datagen.SEED_DB_CLUSTERED)
    queries = datagen.query_codes("clustered", nq, 256)
    ks = datagen.choice_u32(nq, cfg["ks"], datagen.SEED_K)
    dq = to_dev(queries)
    idx = mih.build(dc, cfg["m"])
    idx.autotune(dq[:2000], ks[:2000].tolist())
    ids, dists = idx.knn(dq, ks.tolist())
    same_as_linscan(mih, dc, dq, ks.tolist(), ids, dists, "1e9 x 256 clustered")
    codes = dc.cpu().numpy().view(np.uint64)
    check_rows(ids, dists, ks, sample(nq, 24, 103), codes, queries, "1e9 x 256 clustered")
    idx.close()
    del dc
    torch.cuda.empty_cache()
