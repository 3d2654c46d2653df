"""Seeded random configurations through the C ABI against the oracle.

Each case draws a code length, database size and kind (uniform, clustered,
or a small pool of codes repeated many times, so that distances tie and
buckets overflow), a number of substrings, table and codes modes, a launch
tuning (probes per lane, chunk, occupancy filter, sweep, lookahead), inline,
indirect or mixed candidate codes, queries
that include exact copies and near copies of database codes, per-query k
(k = 0 and k > n among them) and an r-neighbour radius.  Every kNN row (of
the multi-index search and of the linear scan) and every r-neighbour list
must equal the oracle's, ids and distances both.
"""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import as_u32, assert_same, to_dev

pytestmark = pytest.mark.gpu

SEED = 20131002
CASES = 120


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def draw(rng):
    bits = int(rng.choice([64, 128, 192, 256]))
    W = bits // 64
    # substrings of at most 24 bits for the dense tables (their arrays have
    # 2^s entries), up to 32 bits for SORTED tables
    tmode = str(rng.choice(["direct", "sorted", "grouped"] + (["heads"] if bits == 64 else [])))
    smax = 32 if tmode == "sorted" else 24
    m_lo = -(-bits // smax)
    m = int(rng.integers(m_lo, min(m_lo + 6, 64) + 1))
    cmode = "inline" if tmode in ("grouped", "heads") else str(rng.choice(["inline", "indirect", "mixed"]))
    inline_tables = int(rng.integers(1, m)) if cmode == "mixed" and m > 1 else 0
    if cmode == "mixed" and m == 1:
        cmode = "inline"
    n = int(rng.choice([1, 2, 3, 17, 257, 4097, 20_000, 60_000]))
    nq = int(rng.integers(1, 41))
    kind = str(rng.choice(["uniform", "clustered", "pool"]))
    J = int(rng.choice([4, 8, 16]))
    tuning = dict(probes_per_lane=J, chunk=64 * J * int(rng.choice([1, 2, 8])), blocks_per_cu=0,
                  occupancy_filter=int(rng.integers(0, 2)), sweep_shift=int(rng.choice([0, 0, 9])),
                  sweep_bits=18, lookahead=int(rng.choice([1, 3, 16, 32])))
    # partition size and queries per item of the sweeps, from the draws so far
    tuning["sweep_bits"] = (12, 16, 18)[m % 3]
    tuning["sweep_queries"] = 64 * (1 + (7 * J + m) % 6)
    tuning["small_batch"] = (0, 512)[m % 2]   # device rounds, or one launch for these small batches
    return dict(bits=bits, W=W, m=m, tmode=tmode, cmode=cmode, inline_tables=inline_tables, n=n, nq=nq,
                kind=kind, tuning=tuning)


def make_data(rng, c, case):
    n, bits, nq = c["n"], c["bits"], c["nq"]
    seed = 1000 + 10 * case
    if c["kind"] == "uniform":
        codes = datagen.uniform_codes(n, bits, seed)
    elif c["kind"] == "clustered":
        codes = datagen.clustered_codes(n, bits, seed)
    else:
        pool = datagen.uniform_codes(max(1, min(n, 40)), bits, seed)
        codes = pool[rng.integers(0, pool.shape[0], size=n)]
    queries = datagen.uniform_codes(nq, bits, seed + 1)
    # some exact copies of database codes, some with a few bits flipped
    for i in range(nq):
        r = rng.random()
        if r < 0.3:
            queries[i] = codes[rng.integers(0, n)]
        elif r < 0.5:
            queries[i] = codes[rng.integers(0, n)]
            for _ in range(int(rng.integers(1, 6))):
                b = int(rng.integers(0, bits))
                queries[i, b // 64] ^= np.uint64(1) << np.uint64(b % 64)
    ks = rng.choice([0, 1, 5, 50, n, n + 3, 4096], size=nq)
    ks = np.minimum(ks, 4096).astype(np.uint32)
    return np.ascontiguousarray(codes), np.ascontiguousarray(queries), ks


@pytest.mark.parametrize("case", range(CASES))
def test_random_configuration(mih, case):
    rng = np.random.default_rng([SEED, case])
    c = draw(rng)
    codes, queries, ks = make_data(rng, c, case)
    what = f"case {case}: {c}"
    print(what, flush=True)
    idx = mih.build(to_dev(codes), c["m"], table_mode=c["tmode"], codes_mode=c["cmode"],
                    inline_tables=c["inline_tables"])
    idx.set_tuning(**c["tuning"])
    dq = to_dev(queries)
    ids, dists = idx.knn(dq, ks.tolist())
    oi, od = oracle.knn(codes, queries, ks)
    assert_same(ids, dists, oi, od, what)
    li, ld = mih.linscan_knn(to_dev(codes), dq, ks.tolist())
    assert_same(li, ld, oi, od, what + " (linear scan)")
    r = int(rng.integers(0, c["bits"] // 4 + 1))
    off, rid, rdist = idx.rnn(dq, r)
    off = off.cpu().numpy()
    gi, gd = as_u32(rid), as_u32(rdist)
    for i in range(c["nq"]):
        ri, rd = oracle.rnn(codes, queries[i], r)
        a, b = int(off[i]), int(off[i + 1])
        assert np.array_equal(gi[a:b], ri) and np.array_equal(gd[a:b], rd), f"{what} r={r} query {i}"
    idx.close()
