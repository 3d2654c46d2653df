"""GPU r-neighbour search (mih_rnn and linscan_rnn through the C ABI) against
the CPU oracle's r-neighbour definition, bit-exact: every code within
distance r, in ascending (distance, id) order, for every query."""
import numpy as np
import pytest

import datagen
import oracle
from oracle import formulas
from gpu_util import as_u32, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def oracle_rnn_all(codes, queries, radii):
    ids, dists, offs = [], [], [0]
    for q, r in zip(queries, radii):
        i, d = oracle.rnn(codes, q, int(r))
        ids.append(i)
        dists.append(d)
        offs.append(offs[-1] + len(i))
    cat = (lambda xs: np.concatenate(xs) if xs else np.zeros(0, np.uint32))
    return np.array(offs, dtype=np.int64), cat(ids), cat(dists)


def assert_rnn_same(got, expect, what):
    go, gi, gd = got
    eo, ei, ed = expect
    go = go.cpu().numpy()
    assert np.array_equal(go, eo), f"{what}: offsets differ (totals {go[-1]} vs {eo[-1]})"
    gi, gd = as_u32(gi), as_u32(gd)
    if not (np.array_equal(gi, ei) and np.array_equal(gd, ed)):
        bad = np.nonzero((gi != ei) | (gd != ed))[0]
        q = int(np.searchsorted(eo, bad[0], side="right") - 1)
        raise AssertionError(f"{what}: {len(bad)} entries differ, first in query {q}")


def planted(query: np.ndarray, count: int, max_flips: int, seed: int) -> np.ndarray:
    """`count` codes within max_flips bits of `query` (seeded bit positions)."""
    W = query.shape[0]
    pos = datagen.choice_u32(count * max_flips, list(range(64 * W)), seed).reshape(count, max_flips)
    out = np.repeat(query[None, :], count, axis=0).copy()
    for f in range(max_flips):
        w, b = pos[:, f] // 64, pos[:, f] % 64
        out[np.arange(count), w] ^= (np.uint64(1) << b.astype(np.uint64))
    return out


@pytest.mark.parametrize("tmode,cmode", [("direct", "inline"), ("sorted", "indirect"), ("heads", "inline")])
def test_mih_rnn_uniform_radii(mih, tmode, cmode):
    n, nq = 200_003, 24
    codes = datagen.uniform_codes(n, 64, 61)
    queries = datagen.uniform_codes(nq, 64, 62)
    queries[3] = codes[17]          # an exact match (r = 0 finds it)
    idx = mih.build(to_dev(codes), 3, table_mode=tmode, codes_mode=cmode)
    dq = to_dev(queries)
    lens, _ = formulas.partition(64, 3)
    for r in [0, 3, 9, 14, 17]:
        for look in (1, 16):
            idx.set_tuning(lookahead=look)
            off, ids, dists, st = idx.rnn(dq, r, stats=True)
            assert_rnn_same((off, ids, dists), oracle_rnn_all(codes, queries, [r] * nq),
                            f"{tmode}/{cmode} r={r} look={look}")
            # one step per round: steps 0..r and nothing more, C(s_a, r')
            # buckets per step (Eq. 1); running ahead may take more
            shells = nq * sum(formulas.shell(lens[t % 3], t // 3) for t in range(r + 1))
            if look == 1:
                assert st["steps"] == nq * (r + 1)
                assert st["probes"] == shells
            else:
                assert st["steps"] >= nq * (r + 1) and st["probes"] >= shells
    idx.close()


def test_mih_rnn_long_lists_and_reruns(mih):
    # thousands of planted neighbours per query: the first buffer overflows
    # (exact re-run) and lists longer than one workgroup's sort take the
    # radix-sort path
    base = datagen.uniform_codes(50_000, 64, 63)
    queries = datagen.uniform_codes(3, 64, 64)
    parts = [base, planted(queries[0], 9000, 4, 65), planted(queries[1], 1500, 3, 66)]
    codes = np.concatenate(parts)
    perm = np.argsort(datagen.uniform_f64(codes.shape[0], 67), kind="stable")
    codes = np.ascontiguousarray(codes[perm])
    idx = mih.build(to_dev(codes), 4)
    radii = [4, 3, 12]
    off, ids, dists, st = idx.rnn(to_dev(queries), radii, stats=True)
    got = (off, ids, dists)
    expect = oracle_rnn_all(codes, queries, radii)
    assert expect[0][1] > 4096
    assert_rnn_same(got, expect, "planted")
    assert st["reruns"] >= 1


def test_mih_rnn_per_query_radius_and_whole_database(mih):
    codes = datagen.uniform_codes(5000, 128, 68)
    queries = datagen.uniform_codes(6, 128, 69)
    radii = [0, 200, 40, 128, 35, 1]     # 200 and 128 return every code
    idx = mih.build(to_dev(codes), 6)
    got = idx.rnn(to_dev(queries), radii)
    expect = oracle_rnn_all(codes, queries, [min(r, 128) for r in radii])
    assert expect[0][2] - expect[0][1] == 5000
    assert_rnn_same(got, expect, "per-query r")


def test_mih_rnn_clustered_256_equals_linscan(mih):
    n, nq = 80_000, 40
    codes = datagen.clustered_codes(n, 256, datagen.SEED_DB_CLUSTERED)
    queries = datagen.clustered_codes(nq, 256, datagen.SEED_Q_CLUSTERED)
    dc, dq = to_dev(codes), to_dev(queries)
    idx = mih.build(dc, 8, table_mode="sorted")
    for r in [20, 40]:
        got = idx.rnn(dq, r)
        lin = mih.linscan_rnn(dc, dq, r)
        for a, b in zip(got, lin):
            assert bool((a == b).all()), f"MIH vs linscan r={r}"
        sel = list(range(0, nq, 8))
        expect = oracle_rnn_all(codes, queries[sel], [r] * len(sel))
        off = got[0].cpu().numpy()
        gi = np.concatenate([as_u32(got[1])[off[i]:off[i + 1]] for i in sel])
        gd = np.concatenate([as_u32(got[2])[off[i]:off[i + 1]] for i in sel])
        assert np.array_equal(gi, expect[1]) and np.array_equal(gd, expect[2])


def test_linscan_rnn_matches_oracle(mih):
    codes = datagen.uniform_codes(100_000, 64, 70)
    queries = datagen.uniform_codes(33, 64, 71)
    queries[5] = codes[99_999]
    dc, dq = to_dev(codes), to_dev(queries)
    for r in [0, 10, 15]:
        got = mih.linscan_rnn(dc, dq, r)
        assert_rnn_same(got, oracle_rnn_all(codes, queries, [r] * 33), f"linscan r={r}")
    # planted long lists through the linear scan's re-run and radix paths
    q2 = datagen.uniform_codes(2, 64, 72)
    c2 = np.concatenate([codes, planted(q2[0], 6000, 3, 73)])
    got = mih.linscan_rnn(to_dev(c2), to_dev(q2), [3, 8])
    assert_rnn_same(got, oracle_rnn_all(c2, q2, [3, 8]), "linscan planted")


def test_rnn_empty_inputs(mih):
    import torch
    codes = datagen.uniform_codes(1000, 64, 74)
    idx = mih.build(to_dev(codes), 4)
    empty = torch.empty((0, 1), dtype=torch.int64, device="cuda")
    off, ids, dists = idx.rnn(empty, 5)
    assert off.tolist() == [0] and ids.numel() == 0
    off, ids, dists = mih.linscan_rnn(to_dev(codes), empty, 5)
    assert off.tolist() == [0] and ids.numel() == 0
    q = to_dev(datagen.uniform_codes(3, 64, 75))
    off, ids, dists = mih.linscan_rnn(empty, q, 64)
    assert off.tolist() == [0, 0, 0, 0]


def test_knn_and_rnn_share_the_engine(mih):
    # alternating calls reuse the index's engine; every answer stays exact
    codes = datagen.uniform_codes(120_000, 64, 76)
    queries = datagen.uniform_codes(20, 64, 77)
    idx = mih.build(to_dev(codes), 3)
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, 25)
    expect = oracle_rnn_all(codes, queries, [12] * 20)
    for _ in range(2):
        ids, dists = idx.knn(dq, 25)
        assert np.array_equal(as_u32(ids), oi) and np.array_equal(as_u32(dists), od)
        assert_rnn_same(idx.rnn(dq, 12), expect, "rnn after knn")
