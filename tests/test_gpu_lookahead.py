"""Running queries ahead by several steps per round (lookahead) changes
neither exact kNN nor r-neighbour results, and small batches then finish in
fewer rounds (device rounds: the one-launch path for small batches is off).  Every result is checked against the oracle's plain linear
scan, bit for bit."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


@pytest.mark.parametrize("bits,m,kind,tmode,cmode", [(64, 3, "uniform", "direct", "inline"),
                                                     (64, 2, "uniform", "direct", "indirect"),
                                                     (128, 6, "clustered", "sorted", "inline"),
                                                     (64, 3, "uniform", "heads", "inline")])
def test_lookahead_exact_knn(mih, bits, m, kind, tmode, cmode):
    n, nq = 120_007, 40
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode=cmode)
    dq = to_dev(queries)
    # per-query k, with the largest k and k = 0 among them
    rng = np.random.default_rng(7)
    ks = rng.choice([1, 10, 100, 1000], size=nq).astype(np.uint32)
    ks[5] = 4096
    ks[6] = 0
    oi, od = oracle.knn(codes, queries, ks)
    runs = {}
    for look in (1, 2, 5, 16, 32):
        idx.set_tuning(lookahead=look, small_batch=0)
        ids, dists, st = idx.knn(dq, ks.tolist(), stats=True)
        assert_same(ids, dists, oi, od, f"{bits}/{m}/{tmode}/{cmode} look={look}")
        runs[look] = st
    # one step per round enumerates exactly the shells of steps 0..d_k (Eq. 1);
    # running ahead can only add steps, never skip one
    assert runs[1]["probes"] <= runs[16]["probes"]
    assert runs[16]["rounds"] <= runs[1]["rounds"]
    idx.close()


def test_lookahead_k_beyond_n(mih):
    # k > n: every step up to the last one runs, several per round
    n, nq, m, k = 3001, 8, 4, 4096
    codes = datagen.uniform_codes(n, 64, 408)
    queries = datagen.uniform_codes(nq, 64, 409)
    idx = mih.build(to_dev(codes), m)
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, k)
    for look in (1, 16, 32):
        idx.set_tuning(lookahead=look, small_batch=0)
        ids, dists = idx.knn(dq, k)
        assert_same(ids, dists, oi, od, f"k > n look={look}")
    idx.close()


def test_lookahead_cuts_rounds_of_a_small_batch(mih):
    # 20 queries over 200K codes, m = 3: a round of one step per query
    # leaves most waves idle, so the rounds run several steps ahead
    n, nq, m, k = 200_003, 20, 3, 100
    codes = datagen.uniform_codes(n, 64, 401)
    queries = datagen.uniform_codes(nq, 64, 402)
    idx = mih.build(to_dev(codes), m)
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, k)
    idx.set_tuning(lookahead=1, small_batch=0)
    _, _, st1 = idx.knn(dq, k, stats=True)
    idx.set_tuning(lookahead=16, small_batch=0)
    ids, dists, st16 = idx.knn(dq, k, stats=True)
    assert_same(ids, dists, oi, od, "look=16")
    assert st16["rounds"] < st1["rounds"], (st1, st16)
    idx.close()


def test_lookahead_rnn(mih):
    n, nq, r = 150_001, 16, 13
    codes = datagen.uniform_codes(n, 64, 403)
    queries = datagen.uniform_codes(nq, 64, 404)
    idx = mih.build(to_dev(codes), 3)
    dq = to_dev(queries)
    idx.set_tuning(lookahead=16, small_batch=0)
    off, ids, dists = idx.rnn(dq, r)
    for i in range(nq):
        ri, rd = oracle.rnn(codes, queries[i], r)
        a, b = int(off[i]), int(off[i + 1])
        assert np.array_equal(ids[a:b].cpu().numpy().view(np.uint32), ri), i
        assert np.array_equal(dists[a:b].cpu().numpy().view(np.uint32), rd), i
    idx.close()


def test_lookahead_leaves_approximate_search_alone(mih):
    # an approximate query's result depends on the steps it ran: the engine
    # runs it one step per round whatever the tuning says
    n, nq, m, k = 60_000, 12, 4, 20
    codes = datagen.uniform_codes(n, 64, 405)
    queries = datagen.uniform_codes(nq, 64, 406)
    idx = mih.build(to_dev(codes), m)
    dq = to_dev(queries)
    out = {}
    for look in (1, 16):
        idx.set_tuning(lookahead=look, small_batch=0)
        out[look] = idx.knn_approx(dq, k, max_radius=6, stats=True)
    assert np.array_equal(out[1][0].cpu().numpy(), out[16][0].cpu().numpy())
    assert np.array_equal(out[1][1].cpu().numpy(), out[16][1].cpu().numpy())
    assert out[1][2]["probes"] == out[16][2]["probes"]
    idx.close()


def test_lookahead_tuning_is_validated(mih):
    codes = datagen.uniform_codes(1000, 64, 407)
    idx = mih.build(to_dev(codes), 2)
    for bad in (0, 33):
        with pytest.raises(mih.MihError):
            idx.set_tuning(lookahead=bad, small_batch=0)
    assert idx.get_tuning()["lookahead"] == 16
    idx.set_tuning(lookahead=32, small_batch=0)
    assert idx.get_tuning()["lookahead"] == 32
    idx.close()
