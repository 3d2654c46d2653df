"""Serving loop (mih_server_* through the C ABI): each request's result is the
same alone and in a mix of overlapping requests (tolerance 0), and equals
mih_knn's and the oracle's; rounds replayed as a hipGraph equal eager
launches, call after call."""
import numpy as np
import pytest
import torch

import datagen
import oracle
from gpu_util import as_u32, assert_same, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def setup(mih):
    n = 300_000
    codes = datagen.uniform_codes(n, 64, 71)
    pool = datagen.uniform_codes(8000, 64, 72)
    idx = mih.build(to_dev(codes), 3)
    rng = np.random.default_rng(5)
    reqs, off = [], 0
    for _ in range(40):
        size = int(rng.integers(1, 160))
        ks = rng.choice([0, 1, 10, 100, 1000], size=size, p=[0.05, 0.25, 0.25, 0.25, 0.2]).tolist()
        reqs.append((off, size, ks))
        off += size
    assert off <= len(pool)
    return codes, pool, idx, reqs


def _alone(mih, idx, q, ks):
    srv = mih.Server(idx, max_queries=64, buffer_entries=0)
    t = srv.submit(q, ks)
    srv.drain()
    return srv.result(t)


def test_server_alone_equals_mix_equals_batch(mih, setup):
    codes, pool, idx, reqs = setup
    dpool = to_dev(pool)
    alone = []
    for off, size, ks in reqs:
        alone.append(_alone(mih, idx, dpool[off:off + size], ks))
    # the mix: few slots and a small buffer pool, so admission is limited by
    # slots and buffer memory and requests overlap on the device
    srv = mih.Server(idx, max_queries=96, buffer_entries=96 * 3000)
    tickets = []
    for i, (off, size, ks) in enumerate(reqs):
        tickets.append(srv.submit(dpool[off:off + size], ks))
        if i % 3 == 2:
            srv.step()          # requests arrive while others are in flight
    srv.drain()
    st = srv.stats()
    assert st["completed_requests"] == len(reqs) and st["in_flight"] == 0
    for (off, size, ks), t, (ai, ad) in zip(reqs, tickets, alone):
        mi, md = srv.result(t)
        assert torch.equal(mi, ai) and torch.equal(md, ad)
        bi, bd = idx.knn(dpool[off:off + size], ks)
        assert torch.equal(bi, ai) and torch.equal(bd, ad)
    # oracle on a few requests
    for j in (0, 7, 19):
        off, size, ks = reqs[j]
        oi, od = oracle.knn(codes, pool[off:off + size], np.array(ks, dtype=np.uint32))
        assert_same(alone[j][0], alone[j][1], oi, od, f"request {j}")


def test_server_graph_equals_eager_over_replays(mih, setup):
    codes, pool, idx, reqs = setup
    dpool = to_dev(pool)
    eager = mih.Server(idx, max_queries=128, use_graph=False)
    graph = mih.Server(idx, max_queries=128, use_graph=True)
    for rep in range(3):
        off, size, ks = reqs[rep * 5]
        te = eager.submit(dpool[off:off + size], ks)
        eager.drain()
        torch.cuda.synchronize()
        tg = graph.submit(dpool[off:off + size], ks)
        graph.drain()
        ei, ed = eager.result(te)
        gi, gd = graph.result(tg)
        assert torch.equal(ei, gi) and torch.equal(ed, gd), rep


def test_server_rejects_requests_that_cannot_fit(mih, setup):
    codes, pool, idx, reqs = setup
    srv = mih.Server(idx, max_queries=4, buffer_entries=4096)
    with pytest.raises(mih.MihError) as e:
        srv.submit(to_dev(pool[:2]), 1000)        # needs 8000 entries
    assert e.value.status == 5
    t = srv.submit(to_dev(pool[:9]), 10)          # fits, 4 at a time
    srv.drain()
    ids, dists = srv.result(t)
    oi, od = oracle.knn(codes, pool[:9], 10)
    assert_same(ids, dists, oi, od, "small server")


def test_server_overflow_rerun_in_mix(mih):
    base = datagen.uniform_codes(3, 64, 81)
    codes = np.concatenate([np.repeat(base[:1], 6000, axis=0), datagen.uniform_codes(4000, 64, 82)])
    idx = mih.build(to_dev(codes), 3)
    q = np.concatenate([base[:1], datagen.uniform_codes(5, 64, 83)])
    srv = mih.Server(idx, max_queries=8)
    tickets = [srv.submit(to_dev(q), 100), srv.submit(to_dev(q[:1]), 7)]
    srv.drain()
    assert srv.stats()["reruns"] >= 1
    for t, (qq, k) in zip(tickets, [(q, 100), (q[:1], 7)]):
        ids, dists = srv.result(t)
        oi, od = oracle.knn(codes, qq, k)
        assert_same(ids, dists, oi, od, "overflow in server")


def test_work_quantum_keeps_every_result(mih, setup):
    # rounds that probe at most round_masks shell masks per query (a larger
    # step continues over the following rounds from its saved position):
    # batch and serving results are unchanged, the rounds more numerous
    codes, pool, idx, reqs = setup
    dpool = to_dev(pool)
    base = idx.get_tuning()
    ks = [k for _, _, kk in reqs for k in kk]
    nq = len(ks)
    idx.set_tuning(small_batch=0, round_masks=0)
    ref_i, ref_d, ref_st = idx.knn(dpool[:nq], ks, stats=True)
    oi, od = oracle.knn(codes, pool[:nq], np.array(ks, dtype=np.uint32))
    assert_same(ref_i, ref_d, oi, od, "no quantum")
    for J, chunk, rm, look in [(4, 256, 256, 1), (4, 256, 1000, 16), (8, 512, 5000, 16), (4, 1024, 1, 1)]:
        idx.set_tuning(probes_per_lane=J, chunk=chunk, round_masks=rm, lookahead=look, small_batch=0)
        ids, dists, st = idx.knn(dpool[:nq], ks, stats=True)
        what = f"quantum {rm} chunk {chunk} look {look}"
        assert torch.equal(ids, ref_i) and torch.equal(dists, ref_d), what
        assert st["rounds"] > ref_st["rounds"], what
    # with sweeps: steps within one quantum may run partition by partition
    for occ, rm in [(1, 2000), (0, 2000), (1, 1 << 20)]:
        idx.set_tuning(probes_per_lane=4, chunk=256, round_masks=rm, lookahead=16, small_batch=0,
                       occupancy_filter=occ, sweep_shift=5, sweep_bits=16, sweep_queries=64)
        ids, dists = idx.knn(dpool[:nq], ks)
        what = f"quantum {rm} with sweeps, occupancy filter {occ}"
        assert torch.equal(ids, ref_i) and torch.equal(dists, ref_d), what
    idx.set_tuning(occupancy_filter=base["occupancy_filter"], sweep_shift=base["sweep_shift"],
                   sweep_bits=base["sweep_bits"], sweep_queries=base["sweep_queries"])
    # serving with a quantum: every request as alone without one
    idx.set_tuning(probes_per_lane=4, chunk=256, round_masks=512, lookahead=16)
    srv = mih.Server(idx, max_queries=96, buffer_entries=96 * 3000)
    tickets = []
    for i, (off, size, kk) in enumerate(reqs[:20]):
        tickets.append(srv.submit(dpool[off:off + size], kk))
        if i % 2 == 1:
            srv.step()
    srv.drain()
    koff = np.concatenate([[0], np.cumsum(ks)])   # row offset of each query of the batch
    for (off, size, kk), t in zip(reqs[:20], tickets):
        mi, md = srv.result(t)
        a, b = int(koff[off]), int(koff[off + size])
        assert torch.equal(mi.reshape(-1), ref_i[a:b]) and torch.equal(md.reshape(-1), ref_d[a:b])
    srv.close()
    idx.set_tuning(**base)
