"""Approximate kNN (Section 7) on the GPU against MIH-CPU stopped by the same
rule (its k best codes met), bit-exact; against the brute-force
first-encounter reference (the codes met after step T are those with
min_j (m d_j + j) <= T), answers and step counts; and against the exact
oracle when no limit is reached."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import as_u32, assert_same, to_dev
from oracle import first_encounter as fe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mih():
    import paper_1307_2982_amd as m
    m.load()
    return m


def reference(ix_cpu, queries, k, max_step, max_found):
    ids, dists = [], []
    for q in queries:
        i, d = ix_cpu.knn_approx(q, k, max_step=max_step, max_found=max_found)
        ids.append(i)
        dists.append(d)
    return np.concatenate(ids), np.concatenate(dists)


@pytest.mark.parametrize("bits,m,kind,tmode", [(64, 4, "uniform", "direct"), (64, 3, "uniform", "grouped"),
                                               (128, 6, "clustered", "sorted")])
def test_approx_equals_early_stopped_algorithm3(mih, bits, m, kind, tmode):
    n, nq, k = 80_000, 24, 40
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits)
    ix_cpu = oracle.MihCpu(codes, m)
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode="inline")
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, k)
    dk = od.reshape(nq, k)[:, -1]
    for max_radius, budget in [(int(np.median(dk)) - 2, 0), (int(np.median(dk)), 0), (None, 30),
                               (None, 2000), (int(np.median(dk)) - 1, 500)]:
        ids, dists = idx.knn_approx(dq, k, max_radius=max_radius, max_candidates=budget)
        ri, rd = reference(ix_cpu, queries, k, max_radius, budget)
        assert_same(ids, dists, ri, rd, f"{bits}/{m}/{tmode} radius={max_radius} budget={budget}")
    # no limit reached: the exact answer
    ids, dists = idx.knn_approx(dq, k, max_radius=bits, max_candidates=n + 1)
    assert_same(ids, dists, oi, od, "unlimited")
    ix_cpu.close()


def first_encounter_reference(codes, queries, m, k, max_step, max_found):
    bits = 64 * codes.shape[1]
    ids, dists, steps = [], [], 0
    for q in queries:
        i, d, s = fe.early_stop(codes, q, m, k, max_step=max_step, max_found=max_found,
                                guard=fe.device_guard(bits, m))
        ids.append(i)
        dists.append(d)
        steps += s
    return np.concatenate(ids), np.concatenate(dists), steps


@pytest.mark.parametrize("bits,m,kind,tmode", [(64, 4, "uniform", "heads"), (64, 3, "uniform", "direct"),
                                               (128, 6, "clustered", "sorted")])
def test_approx_equals_first_encounter_reference(mih, bits, m, kind, tmode):
    n, nq, k = 60_000, 16, 25
    codes = datagen.db_codes(kind, n, bits)
    queries = datagen.query_codes(kind, nq, bits, first_row=100)
    idx = mih.build(to_dev(codes), m, table_mode=tmode, codes_mode="inline")
    dq = to_dev(queries)
    _, od = oracle.knn(codes, queries, k)
    dk = int(np.median(od.reshape(nq, k)[:, -1]))
    for max_radius, budget in [(dk - 3, 0), (dk - 1, 0), (dk, 0), (None, 1), (None, 17), (None, 900),
                               (dk - 1, 60), (dk + 4, 0)]:
        ids, dists, st = idx.knn_approx(dq, k, max_radius=max_radius, max_candidates=budget, stats=True)
        ri, rd, steps = first_encounter_reference(codes, queries, m, k, max_radius, budget)
        what = f"{bits}/{m}/{tmode} radius={max_radius} budget={budget}"
        assert_same(ids, dists, ri, rd, what)
        assert st["steps"] == steps, what


def test_approx_then_exact_share_the_engine(mih):
    codes = datagen.uniform_codes(50_000, 64, 95)
    queries = datagen.uniform_codes(16, 64, 96)
    idx = mih.build(to_dev(codes), 4)
    dq = to_dev(queries)
    oi, od = oracle.knn(codes, queries, 10)
    for _ in range(2):
        idx.knn_approx(dq, 10, max_candidates=50)
        ids, dists = idx.knn(dq, 10)
        assert np.array_equal(as_u32(ids), oi) and np.array_equal(as_u32(dists), od)
