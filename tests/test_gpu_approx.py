"""Approximate kNN (Section 7) on the GPU against MIH-CPU stopped by the same
rule (its k best codes met), bit-exact, and against the exact oracle when no
limit is reached."""
import numpy as np
import pytest

import datagen
import oracle
from gpu_util import as_u32, assert_same, to_dev

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
