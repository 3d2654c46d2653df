"""Approximate variants of Section 7 in MIH-CPU (Algorithm 3 stopped early),
the reference of the GPU's approximate search, checked against the exact
oracle.  No GPU."""
import numpy as np
import pytest

import datagen
import oracle


@pytest.fixture(scope="module")
def data():
    oracle.build(force=False)
    codes = datagen.uniform_codes(60_000, 64, 93)
    queries = datagen.uniform_codes(12, 64, 94)
    return codes, queries, oracle.MihCpu(codes, 4)


def test_no_limit_is_exact(data):
    codes, queries, ix = data
    for q in queries:
        ei, ed = oracle.knn(codes, q[None, :], 20)
        ai, ad = ix.knn_approx(q, 20, max_step=64, max_found=10**9)
        assert np.array_equal(ai, ei) and np.array_equal(ad, ed)


def test_radius_limit_keeps_every_code_within_the_radius(data):
    # after the step covering radius R every code within R has been met
    # (Proposition 2): the answer starts with exactly the codes of the exact
    # answer within R, and continues with codes farther than R
    codes, queries, ix = data
    k = 50
    for q in queries:
        ei, ed = oracle.knn(codes, q[None, :], k)
        for R in (int(ed[-1]) - 3, int(ed[-1]) - 1, int(ed[-1])):
            ai, ad = ix.knn_approx(q, k, max_step=R)
            c = int((ed <= R).sum())
            assert np.array_equal(ai[:c], ei[:c]) and np.array_equal(ad[:c], ed[:c])
            valid = ai != oracle.SENTINEL
            assert (ad[c:][valid[c:]] > R).all()
            if R >= ed[-1]:
                assert np.array_equal(ai, ei)


def test_candidate_limit_gives_true_distances_in_order(data):
    codes, queries, ix = data
    k = 30
    for q in queries[:6]:
        for budget in (1, 40, 500):
            ai, ad = ix.knn_approx(q, k, max_found=budget)
            valid = ai != oracle.SENTINEL
            d = oracle.distances(codes, q)
            assert np.array_equal(d[ai[valid]], ad[valid])
            pairs = list(zip(ad[valid].tolist(), ai[valid].tolist()))
            assert pairs == sorted(pairs) and len(set(ai[valid].tolist())) == int(valid.sum())
