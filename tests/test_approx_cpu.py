"""Approximate variants of Section 7 in MIH-CPU (Algorithm 3 stopped early),
the reference of the GPU's approximate search.  Pinned two ways: against the
exact oracle when no limit is reached, and against the brute-force
first-encounter reference (``oracle.first_encounter``), which takes the set
of codes met after step T straight from the substring distances
(t_h = min_j (m d_j + j)) and never builds a table.  No GPU."""
import itertools

import numpy as np
import pytest

import datagen
import oracle
from oracle import first_encounter as fe


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


# ------------------------------------------------ the first-encounter reference

def test_partition_matches_the_worked_lengths():
    # Section 2.1 footnote reading: the first (b mod m) substrings one bit longer
    assert fe.partition(64, 3) == ([22, 21, 21], [0, 22, 43])
    assert fe.partition(128, 6) == ([22, 22, 21, 21, 21, 21], [0, 22, 44, 65, 86, 107])
    assert fe.partition(64, 2) == ([32, 32], [0, 32])
    for bits, m in [(64, 3), (128, 5), (256, 8), (192, 7)]:
        assert fe.partition(bits, m) == oracle.partition(bits, m)


def test_first_encounter_step_by_simulating_the_shells():
    # the formula t_h = min_j (m d_j + j) against a literal walk over the
    # shells: step t = m r' + a meets the codes whose substring a equals the
    # query's xor some r'-bit mask (Python integers, every mask enumerated)
    rng = np.random.default_rng(5)
    m = 8                                   # 8-bit substrings of 64-bit codes
    codes = rng.integers(0, 2**63, size=(300, 1), dtype=np.int64).view(np.uint64)
    codes[:40, 0] ^= np.uint64(0x0101010101010101)   # near the query below
    q = codes[7].copy()
    lens, starts = fe.partition(64, m)
    sub = lambda c, j: (int(c) >> starts[j]) & ((1 << lens[j]) - 1)   # noqa: E731
    masks = {r: [x for x in range(256) if bin(x).count("1") == r] for r in range(9)}
    first = {}
    for t in range(m * 9):
        rp, a = divmod(t, m)
        qa = sub(q[0], a)
        keys = {qa ^ x for x in masks[rp]}
        for i in range(len(codes)):
            if i not in first and sub(codes[i, 0], a) in keys:
                first[i] = t
    th, dh = fe.first_steps(codes, q, m)
    assert all(first[i] == th[i] for i in range(len(codes)))
    assert np.array_equal(dh, [bin(int(c) ^ int(q[0])).count("1") for c in codes[:, 0]])
    # Proposition 2: every code within distance T is met by step T
    assert (th <= dh).all()


def test_no_limit_reference_is_the_exact_answer():
    codes = datagen.uniform_codes(20_000, 128, 71)
    queries = datagen.uniform_codes(5, 128, 72)
    for q in queries:
        for m, k in [(4, 1), (5, 17), (8, 100)]:
            ri, rd, steps = fe.early_stop(codes, q, m, k)
            ei, ed = oracle.knn(codes, q[None, :], k)
            assert np.array_equal(ri, ei) and np.array_equal(rd, ed)
            assert steps == int(ed[-1]) + 1          # Algorithm 3 stops after step d_k


CASES = [
    # (kind, bits, n, m, seed, queries); exact MIH-CPU searches of clustered
    # 128-bit codes take ~0.4 s each, hence fewer queries there
    ("uniform", 64, 60_000, 4, 93, 8),
    ("uniform", 64, 40_000, 3, 81, 8),
    ("clustered", 128, 30_000, 5, 0, 3),
]


def _case_data(kind, bits, n, m, seed, nq):
    if kind == "uniform":
        return datagen.uniform_codes(n, bits, seed), datagen.uniform_codes(nq, bits, seed + 1)
    return datagen.db_codes(kind, n, bits), datagen.query_codes(kind, nq, bits)


@pytest.fixture(scope="module", params=CASES, ids=lambda c: f"{c[0]}-{c[1]}-m{c[3]}")
def case(request):
    codes, queries = _case_data(*request.param)
    m = request.param[3]
    ix = oracle.MihCpu(codes, m)
    yield codes, queries, m, ix
    ix.close()


def _limits(ed):
    dk = int(ed[-1])
    radii = [None, 0, 1, max(dk - 3, 0), max(dk - 2, 0), max(dk - 1, 0), dk, dk + 2]
    budgets = [0, 1, 2, 7, 40, 300, 5000]
    return radii, budgets


def test_mihcpu_early_stops_equal_the_first_encounter_reference(case):
    """Element by element, and in the number of steps run, for the radius
    rule, the budget rule and both together."""
    codes, queries, m, ix = case
    bits = 64 * codes.shape[1]
    for q in queries:
        sd = fe.first_steps(codes, q, m)
        for k in (1, 10, 50):
            _, ed = oracle.knn(codes, q[None, :], k)
            radii, budgets = _limits(ed)
            for R, B in itertools.product(radii, budgets):
                ai, ad, st = ix.knn_approx(q, k, max_step=R, max_found=B, stats=True)
                ri, rd, steps = fe.early_stop(codes, q, m, k, max_step=R, max_found=B,
                                              guard=fe.mihcpu_guard(bits, m), steps_and_dists=sd)
                what = f"k={k} R={R} budget={B}"
                assert np.array_equal(ai, ri) and np.array_equal(ad, rd), what
                assert st["radius"] == steps, what


def test_the_pins_tell_apart_the_plausible_mistakes():
    """The comparison above (answer and step count) would catch the two
    mistakes that the looser pins let through: a radius stop one step late,
    and a budget that counts duplicate encounters (a code met in several
    tables) as distinct codes.  For each, some case of the grid gives a
    different answer or a different number of steps."""
    late_differs = dup_differs = 0
    for c in CASES:
        codes, queries = _case_data(*c)
        m = c[3]
        for q, k in itertools.product(queries, (10, 50)):
            _, ed = oracle.knn(codes, q[None, :], k)
            radii, budgets = _limits(ed)
            th, dh = fe.first_steps(codes, q, m)
            dj = fe.substring_distances(codes, q, m)
            enc = np.sort((m * dj + np.arange(m)[:, None]).ravel())   # every encounter
            dk = int(np.partition(dh, k - 1)[k - 1])
            for R in radii:
                if R is None:
                    continue
                a = fe.early_stop(codes, q, m, k, max_step=R, steps_and_dists=(th, dh))
                b = fe.early_stop(codes, q, m, k, max_step=R + 1, steps_and_dists=(th, dh))
                late_differs += not np.array_equal(a[0], b[0]) or a[2] != b[2]
            for B in budgets:
                if B == 0 or B > len(enc):
                    continue
                a = fe.early_stop(codes, q, m, k, max_found=B, steps_and_dists=(th, dh))
                # stop at the first step whose encounters, duplicates
                # included, reach the budget
                last = min(int(enc[B - 1]), dk)
                met = np.nonzero(th <= last)[0]
                wrong = met[np.lexsort((met, dh[met]))[:k]]
                dup_differs += (a[2] != last + 1 or len(wrong) != int((a[0] != fe.SENTINEL).sum())
                                or not np.array_equal(a[0][:len(wrong)], wrong))
    assert late_differs > 0 and dup_differs > 0, (late_differs, dup_differs)
