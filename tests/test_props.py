"""Propositions 1 and 2, the substring partition and the closed forms.

Pins against values the paper prints (tests/golden/paper_numbers.json) and
against brute-force enumeration.
"""
import itertools
import json
import math
import os

import numpy as np
from hypothesis import given, settings, strategies as st

import oracle
from oracle import formulas

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def _subdists(x: int, lens, starts):
    return [bin((x >> s) & ((1 << ln) - 1)).count("1") for ln, s in zip(lens, starts)]


@settings(max_examples=400, deadline=None)
@given(st.integers(min_value=0, max_value=(1 << 128) - 1), st.integers(1, 20), st.integers(0, 128))
def test_proposition_1_and_2(x, m, slack):
    # x is h XOR g; d = popcount(x); any r >= d must satisfy both propositions
    lens, starts = formulas.partition(128, m)
    d = bin(x).count("1")
    r = min(128, d + slack % 5)
    sd = _subdists(x, lens, starts)
    assert sum(sd) == d
    rp, a = divmod(r, m)
    assert any(v <= rp for v in sd)                                      # Prop. 1 (Eq. 2)
    assert any(sd[z] <= rp for z in range(a + 1)) or \
        any(sd[z] <= rp - 1 for z in range(a + 1, m))                    # Prop. 2 (Eq. 3)


def test_step_t_covers_radius_t_by_enumeration():
    # Algorithm 3 step t looks at table t mod m, shell floor(t/m); after steps
    # 0..t every x with popcount <= t has been seen (Proposition 2).  Exhaustive
    # over 12-bit codes for m = 1..5.
    for m in range(1, 6):
        lens, starts = formulas.partition(12, m)
        for x in range(1 << 12):
            sd = _subdists(x, lens, starts)
            first = min(m * sd[j] + j for j in range(m))          # first step that finds x
            assert first <= bin(x).count("1")
            # and no step before `first` finds it
            for t in range(first):
                assert sd[t % m] != t // m


def test_prop1_worked_examples():
    for r, m, rp in GOLDEN["prop1_examples"]["cases"]:
        assert r // m == rp


def test_partition_footnote_and_oracle_partition():
    for bits, m, lens in GOLDEN["subst_lengths_footnote"]["cases"]:
        assert formulas.partition(bits, m)[0] == lens
        assert oracle.partition(bits, m)[0] == lens
        assert max(lens) - min(lens) <= 1 and sum(lens) == bits
    assert oracle.partition(128, 6)[1] == [0, 22, 44, 65, 86, 107]


def test_substring_extraction_straddles_words():
    # bits 44..64 of a 128-bit code: word 0 bits 44..63, then word 1 bit 0
    code = np.array([0xFFF0_0000_0000_0000, 0x1], dtype=np.uint64)
    assert oracle.substring(code, 44, 21) == (0xFFF00 | (1 << 20))
    assert oracle.substring(code, 65, 21) == 0
    rng = np.random.default_rng(0)
    for _ in range(200):
        c = rng.integers(0, 2 ** 63, size=4, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
        big = sum(int(w) << (64 * i) for i, w in enumerate(c))
        s = int(rng.integers(0, 200))
        ln = int(rng.integers(1, 57))
        assert oracle.substring(c, s, ln) == (big >> s) & ((1 << ln) - 1)


def test_ball_sizes_figure1():
    assert formulas.ball(64, 7) == 704_494_193
    about = GOLDEN["ball_64_7"]["about"]
    assert 0.5 * about < formulas.ball(64, 7) < 2 * about
    assert formulas.ball(64, 6) < 1e8          # a 6-bit radius is an order smaller
    assert formulas.ball(10, 10) == 1024
    assert formulas.ball(q=32, r=0) == 1


def test_shell_enumeration_counts():
    for s in range(0, 9):
        for rho in range(0, s + 1):
            masks = [sum(1 << b for b in c) for c in itertools.combinations(range(s), rho)]
            assert len(set(masks)) == formulas.shell(s, rho) == math.comb(s, rho)


def test_lookups_eq5_and_bound_eq4():
    # Eq. 5 equals the direct count m * L(s, floor(s r / q)) and is below its bound
    for q, s, r in [(64, 16, 10), (128, 32, 20), (240, 30, 60), (256, 32, 12)]:
        m = q // s
        assert formulas.lookups(q, s, r) == m * formulas.ball(s, (s * r) // q)
        assert formulas.lookups(q, s, r) <= formulas.lookups_bound(q, s, r) * (1 + 1e-12)
    assert formulas.cost(10 ** 9, 64, 32, 10) == (1 + 10 ** 9 / 2 ** 32) * formulas.lookups(64, 32, 10)


def test_entropy_claims_section_3_2():
    for eps, bound in GOLDEN["radius_growth_h"]["cases"]:
        assert formulas.entropy(eps) < bound


def test_memory_formula_section_6():
    g = GOLDEN["memory_1B"]
    for q, m, gb in g["cases"]:
        gib = formulas.memory_bytes(g["n"], q, m) / 2 ** 30
        assert round(gib) == gb, (q, m, gib)
    e = GOLDEN["empty_sparse_table_bytes"]
    assert 2 ** (e["s"] - 5) * 12 / 2 ** 30 == e["empty_gib"]
    assert 2 ** (e["s"] - 5) * 24 / 2 ** 30 == e["typical_gib"]


def test_table4_heuristic_row():
    t = GOLDEN["table4_q_over_log2n"]
    sel = GOLDEN["table4_selected_m"]
    for q in ("64", "128", "256"):
        for n, v, mm in zip(t["n"], t[q], sel[q]):
            h = formulas.m_heuristic(int(n), int(q))
            assert round(h, 2) == v, (q, n, h)
            assert abs(mm - h) < 2.0
    # Section 6 (number of substrings): the selected m is mostly the nearest integer
    close = sum(abs(mm - formulas.m_heuristic(int(n), int(q))) < 1.0
                for q in ("64", "128", "256") for n, mm in zip(t["n"], sel[q]))
    assert close >= 30
