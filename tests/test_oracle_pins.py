"""Pins for the CPU oracle, none of which re-types its recurrence.

Every check here compares the oracle with something the paper or the mathematics
fixes independently: exhaustive enumeration of alignments, hand-worked scores,
closed forms and invariants.  A dropped term, a sign or index slip, a transposed
substitution matrix or the other gap convention each fails at least one test.
"""
from __future__ import annotations

import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st, HealthCheck

import oracle
from paper_1702_07195_amd import synth
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gap_convention.txt")

HYP = settings(max_examples=150, deadline=None,
               suppress_health_check=[HealthCheck.too_slow, HealthCheck.data_too_large])


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            q, d, s = line.split()
            rows.append((q.strip('"'), d.strip('"'), int(s)))
    return rows


ABC = {"a": 0, "b": 1, "c": 2}
ABC_SM = np.full((3, 3), -10, dtype=np.int32)
np.fill_diagonal(ABC_SM, 5)


def _codes(s):
    return np.array([ABC[c] for c in s], dtype=np.uint8)


@pytest.mark.parametrize("q,d,expected", _golden_rows())
def test_hand_worked_gap_convention(q, d, expected):
    assert oracle.score(_codes(q), _codes(d), ABC_SM, 3, 1) == expected
    # the same value by exhaustive enumeration, so the fixture itself is checked
    assert brute.enumerate_best(_codes(q), _codes(d), ABC_SM, 3, 1) == expected


@st.composite
def tiny_case(draw, max_len=5):
    alpha = draw(st.integers(2, 5))
    q = draw(st.lists(st.integers(0, alpha - 1), min_size=0, max_size=max_len))
    d = draw(st.lists(st.integers(0, alpha - 1), min_size=0, max_size=max_len))
    sm = draw(st.lists(st.integers(-10, 10), min_size=alpha * alpha, max_size=alpha * alpha))
    go = draw(st.integers(0, 12))
    ge = draw(st.integers(0, 12))
    return (np.array(q, dtype=np.uint8), np.array(d, dtype=np.uint8),
            np.array(sm, dtype=np.int32).reshape(alpha, alpha), go, ge)


@HYP
@given(tiny_case())
def test_brute_force_enumeration(case):
    q, d, sm, go, ge = case
    assert oracle.score(q, d, sm, go, ge) == brute.enumerate_best(q, d, sm, go, ge)


def test_brute_force_longer_fixed_cases():
    rng = np.random.Generator(np.random.PCG64(17020))
    for _ in range(12):
        alpha = int(rng.integers(2, 4))
        q = rng.integers(0, alpha, size=int(rng.integers(5, 7))).astype(np.uint8)
        d = rng.integers(0, alpha, size=int(rng.integers(5, 7))).astype(np.uint8)
        sm = synth.random_matrix(rng, alpha, -6, 8)
        go, ge = int(rng.integers(0, 6)), int(rng.integers(0, 4))
        assert oracle.score(q, d, sm, go, ge) == brute.enumerate_best(q, d, sm, go, ge)


def test_matrix_orientation_query_selects_row():
    # SM(x, y) with x from the query: an asymmetric matrix where only (q=a, d=b) pays
    sm = np.array([[-5, 7], [-5, -5]], dtype=np.int32)
    assert oracle.score(np.array([0], np.uint8), np.array([1], np.uint8), sm, 1, 1) == 7
    assert oracle.score(np.array([1], np.uint8), np.array([0], np.uint8), sm, 1, 1) == 0


@HYP
@given(tiny_case(max_len=12))
def test_border_reading_zero_equals_minus_infinity(case):
    # Section 2 sets E and F to 0 on row 0 / column 0; the textbook border is -inf.
    q, d, sm, go, ge = case
    assert oracle.score(q, d, sm, go, ge) == \
        oracle.score(q, d, sm, go, ge, ef_border=oracle.NEG_BORDER)


@HYP
@given(tiny_case(max_len=10))
def test_linear_gap_special_case(case):
    q, d, sm, _, ge = case
    assert oracle.score(q, d, sm, 0, ge) == brute.linear_gap_sw(q, d, sm, ge)


@HYP
@given(tiny_case(max_len=12))
def test_ungapped_limit_is_kadane(case):
    q, d, sm, _, _ = case
    cap = min(len(q), len(d)) * max(int(sm.max()), 0)
    assert oracle.score(q, d, sm, cap, 0) == brute.kadane_diagonals(q, d, sm)
    assert oracle.score(q, d, sm, 0, cap) == brute.kadane_diagonals(q, d, sm)


@HYP
@given(st.integers(2, 4), st.data())
def test_identity_scoring_gives_longest_common_substring(alpha, data):
    a = np.array(data.draw(st.lists(st.integers(0, alpha - 1), max_size=14)), np.uint8)
    b = np.array(data.draw(st.lists(st.integers(0, alpha - 1), max_size=14)), np.uint8)
    big = len(a) + len(b) + 1
    sm = np.full((alpha, alpha), -big, dtype=np.int32)
    np.fill_diagonal(sm, 1)
    assert oracle.score(a, b, sm, big, 0) == brute.longest_common_substring(a, b)


def test_single_residue_query_closed_form():
    rng = np.random.Generator(np.random.PCG64(17021))
    sm = synth.BLOSUM62
    for _ in range(50):
        q = synth.residues(rng, 1)
        d = synth.residues(rng, int(rng.integers(0, 40)))
        want = max([0] + [int(sm[q[0], x]) for x in d])
        assert oracle.score(q, d, sm, 10, 2) == want


@pytest.mark.parametrize("n,k", [(1, 1), (7, 3), (50, 50), (120, 37)])
def test_homopolymer_closed_form(n, k):
    sm = synth.BLOSUM62
    a = synth.CODE["W"]  # SM(W, W) = 11
    s = int(sm[a, a])
    assert oracle.score(np.full(k, a, np.uint8), np.full(n, a, np.uint8), sm, 10, 2) == k * s
    assert oracle.score(np.full(n, a, np.uint8), np.full(k, a, np.uint8), sm, 10, 2) == k * s


@pytest.mark.parametrize("n,expected", [(4680, 32760), (4681, 32767), (4682, 32774)])
def test_saturation_boundary_closed_form(n, expected):
    # SM(a, a) = 7 puts 7 * n on either side of the int16 maximum 32767
    sm = np.array([[7, -3], [-3, 7]], dtype=np.int32)
    s = np.zeros(n, dtype=np.uint8)
    assert oracle.score(s, s, sm, 10, 2) == expected


@HYP
@given(tiny_case(max_len=16))
def test_invariants(case):
    q, d, sm, go, ge = case
    s = oracle.score(q, d, sm, go, ge)
    assert s >= 0
    # swapping the sequences transposes the matrix
    assert oracle.score(d, q, sm.T.copy(), go, ge) == s
    # larger penalties never raise the score
    assert oracle.score(q, d, sm, go + 1, ge) <= s
    assert oracle.score(q, d, sm, go, ge + 1) <= s
    # a prefix or suffix of the database sequence never scores higher
    if len(d):
        assert oracle.score(q, d[:-1], sm, go, ge) <= s
        assert oracle.score(q, d[1:], sm, go, ge) <= s
    # empty sequences score 0
    assert oracle.score(q, d[:0], sm, go, ge) == 0
    assert oracle.score(q[:0], d, sm, go, ge) == 0
    # the full diagonal is one local alignment of a sequence with itself
    assert oracle.score(q, q, sm, go, ge) >= int(sum(int(sm[x, x]) for x in q))


def test_symmetric_matrix_symmetry_blosum():
    rng = np.random.Generator(np.random.PCG64(17022))
    for _ in range(20):
        a = synth.residues(rng, int(rng.integers(1, 80)))
        b = synth.residues(rng, int(rng.integers(1, 80)))
        for sm in (synth.BLOSUM62, synth.BLOSUM50):
            assert oracle.score(a, b, sm, 10, 2) == oracle.score(b, a, sm, 10, 2)


def test_search_matches_pairwise_and_is_order_independent():
    rng = np.random.Generator(np.random.PCG64(17023))
    db = synth.db_from_lengths(rng, synth.lognormal_lengths(rng, 300, 60, 0.7, 0, 300))
    q = synth.residues(rng, 90)
    sm = synth.BLOSUM62
    full = oracle.search(q, db.residues, db.offsets, sm, 10, 2, threads=4)
    single = oracle.search(q, db.residues, db.offsets, sm, 10, 2, threads=1)
    assert np.array_equal(full, single)
    for k in range(0, 300, 37):
        assert full[k] == oracle.score(q, db.seq(k), sm, 10, 2)
    perm = rng.permutation(300)
    pdb = synth.db_from_seqs([db.seq(int(k)) for k in perm])
    assert np.array_equal(oracle.search(q, pdb.residues, pdb.offsets, sm, 10, 2), full[perm])
    idx = np.array([5, 0, 299, 5], dtype=np.int64)
    assert np.array_equal(oracle.search(q, db.residues, db.offsets, sm, 10, 2, index=idx),
                          full[idx])
