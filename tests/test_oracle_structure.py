"""Pins of the oracle's Smolyak structure against the paper's printed values
(Tables 1 and 2) and against closed-form identities."""
import itertools
import math
import os

import numpy as np
import pytest

from oracle.smolyak import (CompactRanker, build_structure,
                            build_structure_literal, comb_coeff, count_sizes,
                            level_vectors, lowest_level)


def _read_table2(golden_dir):
    data = {}
    with open(os.path.join(golden_dir, "table2_mapping.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, val = line.split(":", 1)
            data[key.strip()] = val.strip()
    return data


def test_table2_terms_mapping_and_compact_order(golden_dir):
    g = _read_table2(golden_dir)
    S = build_structure_literal(2, 3, 1, 1)
    terms = [tuple(int(x) for x in t.split(",")) for t in g["terms"].split()]
    assert S.terms == terms
    groups = [[int(x) for x in grp.split()] for grp in g["MB"].split("|")]
    assert (S.MB + 1).tolist() == [x for grp in groups for x in grp]
    sizes = np.diff(S.term_offsets).tolist()
    assert sizes == [len(grp) for grp in groups]
    compact = [tuple(int(x) - 1 for x in t.split(",")) for t in g["compact"].split()]
    assert [tuple(r) for r in S.compact.tolist()] == compact
    assert S.n_terms == int(g["n_terms"])
    assert S.n_s == int(g["n_s"])
    assert S.n_cs == int(g["n_cs"])


def test_table2_combination_coefficients():
    # D_l = (-1)^(L-|l|) C(n-1, L-|l|) for the 7 terms of the 2-D, L=3 example:
    # |l| = 3 -> +1, |l| = 2 -> -1.
    S = build_structure_literal(2, 3, 1, 1)
    assert S.coeffs.tolist() == [-1, 1, -1, 1, -1, 1, 1]


def test_table1_counts(golden_dir):
    with open(os.path.join(golden_dir, "table1_counts.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for D, L, ns, ncs in rows:
        D, L, ns, ncs = int(D), int(L), int(ns), int(ncs)
        _, n_s, n_cs = count_sizes(D, L, 1, 1)
        assert (n_s, n_cs) == (ns, ncs), (D, L)
        if D == 12 and L <= 4:
            S = build_structure(D, L, 1, 1)
            assert S.n_s == ns and S.n_cs == ncs


@pytest.mark.parametrize("D,L,nbA,nbB", [(2, 3, 1, 1), (3, 3, 1, 2), (4, 2, 1, 2),
                                         (3, 4, 2, 1), (2, 5, 1, 3)])
def test_ranker_matches_literal_union(D, L, nbA, nbB):
    A = build_structure_literal(D, L, nbA, nbB)
    B = build_structure(D, L, nbA, nbB)
    assert A.terms == B.terms
    assert np.array_equal(A.compact, B.compact)
    assert np.array_equal(A.MB, B.MB)
    n_st, n_s, n_cs = count_sizes(D, L, nbA, nbB)
    assert (n_st, n_s, n_cs) == (A.n_terms, A.n_s, A.n_cs)


@pytest.mark.parametrize("D,L", [(1, 4), (2, 4), (3, 3), (5, 3), (6, 6)])
def test_combination_identity(D, L):
    """sum of D_l over the terms whose basis holds n is 1 for every compact n
    (so the Smolyak sum reproduces a diagonal operator exactly), and
    sum_R D_l = 1."""
    S = build_structure(D, L, 1, 2)
    acc = np.zeros(S.n_cs, dtype=np.int64)
    for t in range(S.n_terms):
        acc[S.MB[S.term_offsets[t]:S.term_offsets[t + 1]]] += S.coeffs[t]
    assert (acc == 1).all()
    assert int(S.coeffs.sum()) == 1


def test_term_set_restriction_and_count():
    for D, L in [(2, 4), (6, 6), (12, 6)]:
        T = level_vectors(D, L)
        assert all(max(0, L - D + 1) <= sum(l) <= L for l in T)
        assert len(set(T)) == len(T)
        # every level vector with that |l| is present: count by stars and bars
        lo = max(0, L - D + 1)
        assert len(T) == sum(math.comb(m + D - 1, D - 1) for m in range(lo, L + 1))
        assert all(comb_coeff(D, L, l) != 0 for l in T)


def test_compact_closed_form_nb_2l_plus_1():
    # with N_l = 1 + 2l: N_cs = sum_j C(D, j) C(L, j) 2^j (a count of tuples
    # with sum_i ceil(n_i/2) <= L)
    for D, L in [(2, 4), (6, 6), (12, 6), (10, 7)]:
        _, _, ncs = count_sizes(D, L, 1, 2)
        assert ncs == sum(math.comb(D, j) * math.comb(L, j) * 2 ** j for j in range(0, min(D, L) + 1))


def test_lowest_level():
    assert lowest_level(np.arange(7), 1, 2).tolist() == [0, 1, 1, 2, 2, 3, 3]
    assert lowest_level(np.arange(5), 1, 1).tolist() == [0, 1, 2, 3, 4]


def test_ranker_roundtrip():
    rk = CompactRanker(5, 4, 1, 2)
    E = rk.enumerate()
    assert np.array_equal(rk.rank(E), np.arange(E.shape[0]))
    assert rk.contains(E).all()
    # lexicographic, mode 1 slowest
    keys = [tuple(r) for r in E.tolist()]
    assert keys == sorted(keys)


def test_ranker_contains_rejects_non_members():
    """The compact set is {n : 0 <= n_i <= nmax, sum_i g(n_i) <= L} (the union
    of the term bases, Sec. 3 and Table 2).  Tuples just past the level budget,
    with a negative entry or with an entry above the largest one-mode index are
    outside it; brute force over a box decides every tuple."""
    D, L = 3, 3
    rk = CompactRanker(D, L, 1, 2)
    g = lambda n: (n + 1) // 2          # lowest level holding index n (nb = 2l+1)
    nmax = 2 * L
    box = np.array(list(itertools.product(range(-1, nmax + 2), repeat=D)), dtype=np.int64)
    want = np.array([all(0 <= x <= nmax for x in t) and sum(g(x) for x in t) <= L
                     for t in box.tolist()])
    got = rk.contains(box)
    assert np.array_equal(got, want)
    assert (~want).sum() > 0 and want.sum() == rk.size
    # level budget L + 1 exactly: rejected
    assert not rk.contains(np.array([[3, 2, 2], [6, 1, 0], [0, 0, 7]])).any()
    assert not rk.contains(np.array([[-1, 0, 0], [0, -2, 1]])).any()
    assert rk.contains(np.array([[2, 2, 1], [6, 0, 0], [0, 0, 5]])).all()
