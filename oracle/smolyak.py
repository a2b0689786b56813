"""Smolyak term set, combination coefficients, compact basis, mapping table.

Oracle (test infrastructure only).

Sec. 2 (Method), the Smolyak representation S_L: the terms are the level
vectors l (l_i >= 0) with L-n+1 <= |l| <= L, each weighted by
D_l = (-1)^(L-|l|) * C(n-1, L-|l|); the per-mode sizes follow N_l = A + B*l.
Sec. 3 (Implementation) and Table 2: the compact basis is the union of all
term bases with duplicates removed, and the mapping table M^B sends (term,
position in term) to the compact index.  Table 2 fixes the orderings:
terms are listed with l_1 varying fastest, positions inside a term with mode 1
fastest, and the compact basis is lexicographic with mode 1 slowest.

Indices here are 0-based (the paper's are 1-based).
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass

import numpy as np


def size_of_level(level, A: int, B: int):
    """N_l = A + B*l (Sec. 2)."""
    return A + B * level


def level_vectors(D: int, L: int) -> list[tuple[int, ...]]:
    """All l in N^D with L-D+1 <= |l| <= L, l_1 fastest (Table 2 order)."""
    lo = L - D + 1
    out: list[tuple[int, ...]] = []

    # Recurse from the slowest mode (mode D) to the fastest (mode 1) so that
    # the emitted sequence has l_1 varying fastest.
    def rec(mode: int, budget: int, suffix: tuple[int, ...]):
        if mode < 0:
            l = suffix
            if sum(l) >= lo:
                out.append(l)
            return
        for v in range(budget + 1):
            rec(mode - 1, budget - v, (v,) + suffix)

    # rec builds tuples right-to-left, so iterate the slowest mode outermost.
    rec(D - 1, L, ())
    return out


def comb_coeff(D: int, L: int, l) -> int:
    """D_l = (-1)^(L-|l|) C(D-1, L-|l|) (Sec. 2)."""
    s = L - int(sum(l))
    if s < 0 or s > D - 1:
        return 0
    return (-1) ** s * math.comb(D - 1, s)


def term_basis_tuples(l, nbA: int, nbB: int) -> list[tuple[int, ...]]:
    """Basis tuples of one term, mode 1 fastest (Table 2 ordering)."""
    sizes = [size_of_level(li, nbA, nbB) for li in l]
    # itertools.product varies the last factor fastest: feed reversed sizes
    # and reverse each tuple back.
    return [tuple(reversed(t)) for t in
            itertools.product(*[range(s) for s in reversed(sizes)])]


@dataclass
class SmolyakStructure:
    D: int
    L: int
    nbA: int
    nbB: int
    terms: list            # list of level tuples, Table 2 order
    coeffs: np.ndarray     # D_l per term, int64
    compact: np.ndarray    # [N_cs, D] int64, lexicographic, mode 1 slowest
    term_offsets: np.ndarray  # [N_st+1], start of each term in the N_s layout
    MB: np.ndarray         # [N_s] compact index of every (term, position)

    @property
    def n_terms(self):
        return len(self.terms)

    @property
    def n_cs(self):
        return self.compact.shape[0]

    @property
    def n_s(self):
        return int(self.term_offsets[-1])


def build_structure_literal(D: int, L: int, nbA: int, nbB: int) -> SmolyakStructure:
    """Builds everything by the paper's definitions, literally: enumerate every
    term's basis tuples, take the union (duplicates removed), sort it, and map
    each (term, position) to its compact index.  Small cases only."""
    terms = level_vectors(D, L)
    coeffs = np.array([comb_coeff(D, L, l) for l in terms], dtype=np.int64)
    per_term = [term_basis_tuples(l, nbA, nbB) for l in terms]
    union = sorted(set(itertools.chain.from_iterable(per_term)))
    index = {t: i for i, t in enumerate(union)}
    offsets = np.zeros(len(terms) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum([len(p) for p in per_term])
    MB = np.fromiter((index[t] for p in per_term for t in p), dtype=np.int64,
                     count=int(offsets[-1]))
    compact = np.array(union, dtype=np.int64).reshape(len(union), D)
    return SmolyakStructure(D, L, nbA, nbB, terms, coeffs, compact, offsets, MB)


# ---------------------------------------------------------------------------
# Closed-form characterisation of the compact basis (faster; pinned against
# the literal union above on small cases).  A basis index n of one mode
# belongs to a term of level l iff n < N_l, so the lowest level holding n is
# g(n) = min{l : A + B l > n}; a tuple n is in the compact basis iff some l in
# R(l) dominates g(n), i.e. iff sum_i g(n_i) <= L.
# ---------------------------------------------------------------------------

def lowest_level(n, nbA: int, nbB: int):
    n = np.asarray(n)
    return np.maximum(0, (n - nbA) // nbB + 1)


class CompactRanker:
    """Rank of a tuple in the lexicographic (mode 1 slowest) compact order."""

    def __init__(self, D: int, L: int, nbA: int, nbB: int):
        self.D, self.L, self.nbA, self.nbB = D, L, nbA, nbB
        nmax = size_of_level(L, nbA, nbB) - 1
        self.nmax = nmax
        g = lowest_level(np.arange(nmax + 1), nbA, nbB)
        self.g = g
        # cnt[d][b]: number of tuples over d modes with sum g <= b
        cnt = np.zeros((D + 1, L + 1), dtype=np.int64)
        cnt[0, :] = 1
        for d in range(1, D + 1):
            for b in range(L + 1):
                cnt[d, b] = sum(int(cnt[d - 1, b - gv]) for gv in g if gv <= b)
        self.cnt = cnt
        # pre[d][b][x] = sum_{v<x, g(v)<=b} cnt[d][b-g(v)]
        pre = np.zeros((D + 1, L + 1, nmax + 2), dtype=np.int64)
        for d in range(D + 1):
            for b in range(L + 1):
                acc = 0
                for x in range(nmax + 1):
                    pre[d, b, x] = acc
                    if g[x] <= b:
                        acc += int(cnt[d, b - g[x]])
                pre[d, b, nmax + 1] = acc
        self.pre = pre

    @property
    def size(self):
        return int(self.cnt[self.D, self.L])

    def rank(self, tuples: np.ndarray) -> np.ndarray:
        """tuples: [M, D] ints, all members of the compact set."""
        t = np.asarray(tuples, dtype=np.int64)
        budget = np.full(t.shape[0], self.L, dtype=np.int64)
        r = np.zeros(t.shape[0], dtype=np.int64)
        for i in range(self.D):
            rest = self.D - 1 - i
            r += self.pre[rest, budget, t[:, i]]
            budget = budget - self.g[t[:, i]]
        return r

    def contains(self, tuples: np.ndarray) -> np.ndarray:
        t = np.asarray(tuples, dtype=np.int64)
        ok = np.all((t >= 0) & (t <= self.nmax), axis=1)
        tc = np.clip(t, 0, self.nmax)
        return ok & (self.g[tc].sum(axis=1) <= self.L)

    def enumerate(self) -> np.ndarray:
        """All compact tuples in rank order."""
        out = []

        def rec(prefix, budget):
            if len(prefix) == self.D:
                out.append(prefix)
                return
            for x in range(self.nmax + 1):
                if self.g[x] <= budget:
                    rec(prefix + (x,), budget - int(self.g[x]))

        rec((), self.L)
        return np.array(out, dtype=np.int64).reshape(len(out), self.D)


def build_structure(D: int, L: int, nbA: int, nbB: int) -> SmolyakStructure:
    """Same result as build_structure_literal, computed with the ranker
    (usable up to a few million basis entries)."""
    terms = level_vectors(D, L)
    coeffs = np.array([comb_coeff(D, L, l) for l in terms], dtype=np.int64)
    rk = CompactRanker(D, L, nbA, nbB)
    compact = rk.enumerate()
    sizes = [int(np.prod([size_of_level(li, nbA, nbB) for li in l])) for l in terms]
    offsets = np.zeros(len(terms) + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(sizes)
    MB = np.empty(int(offsets[-1]), dtype=np.int64)
    for t, l in enumerate(terms):
        nbs = [size_of_level(li, nbA, nbB) for li in l]
        # all tuples of this term, mode 1 fastest (Fortran order)
        grids = np.indices(nbs).reshape(D, -1, order="F").T
        MB[offsets[t]:offsets[t + 1]] = rk.rank(grids)
    return SmolyakStructure(D, L, nbA, nbB, terms, coeffs, compact, offsets, MB)


def count_sizes(D: int, L: int, nbA: int, nbB: int) -> tuple[int, int, int]:
    """(N_st, N_s, N_cs) by counting, without enumeration (Table 1 scale).

    N_s = sum over R(l) of prod_i N_{l_i} and N_cs = #{n : sum_i g(n_i) <= L},
    each computed as a coefficient extraction from a D-th power of a
    one-mode polynomial in the level variable."""
    # per-mode polynomials truncated at degree L
    P = [size_of_level(l, nbA, nbB) for l in range(L + 1)]       # sizes
    G = [size_of_level(l, nbA, nbB) - (size_of_level(l - 1, nbA, nbB) if l > 0 else 0)
         for l in range(L + 1)]                                  # new indices at level l
    ONE = [1] * (L + 1)

    def power(poly, e):
        res = [1] + [0] * L
        for _ in range(e):
            nxt = [0] * (L + 1)
            for a, ca in enumerate(res):
                if ca == 0:
                    continue
                for b, cb in enumerate(poly):
                    if a + b > L:
                        break
                    nxt[a + b] += ca * cb
            res = nxt
        return res

    lo = max(0, L - D + 1)
    PD = power(P, D)
    GD = power(G, D)
    CD = power(ONE, D)
    n_s = sum(PD[m] for m in range(lo, L + 1))
    n_cs = sum(GD[m] for m in range(0, L + 1))
    n_st = sum(CD[m] for m in range(lo, L + 1))
    return n_st, n_s, n_cs
