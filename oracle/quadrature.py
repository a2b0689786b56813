"""Smolyak quadrature with the term set R(l) and weights D_l.

Oracle (test infrastructure only).  Used only to pin R(l), D_l and the
one-mode Gauss-Hermite rules: the Smolyak combination of Sec. 2
(S_L = sum_{R(l)} D_l S_{l_1} x ... x S_{l_n}), applied to grids instead of
bases, is a quadrature rule whose exactness on monomials is known in closed
form.
"""
from __future__ import annotations

import numpy as np

from .hermite import gauss_hermite
from .smolyak import comb_coeff, level_vectors, size_of_level


def smolyak_integrate_monomial(D: int, L: int, nqA: int, nqB: int, alpha) -> float:
    """sum_l D_l prod_i GH_{nq(l_i)}[x^{alpha_i}] with the e^{-x^2} weight."""
    total = 0.0
    cache = {}
    for l in level_vectors(D, L):
        Dl = comb_coeff(D, L, l)
        if Dl == 0:
            continue
        prod = 1.0
        for li, ai in zip(l, alpha):
            key = (li, ai)
            if key not in cache:
                x, w, _ = gauss_hermite(size_of_level(li, nqA, nqB))
                cache[key] = float(np.sum(w * x ** ai))
            prod *= cache[key]
        total += Dl * prod
    return total
