"""Pins of the oracle's one-mode tables against closed forms (not against the
library routines the oracle calls)."""
import math

import numpy as np
import pytest

from oracle.hermite import (LevelTables, gauss_hermite, hermite_functions,
                            hermite_second_derivatives)


def hermite_poly_explicit(n, x):
    """Physicists' H_n(x) = n! sum_m (-1)^m (2x)^(n-2m) / (m! (n-2m)!)."""
    x = np.asarray(x, dtype=np.float64)
    s = np.zeros_like(x)
    for m in range(n // 2 + 1):
        s += (-1) ** m * (2 * x) ** (n - 2 * m) / (math.factorial(m) * math.factorial(n - 2 * m))
    return math.factorial(n) * s


@pytest.mark.parametrize("nq", [2, 4, 6, 8, 12, 16])
def test_nodes_are_roots_and_rule_is_exact(nq):
    x, w, wt = gauss_hermite(nq)
    # nodes are the roots of H_nq (relative to the polynomial's scale)
    scale = np.abs(hermite_poly_explicit(nq, x + 0.1)).max()
    assert np.abs(hermite_poly_explicit(nq, x)).max() < 1e-11 * scale
    # exact for x^p e^{-x^2}, p <= 2 nq - 1:  int = Gamma((p+1)/2) for even p
    for p in range(0, 2 * nq):
        exact = math.gamma((p + 1) / 2) if p % 2 == 0 else 0.0
        got = float(np.sum(w * x ** p))
        scale = float(np.sum(w * np.abs(x) ** p))
        assert abs(got - exact) <= 1e-13 * max(1.0, scale), p
    # modified weights: wt = w e^{x^2}
    assert np.allclose(wt, w * np.exp(x * x), rtol=1e-15)


def test_hermite_functions_closed_form():
    x = np.linspace(-5, 5, 41)
    b = hermite_functions(12, x)
    for n in range(12):
        ref = hermite_poly_explicit(n, x) * np.exp(-x * x / 2) / math.sqrt(
            2.0 ** n * math.factorial(n) * math.sqrt(math.pi))
        assert np.allclose(b[:, n], ref, atol=1e-13, rtol=1e-12)


def test_second_derivative_finite_difference():
    x = np.linspace(-3, 3, 13)
    h = 1e-3
    d2 = hermite_second_derivatives(7, x)
    fd = (hermite_functions(7, x + h) - 2 * hermite_functions(7, x) + hermite_functions(7, x - h)) / h ** 2
    assert np.allclose(d2, fd, atol=1e-6)


@pytest.mark.parametrize("level", range(0, 8))
def test_level_tables_orthonormal_and_kinetic(level):
    T = LevelTables(level, 1, 2, 2, 2)
    # b^T W b = I exactly (quadrature degree 2(nb-1) <= 2 nq - 1)
    M = T.wtb_T @ T.b
    assert np.abs(M - np.eye(T.nb)).max() < 1e-13
    # <m| -1/2 d^2 + 1/2 Q^2 |n> = (n + 1/2) delta (harmonic oscillator)
    Hho = T.wtb_T @ (-0.5 * T.d2b + 0.5 * (T.x ** 2)[:, None] * T.b)
    assert np.abs(Hho - np.diag(np.arange(T.nb) + 0.5)).max() < 1e-12
