"""One-mode primitive basis and grid tables.

Oracle (test infrastructure only).

The paper's worked example uses the "Hm" primitive basis (harmonic-oscillator
Hermite functions centred at Q0=0 with scaleQ=1, Example subsection of Sec. 4) and the
basis<->grid transforms eq_b_to_g and eq_g_to_b of Sec. 2, where the grid
transform weights each point by w_u b_k(Q_u).  Reading of the weight
convention: the Gauss-Hermite weights w_u integrate f(x) e^{-x^2}; the
Hermite functions already carry e^{-x^2/2}, so the weight that makes
sum_u wt_u f(Q_u) approximate the plain integral of f is wt_u = w_u e^{Q_u^2}.

Tables per level (nb functions, nq points):
  x, wt      nodes and modified weights              [nq]
  b          b_k(x_u)                                 [nq, nb]
  d2b        second derivative d^2 b_k / dx^2 (x_u)   [nq, nb]
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.hermite import hermgauss


def gauss_hermite(nq: int):
    """Nodes x_u and weights w_u of the nq-point Gauss-Hermite rule (library
    routine), plus the modified weights wt_u = w_u exp(x_u^2)."""
    x, w = hermgauss(nq)
    return x, w, w * np.exp(x * x)


def hermite_functions(nb: int, x: np.ndarray) -> np.ndarray:
    """Orthonormal Hermite functions b_0..b_{nb-1} at x, shape [len(x), nb].

    b_0 = pi^{-1/4} e^{-x^2/2}, b_1 = sqrt(2) x b_0,
    b_{n+1} = sqrt(2/(n+1)) x b_n - sqrt(n/(n+1)) b_{n-1}
    (the three-term recurrence of the normalised physicists' polynomials
    times the Gaussian; positive leading coefficient)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros((x.size, nb))
    if nb == 0:
        return out
    out[:, 0] = np.pi ** -0.25 * np.exp(-0.5 * x * x)
    if nb > 1:
        out[:, 1] = np.sqrt(2.0) * x * out[:, 0]
    for n in range(1, nb - 1):
        out[:, n + 1] = (np.sqrt(2.0 / (n + 1)) * x * out[:, n]
                         - np.sqrt(n / (n + 1)) * out[:, n - 1])
    return out


def hermite_second_derivatives(nb: int, x: np.ndarray) -> np.ndarray:
    """d^2 b_n/dx^2 = (x^2 - (2n+1)) b_n (the Hermite-function ODE)."""
    b = hermite_functions(nb, x)
    n = np.arange(nb)
    return (np.asarray(x)[:, None] ** 2 - (2 * n[None, :] + 1)) * b


class LevelTables:
    """Tables for level l with nb = nbA + nbB l functions and nq = nqA + nqB l
    points."""

    def __init__(self, level: int, nbA: int, nbB: int, nqA: int, nqB: int):
        self.level = level
        self.nb = nbA + nbB * level
        self.nq = nqA + nqB * level
        self.x, self.w, self.wt = gauss_hermite(self.nq)
        self.b = hermite_functions(self.nb, self.x)            # [nq, nb]
        self.d2b = hermite_second_derivatives(self.nb, self.x)  # [nq, nb]
        self.wtb_T = (self.wt[:, None] * self.b).T              # [nb, nq]


def tables_for(L: int, nbA: int, nbB: int, nqA: int, nqB: int) -> list[LevelTables]:
    return [LevelTables(l, nbA, nbB, nqA, nqB) for l in range(L + 1)]
