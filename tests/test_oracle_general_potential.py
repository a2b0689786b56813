"""Pins of the oracle's Route 1 (Alg. 1 taken literally) with a general,
non-polynomial coupling potential V(Q).

A general V makes each term's product rule inexact, so the masked-Galerkin
closed form (Route 2) no longer applies.  What still fixes the result:

* A polynomial V passed as a function must give Route 2 exactly (the
  function path reaches the same per-term quadrature).
* For V = f(Q_a) (one mode), each term's operator is the one-mode quadrature
  matrix F^(l_a) of f on mode a times the identity on the other modes (their
  rules integrate products of basis functions exactly), so the combination
  technique gives sum_{|j| <= L} Delta F^(j_a) (x) Delta P^(j_i): with
  n_rest = m_rest and S = sum_{i != a} g(n_i), H_S[n, m] = F^(L - S)[n_a, m_a]
  (zero when n_a or m_a exceeds 2 (L - S)), and zero for n_rest != m_rest.
* For V = f(Q_a) h(Q_b) the same argument gives
  H_S[n, m] = sum_{j <= M} (F^(j) - F^(j-1))[n_a, m_a] H^(M - j)[n_b, m_b],
  M = L - sum_{i != a, b} g(n_i).
* Hermiticity.
F^(l)[n, m] = sum_u wt_u phi_n(x_u) f(x_u) phi_m(x_u) on the 2l+2-point
Gauss-Hermite rule, with Hermite functions from scipy's Hermite polynomials
(independent of the oracle's tables).
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite import hermgauss
from scipy.special import eval_hermite

import sg_inputs
from oracle.action import Oracle, galerkin_masked_matrix


def _phi(nmax, x):
    """Orthonormal Hermite functions phi_0..phi_nmax at x: [nmax+1, len(x)]."""
    out = []
    for n in range(nmax + 1):
        norm = 1.0 / math.sqrt(2.0 ** n * math.factorial(n) * math.sqrt(math.pi))
        out.append(norm * eval_hermite(n, x) * np.exp(-0.5 * x * x))
    return np.array(out)


def _F(f, l):
    """One-mode quadrature matrix of f at level l (nb = 2l+1, nq = 2l+2)."""
    x, w = hermgauss(2 * l + 2)
    wt = w * np.exp(x * x)
    P = _phi(2 * l, x)
    return (P * (wt * f(x))) @ P.T


def _Fpad(f, l, size):
    M = np.zeros((size, size))
    if l >= 0:
        F = _F(f, l)
        M[:F.shape[0], :F.shape[1]] = F
    return M


def _g(n):
    return (n + 1) // 2


def _dense(O):
    n = O.S.n_cs
    return np.stack([O.apply_literal(np.eye(n)[:, j].astype(complex)) for j in range(n)], axis=1)


def _coupling_part(O):
    """H_S minus its exact harmonic diagonal sum_i omega_i (n_i + 1/2)."""
    H = _dense(O)
    h0 = (O.S.compact + 0.5) @ O.inst.omega
    return H - np.diag(h0)


def f1(x):
    return np.cos(1.3 * x) + 0.4 * np.exp(-x * x)


def f2(x):
    return 1.0 / (1.0 + 0.5 * x * x)


@pytest.mark.parametrize("D,L", [(2, 4), (3, 3), (4, 2)])
def test_polynomial_as_function_equals_route2(D, L):
    inst = sg_inputs.small_instance(D, L, seed=40 + D + L)
    c, k = inst.c, inst.k

    def poly(Q):
        V = 0.0
        for i in range(D):
            for j in range(i + 1, D):
                V = V + c[i, j] * Q[i] ** 2 * Q[j] ** 2 + k[i, j] * Q[i] ** 2 * Q[j]
        return V

    O = Oracle(inst, coupling=poly)
    rng = np.random.default_rng(5)
    psi = rng.standard_normal(O.S.n_cs) + 1j * rng.standard_normal(O.S.n_cs)
    r1 = O.apply_literal(psi)
    r2 = galerkin_masked_matrix(inst) @ psi
    assert np.linalg.norm(r1 - r2) / np.linalg.norm(r2) < 1e-13


@pytest.mark.parametrize("D,L,a", [(2, 4, 0), (2, 4, 1), (3, 3, 1), (4, 2, 3), (3, 0, 2), (1, 5, 0)])
def test_one_mode_potential_closed_form(D, L, a):
    inst = sg_inputs.small_instance(D, L, seed=7)
    O = Oracle(inst, coupling=lambda Q: f1(Q[a]))
    Hc = _coupling_part(O)
    comp = O.S.compact
    n = comp.shape[0]
    ref = np.zeros((n, n))
    Fs = {}
    for r in range(n):
        for s in range(n):
            rest = [i for i in range(D) if i != a]
            if any(comp[r, i] != comp[s, i] for i in rest):
                continue
            M = L - sum(_g(int(comp[r, i])) for i in rest)
            if max(comp[r, a], comp[s, a]) > 2 * M:
                continue
            if M not in Fs:
                Fs[M] = _F(f1, M)
            ref[r, s] = Fs[M][comp[r, a], comp[s, a]]
    assert np.abs(Hc - ref).max() < 1e-13
    # the potential is genuinely inexact here: the level-L and level-0 rules differ
    assert abs(_F(f1, 0)[0, 0] - _F(f1, L)[0, 0]) > 1e-4 or L == 0


@pytest.mark.parametrize("D,L,a,b", [(2, 4, 0, 1), (3, 3, 0, 2), (4, 2, 1, 3), (2, 5, 1, 0)])
def test_two_mode_product_closed_form(D, L, a, b):
    inst = sg_inputs.small_instance(D, L, seed=9)
    O = Oracle(inst, coupling=lambda Q: f1(Q[a]) * f2(Q[b]))
    Hc = _coupling_part(O)
    comp = O.S.compact
    n = comp.shape[0]
    size = 2 * L + 1
    Fp = [_Fpad(f1, j, size) for j in range(-1, L + 1)]   # Fp[j + 1] = F^(j)
    Hp = [_Fpad(f2, j, size) for j in range(-1, L + 1)]
    ref = np.zeros((n, n))
    rest = [i for i in range(D) if i not in (a, b)]
    for r in range(n):
        for s in range(n):
            if any(comp[r, i] != comp[s, i] for i in rest):
                continue
            M = L - sum(_g(int(comp[r, i])) for i in rest)
            na_, ma_, nb_, mb_ = comp[r, a], comp[s, a], comp[r, b], comp[s, b]
            v = 0.0
            for j in range(M + 1):
                dF = Fp[j + 1][na_, ma_] - Fp[j][na_, ma_]
                v += dF * Hp[M - j + 1][nb_, mb_]
            ref[r, s] = v
    assert np.abs(Hc - ref).max() < 1e-13


@pytest.mark.parametrize("D,L", [(3, 3), (4, 3), (5, 2)])
def test_general_potential_hermitian(D, L):
    inst = sg_inputs.small_instance(D, L, seed=11)
    V = sg_inputs.general_potential(D, seed=3)
    O = Oracle(inst, coupling=V)
    rng = np.random.default_rng(2)
    n = O.S.n_cs
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lhs = np.vdot(x, O.apply_literal(y))
    rhs = np.conj(np.vdot(y, O.apply_literal(x)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_general_potential_points_match_grid_form():
    """The (n, D) point interface the library calls and the broadcasting
    interface Route 1 uses evaluate the same function."""
    V = sg_inputs.general_potential(4, seed=3)
    rng = np.random.default_rng(0)
    P = rng.standard_normal((50, 4))
    a = V.at_points(P)
    b = np.array([V([P[i, 0], P[i, 1], P[i, 2], P[i, 3]]) for i in range(50)])
    assert np.array_equal(a, b)
