"""Pins of the oracle's operator action: Route 1 (Alg. 1 taken literally)
against Route 2 (masked Galerkin closed form), brute force on the full direct
product, hand-derived matrix elements, the uncoupled closed form, Hermiticity
and Smolyak-quadrature exactness."""
import math
import os

import numpy as np
import pytest

import sg_inputs
from oracle.action import (Oracle, brute_force_masked, galerkin_masked_apply,
                           galerkin_masked_matrix, galerkin_rows)
from oracle.quadrature import smolyak_integrate_monomial
from oracle.smolyak import CompactRanker


def _rand(n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _dense(O):
    n = O.S.n_cs
    return np.stack([O.apply_literal(np.eye(n)[:, j].astype(complex)) for j in range(n)], axis=1)


@pytest.mark.parametrize("D,L", [(1, 3), (2, 4), (3, 3), (4, 2), (2, 5)])
def test_route1_equals_route2_equals_brute_force(D, L):
    inst = sg_inputs.small_instance(D, L, seed=10 * D + L)
    O = Oracle(inst)
    psi = _rand(O.S.n_cs, 1)
    r1 = O.apply_literal(psi)
    H2 = galerkin_masked_matrix(inst)
    r2 = H2 @ psi
    Hb = brute_force_masked(inst, O.S.compact)
    r3 = Hb @ psi
    nrm = np.linalg.norm(r2)
    assert np.linalg.norm(r1 - r2) / nrm < 1e-13
    assert np.linalg.norm(r3 - r2) / nrm < 1e-13


def test_unmasked_galerkin_differs():
    """The mask matters: the plain Galerkin matrix restricted to the compact
    basis is not H_S for coupled H (so a dropped mask fails the route check)."""
    inst = sg_inputs.small_instance(2, 3, seed=5)
    O = Oracle(inst)
    H1 = _dense(O)
    Hb = brute_force_masked(inst, O.S.compact)
    assert np.abs(H1 - Hb).max() < 1e-13
    Hu = brute_force_masked(inst, O.S.compact, mask=False)
    assert np.abs(Hu - H1).max() > 1e-3


def test_golden_matrix_elements(golden_dir):
    inst = sg_inputs.small_instance(2, 2, seed=0)
    inst.omega = np.array([1.0, 1.5])
    inst.c = np.array([[0.0, 0.1], [0.0, 0.0]])
    inst.k = np.array([[0.0, 0.2], [0.0, 0.0]])
    O = Oracle(inst)
    H1 = _dense(O)
    H2 = galerkin_masked_matrix(inst).toarray()
    rk = CompactRanker(2, 2, 1, 2)
    with open(os.path.join(golden_dir, "matrix_elements.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    assert len(rows) >= 6
    for n0, n1, m0, m1, v in rows:
        i = int(rk.rank(np.array([[int(n0), int(n1)]]))[0])
        j = int(rk.rank(np.array([[int(m0), int(m1)]]))[0])
        assert abs(H1[i, j].real - float(v)) < 1e-13, (n0, n1, m0, m1)
        assert abs(H1[j, i].real - float(v)) < 1e-13
        assert abs(H2[i, j] - float(v)) < 1e-14


@pytest.mark.parametrize("D,L", [(2, 4), (3, 3), (4, 3)])
def test_uncoupled_is_diagonal_harmonic(D, L):
    inst = sg_inputs.small_instance(D, L, seed=3)
    inst.c[:] = 0.0
    inst.k[:] = 0.0
    O = Oracle(inst)
    psi = _rand(O.S.n_cs, 2)
    E = (inst.omega[None, :] * (O.S.compact + 0.5)).sum(axis=1)
    r = O.apply_literal(psi)
    assert np.linalg.norm(r - E * psi) / np.linalg.norm(E * psi) < 1e-13


@pytest.mark.parametrize("D,L", [(2, 4), (3, 3), (5, 2)])
def test_hermiticity(D, L):
    inst = sg_inputs.small_instance(D, L, seed=4)
    O = Oracle(inst)
    phi, psi = _rand(O.S.n_cs, 5), _rand(O.S.n_cs, 6)
    lhs = np.vdot(phi, O.apply_literal(psi))
    rhs = np.conj(np.vdot(psi, O.apply_literal(phi)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_general_size_maps_route1_vs_brute_force():
    """N_l = A + B l with other A, B (Route 2 needs nq >= nb+1; brute force
    needs exactness at the top level only)."""
    inst = sg_inputs.small_instance(2, 3, seed=8, nb=(2, 1), nq=(4, 1))
    O = Oracle(inst)
    psi = _rand(O.S.n_cs, 9)
    r1 = O.apply_literal(psi)
    r2 = galerkin_masked_matrix(inst) @ psi
    assert np.linalg.norm(r1 - r2) / np.linalg.norm(r2) < 1e-13


def test_galerkin_rows_match_matrix():
    inst = sg_inputs.small_instance(4, 3, seed=11)
    rk = CompactRanker(4, 3, 1, 2)
    E = rk.enumerate()
    H = galerkin_masked_matrix(inst, rk, E).toarray()
    sel = E[[0, 3, 17, len(E) - 1]]
    for (cols, vals), i in zip(galerkin_rows(inst, rk, sel), [0, 3, 17, len(E) - 1]):
        row = np.zeros(len(E))
        np.add.at(row, cols, vals)
        assert np.abs(row - H[i]).max() < 1e-14


@pytest.mark.parametrize("D,L,seed", [(2, 4, 1), (4, 3, 2), (5, 3, 3), (3, 5, 4)])
def test_masked_apply_matches_route1_and_matrix(D, L, seed):
    """The matrix-free Route 2 equals the literal Alg. 1 (Route 1) and the
    assembled masked matrix on the same state."""
    inst = sg_inputs.small_instance(D, L, seed=seed)
    O = Oracle(inst)
    psi = _rand(O.S.n_cs, seed)
    r1 = O.apply_literal(psi)
    r2 = galerkin_masked_matrix(inst) @ psi
    r3 = galerkin_masked_apply(inst, psi, O.S.compact)
    assert np.linalg.norm(r3 - r1) / np.linalg.norm(r1) < 1e-13
    assert np.abs(r3 - r2).max() < 1e-13 * np.abs(r2).max()


def test_masked_apply_rejects_unordered_basis():
    inst = sg_inputs.small_instance(2, 2, seed=1)
    rk = CompactRanker(2, 2, 1, 2)
    E = rk.enumerate()[::-1]
    with pytest.raises(ValueError):
        galerkin_masked_apply(inst, np.ones(len(E)), E)


def _exact_monomial(alpha):
    out = 1.0
    for a in alpha:
        if a % 2:
            return 0.0
        out *= math.gamma((a + 1) / 2)
    return out


def test_smolyak_quadrature_exactness():
    """The Smolyak combination of the 2l+2-point rules with weights D_l is
    exact on prod_i x_i^a_i e^{-x_i^2} when sum_i max(0, ceil((a_i-3)/4)) <= L;
    e.g. D=3, L=2."""
    D, L = 3, 2
    for alpha in [(0, 0, 0), (2, 2, 2), (4, 0, 0), (6, 2, 0), (7, 3, 1),
                  (10, 0, 0), (11, 2, 2), (6, 6, 2), (4, 4, 3)]:
        need = sum(max(0, math.ceil((a - 3) / 4)) for a in alpha)
        assert need <= L
        got = smolyak_integrate_monomial(D, L, 2, 2, alpha)
        ex = _exact_monomial(alpha)
        assert abs(got - ex) <= 1e-12 * max(1.0, abs(ex)), alpha
    # and not exact beyond that level
    got = smolyak_integrate_monomial(D, L, 2, 2, (12, 0, 0))
    assert abs(got - _exact_monomial((12, 0, 0))) > 1e-3
