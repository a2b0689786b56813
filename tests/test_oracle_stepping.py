"""Pins of the oracle's Taylor, Runge-Kutta, Bulirsch-Stoer and
short-iterative-Lanczos propagators: the uncoupled closed form (each
eigencomponent is multiplied by a known polynomial or phase), a dense matrix
exponential of the coupled operator, and the convergence orders of the
Runge-Kutta tableaux and of the extrapolation."""
import numpy as np
import pytest
from scipy.linalg import expm

import sg_inputs
from oracle.action import Oracle, galerkin_masked_matrix
from oracle.propagate import coherent_coefficients
from oracle.stepping import (RK_TABLEAUX, lanczos_basis, propagate, rk_step, sil_step,
                             taylor_factor, taylor_step)


def _uncoupled():
    inst = sg_inputs.small_instance(3, 3, seed=2)
    inst.c[:] = 0.0
    inst.k[:] = 0.0
    O = Oracle(inst)
    E = (inst.omega[None, :] * (O.S.compact + 0.5)).sum(axis=1)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    return O, E, psi0


@pytest.mark.parametrize("order", [1, 2, 3, 4, 6, 10])
def test_taylor_uncoupled_polynomial(order):
    O, E, psi0 = _uncoupled()
    dt = 0.07
    got = taylor_step(O.apply_literal, psi0, dt, order)
    ref = np.array([taylor_factor(-1j * e * dt, order) for e in E]) * psi0
    assert np.linalg.norm(got - ref) < 1e-13


@pytest.mark.parametrize("order", [1, 2, 3, 4])
def test_rk_uncoupled_polynomial(order):
    """On a linear equation an explicit Runge-Kutta method of order s <= 4
    with s stages multiplies each eigencomponent by the degree-s Taylor
    polynomial of exp(z)."""
    O, E, psi0 = _uncoupled()
    dt = 0.05
    got = rk_step(O.apply_literal, psi0, dt, order)
    ref = np.array([taylor_factor(-1j * e * dt, order) for e in E]) * psi0
    assert np.linalg.norm(got - ref) < 1e-13


def test_rk_tableaux_consistent():
    """Row sums of A (the stage times) and sum(b) = 1, and the order
    conditions up to each tableau's order."""
    for s, (A, b) in RK_TABLEAUX.items():
        c = A.sum(axis=1)
        assert abs(b.sum() - 1.0) < 1e-15
        if s >= 2:
            assert abs(b @ c - 0.5) < 1e-15
        if s >= 3:
            assert abs(b @ c ** 2 - 1.0 / 3.0) < 1e-15
            assert abs(b @ (A @ c) - 1.0 / 6.0) < 1e-15
        if s >= 4:
            assert abs(b @ c ** 3 - 0.25) < 1e-15
            assert abs(b @ (c * (A @ c)) - 1.0 / 8.0) < 1e-15
            assert abs(b @ (A @ c ** 2) - 1.0 / 12.0) < 1e-15
            assert abs(b @ (A @ (A @ c)) - 1.0 / 24.0) < 1e-15


def test_rk4_global_error_order():
    """Halving dt divides the RK4 error at a fixed time by about 16."""
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    t = 0.8
    exact = expm(-1j * H * t) @ psi0
    errs = []
    for n in (8, 16, 32):
        got = propagate("rk", lambda v: H @ v, psi0, t / n, n, 4)
        errs.append(np.linalg.norm(got - exact))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, errs


def test_sil_uncoupled_exact_phase():
    """The start vector meets few distinct energies: once the Krylov space
    holds all of them the step is exact."""
    O, E, psi0 = _uncoupled()
    dt = 0.3
    ndist = len(np.unique(np.round(E, 12)))
    got = sil_step(O.apply_literal, psi0, dt, ndist + 2)
    ref = np.exp(-1j * E * dt) * psi0
    assert np.linalg.norm(got - ref) < 1e-12


def test_sil_coupled_vs_dense_exponential():
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    dt = 0.05
    got = propagate("sil", O.apply_literal, psi0, dt, 10, 16)
    ref = expm(-1j * H * dt * 10) @ psi0
    assert np.linalg.norm(got - ref) < 1e-12


def test_lanczos_basis_orthonormal_and_projects():
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    V, T, b0 = lanczos_basis(O.apply_literal, psi0, 12)
    assert np.abs(V.conj().T @ V - np.eye(V.shape[1])).max() < 1e-13
    P = V.conj().T @ H @ V
    assert np.abs(P - T).max() < 1e-11
    assert abs(b0 - np.linalg.norm(psi0)) < 1e-15


def test_sil_stops_on_invariant_space():
    """A single eigenvector: the space is invariant after one vector."""
    O, E, psi0 = _uncoupled()
    v = np.zeros_like(psi0)
    v[3] = 2.0
    V, T, b0 = lanczos_basis(O.apply_literal, v, 8)
    assert V.shape[1] == 1 and abs(T[0, 0] - E[3]) < 1e-13 and b0 == 2.0
    got = sil_step(O.apply_literal, v, 0.4, 8)
    assert np.linalg.norm(got - np.exp(-1j * E[3] * 0.4) * v) < 1e-13


def test_bs_one_column_closed_form():
    """One column (two midpoint substeps, no extrapolation) multiplies an
    eigencomponent by 1 + X + X^2/2 + X^3/8, X = -i E dt (worked out by hand
    from the midpoint recurrence on y' = lambda y)."""
    from oracle.stepping import bs_step
    O, E, psi0 = _uncoupled()
    dt = 0.06
    got = bs_step(O.apply_literal, psi0, dt, 1)
    X = -1j * E * dt
    ref = (1 + X + X ** 2 / 2 + X ** 3 / 8) * psi0
    assert np.linalg.norm(got - ref) < 1e-14


@pytest.mark.parametrize("k,ratio", [(2, 16.0), (3, 64.0)])
def test_bs_global_order(k, ratio):
    """k columns over the substep counts 2, 4, .., 2k: global order 2k."""
    from oracle.stepping import bs_step
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    t = 1.0
    exact = expm(-1j * H * t) @ psi0
    errs = []
    for n in (10, 20):
        got = propagate("bs", lambda v: H @ v, psi0, t / n, n, k)
        errs.append(np.linalg.norm(got - exact))
    r = errs[0] / errs[1]
    assert 0.75 * ratio < r < 1.3 * ratio, errs


def test_bs_converged_vs_dense_exponential():
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    got = propagate("bs", O.apply_literal, psi0, 0.02, 10, 5)
    ref = expm(-1j * H * 0.2) @ psi0
    assert np.linalg.norm(got - ref) < 1e-12
