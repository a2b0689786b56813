"""Pins of the oracle's propagation pieces: Chebyshev against a dense
eigendecomposition, the uncoupled closed form, conservation laws, the
Chebyshev series itself and the displaced-Gaussian coefficients."""
import math

import numpy as np
import pytest

import sg_inputs
from oracle.action import Oracle, galerkin_masked_matrix
from oracle.hermite import gauss_hermite, hermite_functions
from oracle.propagate import (chebyshev_coefficients, chebyshev_step,
                              coherent_coefficients, exact_propagator,
                              propagate, spectral_bounds_dense,
                              spectral_bounds_sparse)


def test_chebyshev_series_is_exponential():
    """sum_k a_k (-i)^k T_k(x) = exp(-i R x) on [-1, 1]."""
    for R in [0.3, 1.0, 5.0, 20.0]:
        a = chebyshev_coefficients(R)
        x = np.linspace(-1, 1, 101)
        T0, T1 = np.ones_like(x), x
        s = a[0] * T0 + a[1] * (-1j) * T1
        for k in range(2, len(a)):
            T0, T1 = T1, 2 * x * T1 - T0
            s = s + a[k] * (-1j) ** k * T1
        assert np.abs(s - np.exp(-1j * R * x)).max() < 5e-15 * max(1, R)


def test_chebyshev_vs_eigh_config0():
    inst = sg_inputs.config0()
    O = Oracle(inst)
    H = galerkin_masked_matrix(inst).toarray()
    lo, hi = spectral_bounds_dense(H)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    apply = O.apply_literal
    psi, rec = propagate(apply, psi0, 0.1, 20, lo, hi, check_every=5)
    ref = exact_propagator(H, psi0, 20 * 0.1)
    assert np.linalg.norm(psi - ref) < 1e-12
    # energies recorded from phi_1 equal <psi|H|psi>
    e_ref = float(np.real(np.vdot(psi0, H @ psi0)))
    for _, nrm, e in rec:
        assert abs(nrm - 1.0) < 1e-13
        assert abs(e - e_ref) < 1e-12


def test_uncoupled_closed_form():
    inst = sg_inputs.small_instance(3, 3, seed=2)
    inst.c[:] = 0.0
    inst.k[:] = 0.0
    O = Oracle(inst)
    E = (inst.omega[None, :] * (O.S.compact + 0.5)).sum(axis=1)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    lo, hi = E.min(), E.max()
    pad = 0.05 * (hi - lo)
    psi, rec = propagate(O.apply_literal, psi0, 0.05, 40, lo - pad, hi + pad, check_every=8)
    ref = np.exp(-1j * E * 40 * 0.05) * psi0
    # the energy each step records (from phi_1) is the closed form
    # <psi|H|psi> = sum_n |c_n|^2 E_n of the uncoupled operator
    e_closed = float(np.sum(np.abs(psi0) ** 2 * E))
    assert len(rec) == 5
    for _, nrm, e in rec:
        assert abs(nrm - 1.0) < 1e-13
        assert abs(e - e_closed) < 1e-12
    assert np.linalg.norm(psi - ref) < 1e-12
    # autocorrelation C(t) = sum |c_n|^2 e^{-i E_n t}
    C = np.vdot(psi0, psi)
    assert abs(C - np.sum(np.abs(psi0) ** 2 * np.exp(-1j * E * 2.0))) < 1e-12


def test_norm_energy_conservation_long():
    inst = sg_inputs.small_instance(4, 3, seed=6)
    H = galerkin_masked_matrix(inst)
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    lo, hi = spectral_bounds_dense(H.toarray())
    psi, rec = propagate(lambda v: H @ v, psi0, 0.05, 500, lo, hi, check_every=50)
    e0 = rec[0][2]
    for _, nrm, e in rec:
        assert abs(nrm - 1.0) < 1e-12
        assert abs(e - e0) < 1e-11


def test_sparse_bounds_contain_spectrum():
    inst = sg_inputs.small_instance(3, 3, seed=7)
    H = galerkin_masked_matrix(inst)
    ev = np.linalg.eigvalsh(H.toarray())
    lo, hi = spectral_bounds_sparse(H)
    assert lo < ev[0] and hi > ev[-1]


def test_coherent_coefficients_are_projections():
    """c_n = <b_n | pi^{-1/4} exp(-(x-s)^2/2)> by a 60-point quadrature."""
    x, w, wt = gauss_hermite(60)
    for s in [-1.0, -0.3, 0.0, 0.7]:
        b = hermite_functions(12, x)
        f = math.pi ** -0.25 * np.exp(-0.5 * (x - s) ** 2)
        proj = (wt * f) @ b
        compact = np.arange(12)[:, None]
        c, nrm = coherent_coefficients(compact, np.array([s]))
        assert np.abs(c.real * nrm - proj).max() < 1e-13
        # the full (untruncated) series has unit norm
        assert nrm <= 1.0 + 1e-15 and nrm > 0.99
