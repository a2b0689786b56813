"""Pins of the two-state (vibronic) oracle: the literal per-term route against
the masked-Galerkin closed form and the full direct product, the uncoupled
closed form and its spectrum, Hermiticity, the symmetry that exchanges the
two states, the reduction to the one-state oracle, and the matrix-free
closed form against the assembled one."""
import numpy as np
import pytest

import sg_inputs
from oracle.action import Oracle
from oracle.vibronic import VibronicOracle, brute_force_masked, masked_apply, masked_matrix


def _rand(shape, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def _full_params(inst, seed):
    """every parameter non-zero (kappa and lambda on all modes)"""
    rng = np.random.default_rng(seed)
    inst.kappa = rng.uniform(-0.2, 0.2, size=inst.kappa.shape)
    inst.lam = rng.uniform(-0.3, 0.3, size=inst.lam.shape)
    return inst


@pytest.mark.parametrize("D,L", [(1, 3), (2, 3), (3, 2), (2, 4)])
def test_route1_equals_route2_equals_brute_force(D, L):
    inst = _full_params(sg_inputs.vibronic_small(D, L, seed=10 * D + L), 1)
    O = VibronicOracle(inst)
    n = O.S.n_cs
    H2 = masked_matrix(inst).toarray()
    HB = brute_force_masked(inst, O.S.compact)
    assert np.abs(H2 - HB).max() < 1e-13 * np.abs(HB).max()
    psi = _rand((2, n), 3)
    r1 = O.apply_literal(psi).reshape(-1)
    r2 = H2 @ psi.reshape(-1)
    assert np.linalg.norm(r1 - r2) / np.linalg.norm(r2) < 1e-13
    # the unmasked product differs (from two modes on, where the joint level
    # can exceed L): the mask is what the Smolyak sum does
    if D > 1:
        HU = brute_force_masked(inst, O.S.compact, mask=False)
        assert np.abs(HU - HB).max() > 1e-3


def test_uncoupled_is_two_shifted_harmonic_spectra():
    inst = sg_inputs.vibronic_small(3, 3, seed=4, quartic=False)
    inst.kappa[:] = 0.0
    inst.lam[:] = 0.0
    O = VibronicOracle(inst)
    N = O.S.compact
    h0 = (inst.omega[None, :] * (N + 0.5)).sum(axis=1)
    psi = _rand((2, O.S.n_cs), 5)
    out = O.apply_literal(psi)
    for s in range(2):
        assert np.abs(out[s] - (h0 + inst.E[s]) * psi[s]).max() < 1e-12 * np.abs(out).max()
    ev = np.linalg.eigvalsh(masked_matrix(inst).toarray())
    want = np.sort(np.concatenate([h0 + inst.E[0], h0 + inst.E[1]]))
    assert np.abs(ev - want).max() < 1e-12


@pytest.mark.parametrize("D,L", [(2, 4), (3, 3)])
def test_hermiticity(D, L):
    inst = _full_params(sg_inputs.vibronic_small(D, L, seed=7), 2)
    O = VibronicOracle(inst)
    phi, psi = _rand((2, O.S.n_cs), 8), _rand((2, O.S.n_cs), 9)
    lhs = np.vdot(phi.reshape(-1), O.apply_literal(psi).reshape(-1))
    rhs = np.conj(np.vdot(psi.reshape(-1), O.apply_literal(phi).reshape(-1)))
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_state_exchange_symmetry():
    """Exchanging the states' parameters exchanges the blocks: with P the
    state swap, H'(swapped parameters) = P H P."""
    inst = _full_params(sg_inputs.vibronic_small(3, 3, seed=11), 3)
    import copy
    sw = copy.deepcopy(inst)
    sw.E = inst.E[::-1].copy()
    sw.kappa = inst.kappa[::-1].copy()
    sw.c2 = inst.c2[::-1].copy()
    O, Os = VibronicOracle(inst), VibronicOracle(sw)
    psi = _rand((2, O.S.n_cs), 12)
    a = O.apply_literal(psi)
    b = Os.apply_literal(psi[::-1])
    assert np.abs(a - b[::-1]).max() < 1e-13 * np.abs(a).max()


def test_blocks_reduce_to_the_one_state_oracle():
    """With no interstate coupling, E = 0 and no linear terms, each diagonal
    block is the one-state operator with c = c2[s] and k = 0 (computed by the
    separately pinned one-state oracle)."""
    inst = sg_inputs.vibronic_small(3, 4, seed=13)
    inst.kappa[:] = 0.0
    inst.lam[:] = 0.0
    inst.E[:] = 0.0
    O = VibronicOracle(inst)
    psi = _rand((2, O.S.n_cs), 14)
    out = O.apply_literal(psi)
    for s in range(2):
        one = sg_inputs.small_instance(3, 4, seed=1)
        one.omega = inst.omega.copy()
        one.c = inst.c2[s].copy()
        one.k = np.zeros_like(one.k)
        ref = Oracle(one).apply_literal(psi[s])
        assert np.abs(out[s] - ref).max() < 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("D,L,seed", [(2, 4, 1), (4, 3, 2), (5, 3, 3)])
def test_masked_apply_matches_matrix(D, L, seed):
    inst = _full_params(sg_inputs.vibronic_small(D, L, seed=seed), seed)
    O = VibronicOracle(inst)
    psi = _rand((2, O.S.n_cs), seed)
    ref = (masked_matrix(inst) @ psi.reshape(-1)).reshape(2, -1)
    got = masked_apply(inst, psi, O.S.compact)
    assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()
    r1 = O.apply_literal(psi)
    assert np.linalg.norm(got - r1) / np.linalg.norm(r1) < 1e-13
