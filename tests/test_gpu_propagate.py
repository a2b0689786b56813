"""GPU Chebyshev propagation against the oracle (FP64)."""
import math

import numpy as np
import pytest

import sg_inputs
from oracle.action import Oracle, galerkin_masked_matrix
from oracle.propagate import (coherent_coefficients, exact_propagator, propagate,
                              spectral_bounds_dense, spectral_bounds_sparse)
from tests.gpu_util import empty, rand_state, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2111_13655_amd as sg
    return sg


def test_initial_state_matches_oracle():
    sg = _sg()
    inst = sg_inputs.config1()
    with sg.Problem.from_instance(inst) as P:
        psi = empty(P.n_cs)
        cap = sg.sg_init_gaussian(P.handle, inst.shift, psi)
        got = to_host(psi)
        comp = sg.sg_basis_indices(P.handle)
    ref, nrm = coherent_coefficients(comp, inst.shift)
    assert abs(cap - nrm) < 1e-14
    # same closed form, different rounding order of the products
    assert np.abs(got - ref).max() < 1e-14 * np.abs(ref).max()


def test_propagate_config0_vs_oracle_and_exact():
    """(D, L) = (2, 4): 100 steps of dt = 0.1, same bounds on both sides."""
    sg = _sg()
    inst = sg_inputs.config0()
    say("propagate config0")
    H = galerkin_masked_matrix(inst)
    lo, hi = spectral_bounds_dense(H.toarray())
    O = Oracle(inst)
    psi0, _ = coherent_coefficients(O.S.compact, inst.shift)
    ref, rec = propagate(O.apply_literal, psi0, 0.1, 100, lo, hi, check_every=10)
    exact = exact_propagator(H.toarray(), psi0, 10.0)
    with sg.Problem.from_instance(inst) as P:
        x = to_dev(psi0)
        status, st, nt, et = sg.sg_propagate_chebyshev(P.handle, x, 0.1, 100, lo, hi,
                                                       tol=1e-9, check_every=10)
        out = to_host(x)
    assert status == sg.SG_OK
    assert np.linalg.norm(out - ref) < 1e-11
    assert np.linalg.norm(out - exact) < 1e-11
    assert st["steps_done"] == 100
    assert st["max_norm_drift"] < 1e-12
    # energies at the checks match the oracle's
    for (s, n_o, e_o), e_g in zip(rec, et):
        assert abs(e_g - e_o) < 1e-11


def test_propagate_config1_drift_and_parity():
    """(D, L) = (6, 6): the benchmark trajectory, 1000 steps of dt = 0.05,
    norm and energy checked every 100 steps; final state against the oracle's
    masked-Galerkin propagation with the same bounds."""
    sg = _sg()
    inst = sg_inputs.config1()
    say("propagate config1 (1000 steps)")
    H = galerkin_masked_matrix(inst)
    lo, hi = spectral_bounds_sparse(H)
    comp = None
    with sg.Problem.from_instance(inst) as P:
        comp = sg.sg_basis_indices(P.handle)
        psi0, _ = coherent_coefficients(comp, inst.shift)
        x = to_dev(psi0)
        status, st, nt, et = sg.sg_propagate_chebyshev(P.handle, x, 0.05, 1000, lo, hi,
                                                       tol=1e-9, check_every=100)
        out = to_host(x)
    assert status == sg.SG_OK
    ref, _ = propagate(lambda v: H @ v, psi0, 0.05, 1000, lo, hi)
    dist = np.linalg.norm(out - ref)
    say(f"config1 1000 steps: norm drift {st['max_norm_drift']:.3e}, energy drift "
        f"{st['max_energy_drift']:.3e}, |gpu - oracle| = {dist:.3e}")
    # measured on two boxes: norm drift 0.8e-13 and 1.0e-13, energy drift
    # 4.6e-14, distance from the oracle 1.3e-13
    assert st["max_norm_drift"] < 5e-13
    assert st["max_energy_drift"] < 5e-13
    assert dist < 1e-12


def test_library_bounds_contain_spectrum():
    sg = _sg()
    for inst in (sg_inputs.config0(), sg_inputs.config1()):
        H = galerkin_masked_matrix(inst)
        ev_lo, ev_hi = spectral_bounds_sparse(H, pad=0.0)
        with sg.Problem.from_instance(inst) as P:
            lo, hi = sg.sg_spectral_bounds(P.handle, 40)
        assert lo < ev_lo and hi > ev_hi
        assert hi - lo < 2.0 * (ev_hi - ev_lo)


def test_propagate_with_library_bounds_matches():
    sg = _sg()
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    with sg.Problem.from_instance(inst) as P:
        comp = sg.sg_basis_indices(P.handle)
        psi0, _ = coherent_coefficients(comp, inst.shift)
        x = to_dev(psi0)
        status, st, _, _ = sg.sg_propagate_chebyshev(P.handle, x, 0.1, 50)
        out = to_host(x)
    assert status == sg.SG_OK
    assert np.linalg.norm(out - exact_propagator(H, psi0, 5.0)) < 1e-11


def test_tight_bounds_raise_etol():
    """Bounds that miss most of the spectrum make the series diverge; the norm
    check must stop the call with SG_ETOL (the condition is set from the host,
    every kernel still runs normally)."""
    sg = _sg()
    inst = sg_inputs.config0()
    H = galerkin_masked_matrix(inst).toarray()
    ev = np.linalg.eigvalsh(H)
    with sg.Problem.from_instance(inst) as P:
        psi0 = rand_state(P.n_cs, 3)
        x = to_dev(psi0)
        status, st, nt, _ = sg.sg_propagate_chebyshev(
            P.handle, x, 0.1, 50, ev[0], ev[0] + 0.2 * (ev[-1] - ev[0]), tol=1e-6,
            check_every=1)
    assert status == sg.SG_ETOL
    assert st["steps_done"] < 50


def test_propagate_bitwise_reproducible():
    sg = _sg()
    inst = sg_inputs.config1()
    outs = []
    with sg.Problem.from_instance(inst) as P:
        lo, hi = sg.sg_spectral_bounds(P.handle, 40)
        for _ in range(2):
            psi = empty(P.n_cs)
            sg.sg_init_gaussian(P.handle, inst.shift, psi)
            status, _, _, _ = sg.sg_propagate_chebyshev(P.handle, psi, 0.05, 20, lo, hi,
                                                        check_every=5)
            assert status == sg.SG_OK
            outs.append(to_host(psi))
    assert np.array_equal(outs[0], outs[1])
