"""GPU parity of the tabulated general potential (sg_set_potential) against
the oracle's Route 1 with the same function (FP64: 1e-12), and its use by
the propagators, the eigensolver and the refusals it comes with."""
import numpy as np
import pytest

import sg_inputs
from oracle.action import Oracle
from oracle.propagate import propagate, spectral_bounds_dense
from tests.gpu_util import empty, max_rel, rand_state, say, to_dev, to_host

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _sg():
    import paper_2111_13655_amd as sg
    return sg


def _problem(sg, inst, V):
    P = sg.Problem.from_instance(inst)
    sg.sg_set_potential(P.handle, V.at_points)
    return P


def _apply(P, psi):
    x, y = to_dev(psi), empty(P.n_cs)
    P.apply(x, y)
    return to_host(y)


@pytest.mark.parametrize("D,L", [(1, 0), (3, 0), (1, 6), (2, 4), (3, 3), (4, 2), (4, 4), (5, 3),
                                 (3, 6), (6, 4)])
def test_tabulated_apply_vs_route1(D, L):
    sg = _sg()
    inst = sg_inputs.small_instance(D, L, seed=60 + 10 * D + L)
    V = sg_inputs.general_potential(D, seed=D + L)
    say(f"tabulated apply D={D} L={L}")
    O = Oracle(inst, coupling=V)
    psi = rand_state(O.S.n_cs, 4)
    ref = O.apply_literal(psi)
    with _problem(sg, inst, V) as P:
        out = _apply(P, psi)
        info = sg.sg_problem_info(P.handle)
    assert max_rel(out, ref) < TOL
    assert info["sweep_bytes"] > 8.0 * info["grid_active"]


def test_tabulated_one_mode_potential_on_level0_modes():
    """V = f(Q_3) at D=4 L=3: most terms hold mode 3 at level 0, where the
    library integrates V out over the level-0 points."""
    sg = _sg()
    inst = sg_inputs.small_instance(4, 3, seed=5)

    class F:
        def __call__(self, Q):
            return np.cos(1.3 * Q[3]) + 0.4 * np.exp(-Q[3] ** 2)

        def at_points(self, P):
            return self([P[:, i] for i in range(4)])

    V = F()
    O = Oracle(inst, coupling=V)
    psi = rand_state(O.S.n_cs, 8)
    ref = O.apply_literal(psi)
    with _problem(sg, inst, V) as P:
        assert max_rel(_apply(P, psi), ref) < TOL


def test_polynomial_through_the_table_equals_the_closed_form_path():
    sg = _sg()
    inst = sg_inputs.small_instance(5, 4, seed=12)
    D, c, k = inst.D, inst.c, inst.k

    def poly(P):
        V = np.zeros(P.shape[0])
        for i in range(D):
            for j in range(i + 1, D):
                V += c[i, j] * P[:, i] ** 2 * P[:, j] ** 2 + k[i, j] * P[:, i] ** 2 * P[:, j]
        return V

    psi = rand_state(Oracle(inst).S.n_cs, 2)
    with sg.Problem.from_instance(inst) as P:
        closed = _apply(P, psi)
        sg.sg_set_potential(P.handle, poly)
        tab = _apply(P, psi)
        sg.sg_set_potential(P.handle, None)     # back to the closed-form couplings
        again = _apply(P, psi)
    assert max_rel(tab, closed) < TOL
    assert np.array_equal(again, closed)


def test_tabulated_chebyshev_vs_oracle():
    sg = _sg()
    inst = sg_inputs.small_instance(3, 4, seed=21)
    V = sg_inputs.general_potential(3, seed=4)
    O = Oracle(inst, coupling=V)
    n = O.S.n_cs
    H = np.stack([O.apply_literal(np.eye(n)[:, j].astype(complex)) for j in range(n)], axis=1)
    lo, hi = spectral_bounds_dense(H)
    psi0 = rand_state(n, 6)
    ref, _ = propagate(lambda v: H @ v, psi0, 0.05, 30, lo, hi)
    say("tabulated chebyshev D=3 L=4, 30 steps")
    with _problem(sg, inst, V) as P:
        x = to_dev(psi0)
        status, st, _, _ = sg.sg_propagate_chebyshev(P.handle, x, 0.05, 30, lo, hi, tol=1e-8)
        out = to_host(x)
    assert status == 0
    assert max_rel(out, ref) < 1e-11
    assert st["max_norm_drift"] < 1e-12


def test_tabulated_eigenpairs_vs_dense():
    sg = _sg()
    inst = sg_inputs.small_instance(3, 4, seed=23)
    V = sg_inputs.general_potential(3, seed=5)
    O = Oracle(inst, coupling=V)
    n = O.S.n_cs
    H = np.stack([O.apply_literal(np.eye(n)[:, j].astype(complex)) for j in range(n)], axis=1)
    ref = np.linalg.eigvalsh(0.5 * (H + H.conj().T))[:4]
    with _problem(sg, inst, V) as P:
        status, vals, res, _ = sg.sg_eigensolve(P.handle, 4, tol=1e-10)
    assert status == 0
    assert np.abs(np.asarray(vals) - ref).max() < 1e-9 * max(1.0, np.abs(ref).max())


def test_tabulated_refusals():
    sg = _sg()
    inst = sg_inputs.small_instance(3, 3, seed=1)
    V = sg_inputs.general_potential(3, seed=1)
    with _problem(sg, inst, V) as P:
        x, y = to_dev(rand_state(P.n_cs, 1)), empty(P.n_cs)
        with pytest.raises(sg.SgError):
            P.apply(x, y, sg.SG_MIXED)
        with pytest.raises(sg.SgError):
            sg.sg_set_operator_form(P.handle, True)

        def bad(Q):
            out = V.at_points(Q)
            out[0] = np.nan
            return out
        with pytest.raises(sg.SgError):
            sg.sg_set_potential(P.handle, bad)
        # the previous tables stay in force after a refused call
        O = Oracle(inst, coupling=V)
        psi = rand_state(P.n_cs, 3)
        assert max_rel(_apply(P, psi), O.apply_literal(psi)) < TOL

        def boom(Q):
            raise RuntimeError("from the potential")
        with pytest.raises(RuntimeError):
            sg.sg_set_potential(P.handle, boom)


def test_tabulated_bench_workload_full_vector():
    """The bench's workload (D=8, L=6, its potential): the whole output
    against Route 1."""
    sg = _sg()
    inst, V = sg_inputs.tabulated_d8_l6()
    O = Oracle(inst, coupling=V)
    psi = rand_state(O.S.n_cs, 9)
    say("tabulated D=8 L=6 full vector")
    ref = O.apply_literal(psi)
    with _problem(sg, inst, V) as P:
        assert max_rel(_apply(P, psi), ref) < TOL


@pytest.mark.parametrize("method,order", [("taylor", 12), ("sil", 10), ("rk", 4), ("bs", 3)])
def test_tabulated_other_propagators_vs_oracle(method, order):
    """The other propagators on a tabulated potential (they apply H through
    the same sweep) against the oracle's steppers on Route 1."""
    from oracle import stepping
    sg = _sg()
    inst = sg_inputs.small_instance(3, 3, seed=31)
    V = sg_inputs.general_potential(3, seed=31)
    O = Oracle(inst, coupling=V)
    psi0 = rand_state(O.S.n_cs, 12)
    ref = stepping.propagate(method, O.apply_literal, psi0, 0.02, 5, order)
    codes = {"taylor": "SG_PROP_TAYLOR", "sil": "SG_PROP_SIL", "rk": "SG_PROP_RK", "bs": "SG_PROP_BS"}
    with _problem(sg, inst, V) as P:
        x = to_dev(psi0)
        status, _, _, _ = sg.sg_propagate(P.handle, x, 0.02, 5, getattr(sg, codes[method]), order)
        out = to_host(x)
    assert status == 0
    assert max_rel(out, ref) < 1e-11


def test_tabulated_in_a_batch_is_bitwise_its_own_propagation():
    """A batch holding a tabulated problem and a polynomial one: each
    instance's result is bitwise the one it gets propagated alone (the batch
    runs the tabulated instantiation of the sweep for both)."""
    sg = _sg()
    inst_t = sg_inputs.small_instance(4, 4, seed=41)
    V = sg_inputs.general_potential(4, seed=41)
    inst_p = sg_inputs.small_instance(5, 3, seed=42)
    with _problem(sg, inst_t, V) as PT, sg.Problem.from_instance(inst_p) as PP:
        probs = [PT, PP]
        psi0 = [rand_state(P.n_cs, 50 + i) for i, P in enumerate(probs)]
        bounds = [sg.sg_spectral_bounds(P.handle, 40) for P in probs]
        alone = []
        for P, x0, (lo, hi) in zip(probs, psi0, bounds):
            x = to_dev(x0)
            st, _, _, _ = sg.sg_propagate_chebyshev(P.handle, x, 0.05, 6, lo, hi, tol=1e-6)
            assert st == 0
            alone.append(to_host(x))
        b = sg.sg_batch_create([P.handle for P in probs])
        xs = [to_dev(x0) for x0 in psi0]
        status, _ = sg.sg_batch_propagate(b, xs, [0.05, 0.05], 6, [lo for lo, _ in bounds],
                                          [hi for _, hi in bounds], tol=1e-6)
        out = [to_host(x) for x in xs]
        # a potential changed after the batch was created: the batch refuses
        sg.sg_set_potential(PP.handle, sg_inputs.general_potential(5).at_points)
        with pytest.raises(sg.SgError):
            sg.sg_batch_propagate(b, xs, [0.05, 0.05], 1, [lo for lo, _ in bounds],
                                  [hi for _, hi in bounds], tol=1e-6)
        sg.sg_batch_free(b)
    assert status == 0
    for a_, o in zip(alone, out):
        assert np.array_equal(a_, o)
