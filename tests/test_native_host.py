"""CPU tests of the native library: it loads, exports every symbol the C ABI
header declares, and its host-side term compiler (integer work: term set,
D_l, compact basis ordering, M^B) matches the oracle bit for bit."""
import os
import re

import numpy as np
import pytest

import sg_inputs
from oracle.smolyak import build_structure, count_sizes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _sg():
    import paper_2111_13655_amd as sg
    sg.lib()
    return sg


def test_library_exports_every_declared_symbol():
    sg = _sg()
    decl = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            decl |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sg_\w+)\s*\(", text, re.M))
    assert "sg_apply_H" in decl and "sg_build_terms" in decl
    L = sg.lib()
    for name in sorted(decl):
        assert hasattr(L, name), name


def test_count_sizes_matches_oracle_and_table1():
    sg = _sg()
    for D, L, a, b in [(12, 6, 1, 1), (120, 6, 1, 1), (6, 6, 1, 2), (12, 6, 1, 2),
                       (20, 6, 1, 2), (10, 7, 1, 2), (3, 5, 2, 3)]:
        assert sg.sg_count_sizes(D, L, a, b) == count_sizes(D, L, a, b)
    assert sg.sg_count_sizes(120, 6, 1, 1)[1:] == (289465762509, 4925156775)


@pytest.mark.parametrize("D,L,nb", [(2, 3, (1, 1)), (2, 4, (1, 2)), (3, 3, (1, 2)),
                                    (4, 2, (1, 2)), (6, 6, (1, 2)), (5, 4, (2, 1)),
                                    (1, 6, (1, 2)), (3, 0, (1, 2))])
def test_host_term_compiler_matches_oracle(D, L, nb):
    sg = _sg()
    inst = sg_inputs.small_instance(D, L, seed=1)
    nq = (nb[0] + 1, nb[1])
    h = sg.sg_build_terms_host(D, L, inst.omega, inst.c, inst.k, nb, nq)
    try:
        S = build_structure(D, L, *nb)
        lev, co = sg.sg_term_levels(h)
        assert [tuple(r) for r in lev.tolist()] == S.terms
        assert co.tolist() == S.coeffs.tolist()
        assert np.array_equal(sg.sg_basis_indices(h), S.compact)
        assert np.array_equal(sg.sg_mapping_table(h), S.MB)
        info = sg.sg_problem_info(h)
        assert (info["n_terms"], info["n_s"], info["n_cs"]) == (S.n_terms, S.n_s, S.n_cs)
    finally:
        sg.sg_free(h)


def test_table2_through_the_library(golden_dir):
    sg = _sg()
    h = sg.sg_build_terms_host(2, 3, [1.0, 1.0], np.zeros((2, 2)), None, (1, 1), (1, 1))
    try:
        mb = (sg.sg_mapping_table(h) + 1).tolist()
        assert mb == [1, 5, 8, 1, 5, 8, 10, 1, 5, 2, 6, 1, 5, 8, 2, 6, 9, 1, 2, 3, 1, 5, 2, 6,
                      3, 7, 1, 2, 3, 4]
    finally:
        sg.sg_free(h)


def test_config_sizes():
    sg = _sg()
    # sizes of the two headline workloads (D, L) = (6, 6) and (12, 6)
    for D, L, n_terms, n_cs, n_s in [(6, 6, 923, 8989, 93535), (12, 6, 18564, 369305, 4195284),
                                     (2, 4, 9, 41, 129)]:
        inst = sg_inputs.small_instance(D, L, seed=0)
        h = sg.sg_build_terms_host(D, L, inst.omega, inst.c, inst.k)
        try:
            info = sg.sg_problem_info(h)
            assert (info["n_terms"], info["n_cs"], info["n_s"]) == (n_terms, n_cs, n_s)
            assert info["max_term_grid"] <= 4096
        finally:
            sg.sg_free(h)


def test_operator_form_selection_host_only():
    import paper_2111_13655_amd as sg
    inst = sg_inputs.config0()
    P = sg.Problem.from_instance(inst, host_only=True)
    try:
        info = sg.sg_problem_info(P.handle)
        assert info["fp64_split"] == 1          # nq(l) = 2l+2 > nb(l) = 2l+1
        assert info["flops_fp64"] == info["flops_mixed"]
        assert info["sweep_flops_fp64"] < info["flops_fp64"]
        sg.sg_set_operator_form(P.handle, True)
        info2 = sg.sg_problem_info(P.handle)
        assert info2["fp64_split"] == 0
        assert info2["flops_fp64"] > info["flops_fp64"]   # kinetic contractions
        with pytest.raises(sg.SgError):
            sg.sg_set_operator_form(P.handle, 2)
    finally:
        P.close()
    # nq = nb at some level: the split is not exact, SG_FP64 keeps the grid form
    inst2 = sg_inputs.small_instance(2, 2, seed=5, nb=(1, 2), nq=(1, 2))
    P2 = sg.Problem.from_instance(inst2, host_only=True)
    try:
        assert sg.sg_problem_info(P2.handle)["fp64_split"] == 0
    finally:
        P2.close()


def test_invalid_descriptions_rejected():
    sg = _sg()
    with pytest.raises(sg.SgError) as e:
        sg.sg_build_terms_host(0, 3, [], np.zeros((0, 0)))
    assert e.value.status == sg.SG_EINVAL
    with pytest.raises(sg.SgError):
        sg.sg_build_terms_host(2, 3, [1.0, -1.0], np.zeros((2, 2)))
    with pytest.raises(sg.SgError):  # nq < nb
        sg.sg_build_terms_host(2, 3, [1.0, 1.0], np.zeros((2, 2)), None, (2, 2), (1, 1))
    with pytest.raises(sg.SgError):  # grids beyond 16 points
        sg.sg_build_terms_host(2, 9, [1.0, 1.0], np.zeros((2, 2)))
    with pytest.raises(sg.SgError):
        sg.sg_build_terms_host(2, 3, [1.0, float("nan")], np.zeros((2, 2)))


def test_schedule_setter_host_only():
    """The term-to-workgroup schedule knob: any non-negative grid size is a
    valid schedule; a negative one is rejected."""
    import paper_2111_13655_amd as sg
    P = sg.Problem.from_instance(sg_inputs.config0(), host_only=True)
    try:
        for g in (0, 64, 1 << 20):
            for spread in (1, 2, 4):
                sg.sg_set_schedule(P.handle, g, spread)
        for bad in ((-1, 1), (0, 0), (0, 5)):
            with pytest.raises(sg.SgError) as e:
                sg.sg_set_schedule(P.handle, *bad)
            assert e.value.status == sg.SG_EINVAL
    finally:
        P.close()


def test_propagate_rejects_bad_arguments_host_only():
    """sg_propagate validates method, order, dt and precision before it
    touches the device; a host-only handle is refused for valid ones."""
    import ctypes
    import paper_2111_13655_amd as sg
    P = sg.Problem.from_instance(sg_inputs.config0(), host_only=True)
    dummy = ctypes.c_void_p(16)
    try:
        L = sg.lib()
        for method, order, dt, prec in [(0, 4, 0.1, 0), (5, 4, 0.1, 0), (1, 0, 0.1, 0),
                                        (1, 41, 0.1, 0), (2, 5, 0.1, 0), (3, 65, 0.1, 0),
                                        (4, 0, 0.1, 0), (4, 9, 0.1, 0),
                                        (2, 4, 0.0, 0), (2, 4, float("nan"), 0), (2, 4, 0.1, 7)]:
            st = L.sg_propagate(P.handle, dummy, dt, 1, method, order, 0.0, prec, 0,
                                None, None, None, None)
            assert st == sg.SG_EINVAL, (method, order, dt, prec)
        for method, order in [(1, 1), (1, 40), (2, 1), (2, 4), (3, 1), (3, 64), (4, 1), (4, 8)]:
            st = L.sg_propagate(P.handle, dummy, 0.1, 1, method, order, 0.0, 0, 0,
                                None, None, None, None)
            assert st == sg.SG_EINVAL   # no device tables
    finally:
        P.close()


def test_batch_binding_rejects_bad_state_lists_before_any_launch(monkeypatch):
    """The binding checks the number of states against the batch's size (read
    from the library) before it marshals anything: a short or long list never
    reaches the kernels.  The batch itself needs a device, so its size query
    is replaced here."""
    sg = _sg()
    monkeypatch.setattr(sg, "sg_batch_size", lambda b: (2, [41, 41]))
    called = []
    monkeypatch.setattr(sg, "lib", lambda: called.append(1))
    with pytest.raises(ValueError):
        sg.sg_batch_propagate(None, [], [], 1)
    with pytest.raises(ValueError):
        sg.sg_batch_propagate(None, [object()] * 3, [0.1] * 3, 1)
    assert called == []


def test_batch_abi_refuses_null_batch():
    sg = _sg()
    assert sg.lib().sg_batch_propagate(None, None, 0, None, 1, None, None, 0.0, 0, 0, 0,
                                       None, None) == sg.SG_EINVAL
