"""Batched propagation and the continuous-batching server (GPU).

Both advance many instances with shared launches; every instance must come
out bitwise equal to the same instance propagated alone (same per-term code,
fixed-order reductions), whatever the mix.  The alone runs are themselves
pinned to the oracle by the propagation tests; here one (7, 7) instance, whose
largest term grids (16384 points) run from global scratch instead of LDS, is
also pinned to the oracle's masked-Galerkin rows.
"""
import time

import numpy as np
import pytest

import sg_inputs
from oracle.action import galerkin_rows
from oracle.propagate import coherent_coefficients
from oracle.smolyak import CompactRanker
from tests.gpu_util import empty, rand_state, say, to_dev, to_host

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2111_13655_amd as sg
    return sg


def _mix():
    """A mix of sizes and size maps: several (D, L) and one general map."""
    out = []
    for i, (D, L) in enumerate([(2, 4), (3, 5), (4, 4), (6, 6), (5, 7), (2, 7)]):
        out.append(sg_inputs.small_instance(D, L, seed=500 + i, with_k=True))
    out.append(sg_inputs.small_instance(3, 3, seed=520, with_k=True, nb=(2, 1), nq=(3, 2)))
    return out


def _alone(sg, inst, dt, nsteps, lo, hi, prec, check_every=0):
    # norm-drift gate: FP64 rounding, or the mixed path's 1e-6 bar
    tol = 1e-8 if prec == sg.SG_FP64 else 1e-6
    with sg.Problem.from_instance(inst) as P:
        psi = empty(P.n_cs)
        sg.sg_init_gaussian(P.handle, inst.shift, psi)
        status, st, _, _ = sg.sg_propagate_chebyshev(P.handle, psi, dt, nsteps, lo, hi, tol=tol,
                                                     precision=prec, check_every=check_every)
        assert status == sg.SG_OK
        return to_host(psi), st


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_bitwise_equal_to_alone(use_graph):
    sg = _sg()
    insts = _mix()
    say(f"batch vs alone, graph={use_graph}")
    probs = [sg.Problem.from_instance(i) for i in insts]
    try:
        bounds = [sg.sg_spectral_bounds(P.handle, 40) for P in probs]
        # different dt give different series lengths inside one batch
        dts = [0.05 * (1 + (i % 3)) for i in range(len(insts))]
        psis = []
        for P, inst in zip(probs, insts):
            x = empty(P.n_cs)
            sg.sg_init_gaussian(P.handle, inst.shift, x)
            psis.append(x)
        b = sg.sg_batch_create([P.handle for P in probs])
        try:
            status, stats = sg.sg_batch_propagate(
                b, psis, dts, 7, [lo for lo, _ in bounds], [hi for _, hi in bounds],
                check_every=3, use_graph=use_graph)
        finally:
            sg.sg_batch_free(b)
        assert status == sg.SG_OK
        outs = [to_host(x) for x in psis]
    finally:
        for P in probs:
            P.close()
    for i, inst in enumerate(insts):
        ref, st = _alone(sg, inst, dts[i], 7, bounds[i][0], bounds[i][1], sg.SG_FP64,
                         check_every=3)
        assert np.array_equal(outs[i], ref), i
        assert stats[i]["steps_done"] == 7
        assert stats[i]["cheb_terms"] == st["cheb_terms"]
        assert abs(stats[i]["norm_last"] - 1.0) < 1e-12


def test_batch_schedule_tuner_keeps_results_bitwise():
    """The batch schedule autotuner over the union of the instances' terms:
    every candidate schedule gives bitwise the same apply (the tuner checks
    that itself), the chosen one is a candidate, and a propagation after the
    tuning is still bitwise the alone result."""
    sg = _sg()
    insts = _mix()[:5]
    say("batch schedule tuner")
    probs = [sg.Problem.from_instance(i) for i in insts]
    try:
        bounds = [sg.sg_spectral_bounds(P.handle, 40) for P in probs]
        psis = []
        for P, inst in zip(probs, insts):
            x = empty(P.n_cs)
            sg.sg_init_gaussian(P.handle, inst.shift, x)
            psis.append(x)
        b = sg.sg_batch_create([P.handle for P in probs])
        try:
            g, ms = sg.sg_batch_tune_schedule(b, psis, sg.SG_FP64, reps=2)
            max_grid = max(P.info["max_term_grid"] for P in probs)
            assert g == 0 or (g >= 256 and g <= max_grid and (g & (g - 1)) == 0)
            assert ms > 0.0
            status, _ = sg.sg_batch_propagate(
                b, psis, [0.05] * len(insts), 4, [lo for lo, _ in bounds],
                [hi for _, hi in bounds])
        finally:
            sg.sg_batch_free(b)
        assert status == sg.SG_OK
        outs = [to_host(x) for x in psis]
    finally:
        for P in probs:
            P.close()
    for i, inst in enumerate(insts):
        ref, _ = _alone(sg, inst, 0.05, 4, bounds[i][0], bounds[i][1], sg.SG_FP64)
        assert np.array_equal(outs[i], ref), i


def test_batch_mixed_precision_bitwise_equal_to_alone():
    sg = _sg()
    insts = _mix()[:5]
    say("batch mixed vs alone")
    probs = [sg.Problem.from_instance(i) for i in insts]
    try:
        bounds = [sg.sg_spectral_bounds(P.handle, 40) for P in probs]
        psis = []
        for P, inst in zip(probs, insts):
            x = empty(P.n_cs)
            sg.sg_init_gaussian(P.handle, inst.shift, x)
            psis.append(x)
        b = sg.sg_batch_create([P.handle for P in probs])
        try:
            status, _ = sg.sg_batch_propagate(
                b, psis, [0.05] * len(insts), 5, [lo for lo, _ in bounds],
                [hi for _, hi in bounds], precision=sg.SG_MIXED)
        finally:
            sg.sg_batch_free(b)
        assert status == sg.SG_OK
        outs = [to_host(x) for x in psis]
    finally:
        for P in probs:
            P.close()
    for i, inst in enumerate(insts):
        ref, _ = _alone(sg, inst, 0.05, 5, bounds[i][0], bounds[i][1], sg.SG_MIXED)
        assert np.array_equal(outs[i], ref), i


def test_batch_rejects_bad_arguments():
    sg = _sg()
    inst = sg_inputs.config0()
    with sg.Problem.from_instance(inst) as P:
        with pytest.raises(sg.SgError) as e:
            sg.sg_batch_create([P.handle, P.handle])
        assert e.value.status == sg.SG_EINVAL
        with pytest.raises(sg.SgError) as e:
            sg.sg_batch_create([])
        assert e.value.status == sg.SG_EINVAL
        b = sg.sg_batch_create([P.handle])
        try:
            x = empty(P.n_cs)
            sg.sg_init_gaussian(P.handle, inst.shift, x)
            with pytest.raises(sg.SgError) as e:
                sg.sg_batch_propagate(b, [x], [-1.0], 1)
            assert e.value.status == sg.SG_EINVAL
            # a state list of the wrong length, or a state of the wrong size,
            # is refused before anything is launched
            with pytest.raises(ValueError):
                sg.sg_batch_propagate(b, [x, x], [0.1, 0.1], 1)
            with pytest.raises(ValueError):
                sg.sg_batch_propagate(b, [empty(P.n_cs - 1)], [0.1], 1)
            assert sg.sg_batch_size(b) == (1, [P.n_cs])
            # the C ABI itself refuses a count that differs from the batch's
            import ctypes
            ptrs = (ctypes.c_void_p * 2)(x.data_ptr(), x.data_ptr())
            dts = (ctypes.c_double * 2)(0.1, 0.1)
            st = sg.lib().sg_batch_propagate(b, ptrs, 2, dts, 1, None, None, 0.0, sg.SG_FP64,
                                             0, 0, None, None)
            assert st == sg.SG_EINVAL
        finally:
            sg.sg_batch_free(b)


def test_scratch_path_instance_apply_sampled_rows():
    """(D, L) = (7, 7): the all-ones term has 4^7 grid points, whose two
    buffers exceed a compute unit's LDS and live in global scratch."""
    sg = _sg()
    inst = sg_inputs.small_instance(7, 7, seed=77, with_k=True)
    say("apply (7,7) scratch path, sampled rows")
    with sg.Problem.from_instance(inst) as P:
        assert P.info["max_term_grid"] == 4 ** 7
        n = P.n_cs
        psi = rand_state(n, 11)
        x, y = to_dev(psi), empty(n)
        P.apply(x, y, sg.SG_FP64)
        Hpsi = to_host(y)
        comp = sg.sg_basis_indices(P.handle)
    rk = CompactRanker(inst.D, inst.L, 1, 2)
    rng = np.random.default_rng(1)
    # rows reached by the largest terms: all seven modes at level one
    ones = np.where((comp[:, :7] > 0).all(axis=1))[0]
    rows = np.concatenate([[0, n - 1], ones[:40], rng.choice(n, 100, replace=False)])
    scale = np.abs(Hpsi).max()
    for r, (cols, vals) in zip(rows, galerkin_rows(inst, rk, comp[rows])):
        assert abs(Hpsi[r] - np.dot(vals, psi[cols])) < 1e-12 * scale, r


def _serve_requests():
    rng = np.random.default_rng(900)
    reqs = []
    for i, (D, L) in enumerate([(2, 4), (4, 4), (6, 6), (3, 5), (5, 7), (2, 7), (4, 5)]):
        inst = sg_inputs.draw_instance(rng, D, L, with_k=True)
        reqs.append((inst, 0.05 * (1 + i % 2), int(rng.integers(3, 12))))
    return reqs


def _wait(sg, srv, ticket, n_cs, limit=60.0):
    t0 = time.time()
    while True:
        r = sg.sg_serve_poll(srv, ticket, n_cs)
        if r is not None:
            return r
        assert time.time() - t0 < limit, "request did not finish"
        time.sleep(0.002)


def _submit(sg, srv, inst, dt, nsteps):
    return sg.sg_serve_submit(srv, inst.D, inst.L, inst.omega, inst.c, inst.k, inst.shift,
                              dt, nsteps)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_serve_alone_equals_mix(prec):
    """Each request alone on a server, then all of them arriving at different
    times on a server with fewer slots than requests: bitwise equal states,
    and equal to sg_propagate_chebyshev with the library bounds."""
    sg = _sg()
    p = sg.SG_FP64 if prec == "fp64" else sg.SG_MIXED
    reqs = _serve_requests()
    sizes = [sg.sg_count_sizes(inst.D, inst.L)[2] for inst, _, _ in reqs]
    say(f"serve alone vs mix ({prec})")
    alone = []
    srv = sg.sg_serve_create(max_slots=1, precision=p, check_every=2, tol=1e-6)
    try:
        for (inst, dt, ns), n in zip(reqs, sizes):
            r = _wait(sg, srv, _submit(sg, srv, inst, dt, ns), n)
            assert r["status"] == sg.SG_OK
            assert r["stats"]["steps_done"] == ns
            alone.append(r["psi"].copy())
    finally:
        sg.sg_serve_destroy(srv)
    srv = sg.sg_serve_create(max_slots=3, precision=p, check_every=2, tol=1e-6,
                             compile_threads=2)
    try:
        tickets = []
        for j, (inst, dt, ns) in enumerate(reqs):
            tickets.append(_submit(sg, srv, inst, dt, ns))
            if j % 2:
                time.sleep(0.01)   # later arrivals join running ticks
        mixed = [_wait(sg, srv, t, n) for t, n in zip(tickets, sizes)]
        cnt = sg.sg_serve_counters(srv)
    finally:
        sg.sg_serve_destroy(srv)
    for i, r in enumerate(mixed):
        assert r["status"] == sg.SG_OK
        assert np.array_equal(r["psi"], alone[i]), i
        assert r["t_submit"] <= r["t_admit"] <= r["t_done"]
    assert cnt["finished"] == len(reqs) and cnt["resident"] == 0
    # the server's alone result is sg_propagate_chebyshev's with the library bounds
    for i in (0, 2):
        inst, dt, ns = reqs[i]
        with sg.Problem.from_instance(inst) as P:
            if p == sg.SG_MIXED:
                sg.sg_set_mixed_threshold(P.handle, 16)
            lo, hi = sg.sg_spectral_bounds(P.handle, 40)
        ref, _ = _alone(sg, inst, dt, ns, lo, hi, p)
        assert np.array_equal(ref, alone[i]), i


def test_serve_states_match_oracle_initial_and_norm():
    """One server request of 1 step: norm conserved and the first check saw
    the coherent state's energy (<psi|H|psi> of the oracle's coefficients)."""
    sg = _sg()
    inst = sg_inputs.config0()
    srv = sg.sg_serve_create(max_slots=4, check_every=1)
    try:
        with sg.Problem.from_instance(inst) as P:
            comp = sg.sg_basis_indices(P.handle)
            n = P.n_cs
        psi0, _ = coherent_coefficients(comp, inst.shift)
        r = _wait(sg, srv, _submit(sg, srv, inst, 0.1, 1), n)
    finally:
        sg.sg_serve_destroy(srv)
    from oracle.action import galerkin_masked_matrix
    H = galerkin_masked_matrix(inst)
    e0 = np.vdot(psi0, H @ psi0).real / np.vdot(psi0, psi0).real
    assert r["status"] == sg.SG_OK
    assert abs(r["stats"]["energy0"] - e0) < 1e-12 * abs(e0)
    assert abs(np.linalg.norm(r["psi"]) - 1.0) < 1e-12


def test_serve_errors_cancel_and_budget():
    sg = _sg()
    inst = sg_inputs.config1()
    n = sg.sg_count_sizes(inst.D, inst.L)[2]
    srv = sg.sg_serve_create(max_slots=2)
    try:
        with pytest.raises(sg.SgError) as e:
            sg.sg_serve_poll(srv, 12345)
        assert e.value.status == sg.SG_ENOTFOUND
        with pytest.raises(sg.SgError) as e:
            _submit(sg, srv, inst, -0.1, 5)
        assert e.value.status == sg.SG_EINVAL
        t_long = _submit(sg, srv, inst, 0.05, 100000)
        assert sg.sg_serve_poll(srv, t_long, n) is None     # SG_EAGAIN
        t_short = _submit(sg, srv, sg_inputs.config0(), 0.1, 3)
        time.sleep(0.2)
        sg.sg_serve_cancel(srv, t_long)
        r = _wait(sg, srv, t_long, n)
        assert r["status"] == sg.SG_ECANCELED
        r2 = _wait(sg, srv, t_short, 64)
        assert r2["status"] == sg.SG_OK
        with pytest.raises(sg.SgError) as e:
            sg.sg_serve_poll(srv, t_short)                   # record dropped
        assert e.value.status == sg.SG_ENOTFOUND
        with pytest.raises(sg.SgError) as e:
            sg.sg_serve_cancel(srv, 999999)
        assert e.value.status == sg.SG_ENOTFOUND
    finally:
        sg.sg_serve_destroy(srv)
    # a budget no (6, 6) request fits: refused at submission
    srv = sg.sg_serve_create(max_slots=2, hbm_budget_bytes=1 << 20)
    try:
        with pytest.raises(sg.SgError) as e:
            _submit(sg, srv, inst, 0.05, 5)
        assert e.value.status == sg.SG_ENOMEM
        r = _wait(sg, srv, _submit(sg, srv, sg_inputs.config0(), 0.1, 2), 64)
        assert r["status"] == sg.SG_OK
    finally:
        sg.sg_serve_destroy(srv)


def test_serve_destroy_with_work_in_flight():
    sg = _sg()
    srv = sg.sg_serve_create(max_slots=2)
    for inst, dt, ns in _serve_requests()[:4]:
        _submit(sg, srv, inst, dt, 1000)
    time.sleep(0.3)
    sg.sg_serve_destroy(srv)     # joins the threads, frees resident requests
