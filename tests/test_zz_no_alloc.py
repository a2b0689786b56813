"""The allocation-free propagation entry point against the allocating one:
bitwise the same state, statistics and traces (same kernels, same order), on
two calls in a row, the second on a smaller problem, so the fixed device
array is reused with stale contents from the first call."""
import numpy as np
import pytest

import sg_inputs
from tests.gpu_util import empty, say, to_host

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2111_13655_amd as sg
    return sg


CASES = [((6, 6, 1), "taylor", 12), ((4, 4, 3), "sil", 10), ((6, 6, 1), "bs", 3),
         ((3, 5, 4), "rk", 4)]


def _run(sg, entry, P, inst, method, order, steps=6):
    psi = empty(P.n_cs)
    sg.sg_init_gaussian(P.handle, inst.shift, psi)
    st, stats, nt, et = entry(P.handle, psi, 0.05, steps, method, order, check_every=2)
    assert st == sg.SG_OK
    return to_host(psi), stats, nt, et


def test_noalloc_matches_allocating_propagators():
    sg = _sg()
    methods = {"taylor": sg.SG_PROP_TAYLOR, "rk": sg.SG_PROP_RK, "sil": sg.SG_PROP_SIL,
               "bs": sg.SG_PROP_BS}
    # the calls run back to back; each case after the first starts with the
    # previous call's data in the array, and the second problem is smaller
    for (D, L, seed), name, order in CASES:
        say(f"noalloc {name}-{order} D={D} L={L}")
        inst = sg_inputs.small_instance(D, L, seed=seed) if (D, L) != (6, 6) else sg_inputs.config1()
        with sg.Problem.from_instance(inst) as P:
            a = _run(sg, sg.sg_propagate, P, inst, methods[name], order)
            b = _run(sg, sg.sg_propagate_noalloc, P, inst, methods[name], order)
        assert np.array_equal(a[0], b[0]), name
        assert a[1].keys() == b[1].keys()
        for k in a[1]:   # NaN (no spectral bounds for these methods) equals NaN
            assert a[1][k] == b[1][k] or (np.isnan(a[1][k]) and np.isnan(b[1][k])), k
        assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


def test_noalloc_refuses_work_beyond_the_array():
    sg = _sg()
    inst = sg_inputs.config2()             # N_cs = 369305: 5.9 MB per vector
    with sg.Problem.from_instance(inst) as P:
        psi = empty(P.n_cs)
        sg.sg_init_gaussian(P.handle, inst.shift, psi)
        before = to_host(psi)
        need = (64 + 1 + 1) * 16 * P.n_cs
        assert need > sg.sg_noalloc_scratch_bytes()
        with pytest.raises(sg.SgError) as e:
            sg.sg_propagate_noalloc(P.handle, psi, 0.05, 1, sg.SG_PROP_SIL, 64)
        assert e.value.status == sg.SG_EINVAL
        assert np.array_equal(to_host(psi), before)
        # a propagation that fits runs, and matches the allocating one
        x = psi.clone()
        sg.sg_propagate(P.handle, psi, 0.05, 2, sg.SG_PROP_TAYLOR, 6)
        sg.sg_propagate_noalloc(P.handle, x, 0.05, 2, sg.SG_PROP_TAYLOR, 6)
        assert np.array_equal(to_host(psi), to_host(x))
