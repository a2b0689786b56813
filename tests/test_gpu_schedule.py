"""Term-to-workgroup schedules and their autotuner: a schedule only decides
which threads compute a term, so every schedule must give bitwise the same
H|psi>, and that result must match the oracle."""
import numpy as np
import pytest

import sg_inputs
from oracle.action import Oracle
from tests.gpu_util import device, say, to_host

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2111_13655_amd as sg
    return sg


def _random_state(n, seed):
    import torch
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v /= np.linalg.norm(v)
    return torch.tensor(v, dtype=torch.complex128, device=device())


@pytest.mark.parametrize("prec", [0, 1])
def test_schedules_agree_bitwise(prec):
    import torch
    sg = _sg()
    inst = sg_inputs.config1()
    say(f"schedules (6,6) prec={prec}")
    with sg.Problem.from_instance(inst) as P:
        x = _random_state(P.n_cs, 3)
        y = torch.empty_like(x)
        outs = []
        for g, spread in ((0, 1), (0, 2), (64, 1), (256, 2), (1024, 1), (4096, 2)):
            sg.sg_set_schedule(P.handle, g, spread)
            sg.sg_apply_H(P.handle, x, y, prec)
            outs.append(to_host(y).copy())
        for o in outs[1:]:
            assert np.array_equal(o.view(np.float64), outs[0].view(np.float64))


def test_schedules_agree_bitwise_config2():
    """(D, L) = (12, 6): the default packing (1536-point terms three to a
    wavefront pack) against schedules that run those terms, or every term
    above 512 points, on whole workgroups: bitwise the same H|psi>."""
    import torch
    sg = _sg()
    inst = sg_inputs.config2()
    say("schedules (12,6)")
    with sg.Problem.from_instance(inst) as P:
        x = _random_state(P.n_cs, 4)
        y = torch.empty_like(x)
        outs = []
        for g, spread in ((0, 1), (1025, 1), (513, 2), (4096, 1)):
            sg.sg_set_schedule(P.handle, g, spread)
            sg.sg_apply_H(P.handle, x, y, 0)
            outs.append(to_host(y).copy())
        for o in outs[1:]:
            assert np.array_equal(o.view(np.float64), outs[0].view(np.float64))


def test_tuned_schedule_matches_oracle():
    import torch
    sg = _sg()
    inst = sg_inputs.small_instance(4, 4, seed=21, with_k=True)
    say("tuned schedule (4,4) vs oracle")
    with sg.Problem.from_instance(inst) as P:
        x = _random_state(P.n_cs, 4)
        g, spread = sg.sg_tune_schedule(P.handle, x, sg.SG_FP64, reps=3)
        assert g == 0 or (g >= 64 and g & (g - 1) == 0)
        assert spread in (1, 2)
        y = torch.empty_like(x)
        sg.sg_apply_H(P.handle, x, y, sg.SG_FP64)
        got = to_host(y)
        ref = Oracle(inst).apply_literal(to_host(x))
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_tune_schedule_rejects_bad_arguments():
    sg = _sg()
    with sg.Problem.from_instance(sg_inputs.config0()) as P:
        x = _random_state(P.n_cs, 5)
        for kw in (dict(reps=0), dict(precision=7)):
            with pytest.raises(sg.SgError) as e:
                sg.sg_tune_schedule(P.handle, x, **kw)
            assert e.value.status == sg.SG_EINVAL
