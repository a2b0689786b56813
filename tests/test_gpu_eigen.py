"""Block Davidson on the GPU operator action against the eigenpair oracle."""
import numpy as np
import pytest

import sg_inputs
from oracle.eigen import lowest_eigenpairs
from tests.gpu_util import device, say, to_host

pytestmark = pytest.mark.gpu


def _sg():
    import paper_2111_13655_amd as sg
    return sg


def _solve(sg, inst, nev, tol=1e-9, guess=None, want_vecs=False):
    import torch
    with sg.Problem.from_instance(inst) as P:
        vecs = None
        if want_vecs:
            vecs = torch.empty((nev, P.n_cs), dtype=torch.complex128, device=device())
        status, w, rn, st = sg.sg_eigensolve(P.handle, nev, tol=tol, guess=guess, evecs=vecs)
        out = to_host(vecs) if want_vecs else None
    return status, w, rn, st, out


def test_uncoupled_spectrum_exact():
    sg = _sg()
    inst = sg_inputs.small_instance(3, 4, seed=11, with_k=False)
    inst.c[:] = 0.0
    say("eigen uncoupled (3,4)")
    status, w, rn, st, _ = _solve(sg, inst, 6)
    ref, _ = lowest_eigenpairs(inst, 6)
    assert status == sg.SG_OK
    assert np.abs(w - ref).max() < 1e-10
    assert rn.max() <= 1e-9


@pytest.mark.parametrize("D,L,nev", [(2, 4, 5), (4, 4, 8), (3, 5, 6)])
def test_coupled_small_vs_dense(D, L, nev):
    sg = _sg()
    inst = sg_inputs.small_instance(D, L, seed=40 + D + L, with_k=True)
    say(f"eigen ({D},{L}) nev={nev}")
    status, w, rn, st, vecs = _solve(sg, inst, nev, want_vecs=True)
    ref, rv = lowest_eigenpairs(inst, nev)
    assert status == sg.SG_OK
    assert np.abs(w - ref).max() < 1e-10 * max(1.0, np.abs(ref).max())
    # eigenvectors: real, orthonormal, and equal to the oracle's up to sign
    assert np.abs(vecs.imag).max() == 0.0
    V = vecs.real
    assert np.abs(V @ V.T - np.eye(nev)).max() < 1e-10
    gaps = np.diff(ref)
    for k in range(nev):
        if (k == 0 or gaps[k - 1] > 1e-6) and (k == nev - 1 or gaps[k] > 1e-6):
            assert abs(abs(V[k] @ rv[:, k]) - 1.0) < 1e-8, k


def test_config1_lowest_states():
    """(D, L) = (6, 6): the 4 lowest states against Lanczos on the sparse
    masked-Galerkin matrix."""
    sg = _sg()
    inst = sg_inputs.config1()
    say("eigen config1")
    status, w, rn, st, _ = _solve(sg, inst, 4, tol=1e-8)
    ref, _ = lowest_eigenpairs(inst, 4)
    assert status == sg.SG_OK
    assert np.abs(w - ref).max() < 1e-9 * np.abs(ref).max()


def test_low_level_guess_restart():
    """The paper's two-stage run: solve at a low level, embed the states into
    the nested higher-level basis, and start Davidson there from them."""
    import torch
    sg = _sg()
    rng = np.random.default_rng(5)
    lo_inst = sg_inputs.draw_instance(rng, 4, 3, with_k=True)
    hi_inst = sg_inputs.Instance(D=4, L=5, omega=lo_inst.omega, c=lo_inst.c, k=lo_inst.k,
                                 shift=lo_inst.shift)
    nev = 4
    say("eigen low-level guess")
    with sg.Problem.from_instance(lo_inst) as Plo, sg.Problem.from_instance(hi_inst) as Phi:
        vlo = torch.empty((nev, Plo.n_cs), dtype=torch.complex128, device=device())
        s0, wlo, _, _ = sg.sg_eigensolve(Plo.handle, nev, tol=1e-10, evecs=vlo)
        assert s0 == sg.SG_OK
        guess = torch.empty((nev, Phi.n_cs), dtype=torch.complex128, device=device())
        for k in range(nev):
            sg.sg_embed_basis(Plo.handle, Phi.handle, vlo[k], guess[k])
        g = to_host(guess)
        # the embedding only relabels the coefficients
        assert np.allclose(np.linalg.norm(g, axis=1), 1.0, atol=1e-12)
        s1, w1, _, st1 = sg.sg_eigensolve(Phi.handle, nev, tol=1e-9, guess=guess)
        s2, w2, _, st2 = sg.sg_eigensolve(Phi.handle, nev, tol=1e-9)
    ref, _ = lowest_eigenpairs(hi_inst, nev)
    assert s1 == sg.SG_OK and s2 == sg.SG_OK
    assert np.abs(w1 - ref).max() < 1e-10 * np.abs(ref).max()
    assert np.abs(w2 - ref).max() < 1e-10 * np.abs(ref).max()
    assert st1["applies"] < st2["applies"]


def test_eigensolve_rejects_bad_arguments():
    sg = _sg()
    inst = sg_inputs.config0()
    with sg.Problem.from_instance(inst) as P:
        for kw in (dict(nev=0), dict(nev=2, max_basis=3), dict(nev=2, tol=-1.0)):
            nev = kw.pop("nev")
            with pytest.raises(sg.SgError) as e:
                sg.sg_eigensolve(P.handle, nev, **kw)
            assert e.value.status == sg.SG_EINVAL
