"""Pins of the eigenpair oracle (CPU)."""
import numpy as np

import sg_inputs
from oracle.eigen import literal_matrix, lowest_eigenpairs
from oracle.smolyak import build_structure


def test_uncoupled_eigenvalues_are_harmonic_sums():
    """c = k = 0: H_S is diagonal with entries sum_i omega_i (n_i + 1/2) over
    the compact basis, so its spectrum is that list, sorted."""
    inst = sg_inputs.small_instance(3, 4, seed=11, with_k=False)
    inst.c[:] = 0.0
    w, _ = lowest_eigenpairs(inst, 8)
    S = build_structure(inst.D, inst.L, inst.nb_A, inst.nb_B)
    h0 = np.sort((np.asarray(S.compact) + 0.5) @ inst.omega)
    assert np.allclose(w, h0[:8], rtol=0, atol=1e-12)


def test_eigenpairs_match_the_literal_route():
    """The lowest eigenpairs of Route 2 against a dense decomposition of the
    matrix assembled from Route 1 (the per-term Alg. 1 action)."""
    for D, L, seed in [(2, 4, 3), (3, 3, 4)]:
        inst = sg_inputs.small_instance(D, L, seed=seed, with_k=True)
        w, v = lowest_eigenpairs(inst, 5)
        H1 = literal_matrix(inst)
        assert np.abs(H1 - H1.T).max() < 1e-12
        w1 = np.linalg.eigvalsh(H1)[:5]
        assert np.allclose(w, w1, rtol=0, atol=1e-11 * max(1.0, abs(w1).max()))
        # residuals of the returned vectors under the literal matrix
        assert np.abs(H1 @ v - v * w).max() < 1e-10
