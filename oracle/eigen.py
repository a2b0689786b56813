"""Lowest eigenpairs of the Smolyak operator H_S.

Oracle (test infrastructure only).

The paper converges stationary states with the Davidson method (Sec. 3,
flowchart text) applied to the same operator action; whatever the iteration,
its limits are the eigenpairs of H_S.  The oracle takes them from a plain
eigen-decomposition of the masked-Galerkin matrix (Route 2 of
oracle.action): dense `eigh` for small bases, `eigsh` (implicitly restarted
Lanczos) on the sparse matrix otherwise.
"""
from __future__ import annotations

import numpy as np
from scipy.sparse.linalg import eigsh

from .action import Oracle, galerkin_masked_matrix


def lowest_eigenpairs(inst, nev: int, dense_limit: int = 4000):
    """(eigenvalues ascending [nev], eigenvectors [N_cs, nev])."""
    H = galerkin_masked_matrix(inst)
    n = H.shape[0]
    if n <= dense_limit:
        w, v = np.linalg.eigh(H.toarray())
        return w[:nev], v[:, :nev]
    w, v = eigsh(H, k=nev, which="SA", tol=1e-14)
    order = np.argsort(w)
    return w[order], v[:, order]


def literal_matrix(inst) -> np.ndarray:
    """H_S assembled column by column from the literal per-term action
    (Route 1): an independent path to the same matrix, for small bases."""
    O = Oracle(inst)
    n = O.S.n_cs
    H = np.zeros((n, n))
    e = np.zeros(n)
    for j in range(n):
        e[j] = 1.0
        H[:, j] = O.apply_literal(e).real
        e[j] = 0.0
    return H
