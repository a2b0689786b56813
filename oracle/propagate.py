"""Initial state, Chebyshev propagation, observables.

Oracle (test infrastructure only).

The paper propagates wave packets with "the Chebyshev method" (Sec. 3 flowchart
text; Sec. 5 pyrazine run) and gives no formulas.  Reading used here
(Tal-Ezer & Kosloff 1984), hbar = 1:

  Hs = (H - Ebar) / (dE/2), Ebar = (Emax+Emin)/2, dE = Emax - Emin, R = dE dt/2
  exp(-i H dt) psi = exp(-i Ebar dt) sum_k (2 - delta_k0) J_k(R) phi_k
  phi_0 = psi, phi_1 = -i Hs psi, phi_{k+1} = -2i Hs phi_k + phi_{k-1}

(phi_k = (-i)^k T_k(Hs) psi).  The series stops at the first k > R where
|J_k(R)| and |J_{k+1}(R)| are both below `tol`; terms 0..k-1 are kept.
Bessel values come from scipy.special.jv (library routine).

Initial state (Sec. 5: a Gaussian packet placed so that the Smolyak basis
covers it): psi0(Q) = prod_i pi^{-1/4} exp(-(Q_i - s_i)^2 / 2), whose Hermite
coefficients are those of a coherent state,
c_n = prod_i exp(-a_i^2/2) a_i^{n_i} / sqrt(n_i!), a_i = s_i / sqrt(2);
restricted to the compact basis and normalised.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import jv


def coherent_coefficients(compact: np.ndarray, shift: np.ndarray):
    """Returns (normalised coefficients, captured norm before normalising)."""
    a = np.asarray(shift, dtype=np.float64) / math.sqrt(2.0)
    N = np.asarray(compact)
    nmax = int(N.max()) if N.size else 0
    c = np.ones(N.shape[0])
    for i in range(N.shape[1]):
        # one-mode table e^{-a^2/2} a^n / sqrt(n!) for n = 0..nmax
        tab = np.empty(nmax + 1)
        tab[0] = math.exp(-0.5 * a[i] ** 2)
        for n in range(1, nmax + 1):
            tab[n] = tab[n - 1] * a[i] / math.sqrt(n)
        c *= tab[N[:, i]]
    nrm = float(np.linalg.norm(c))
    return (c / nrm).astype(np.complex128), nrm


def chebyshev_coefficients(R: float, tol: float = 1e-16) -> np.ndarray:
    """a_k = (2 - delta_k0) J_k(R) for k = 0..K-1 (truncation rule above)."""
    k = int(math.floor(R)) + 1
    while not (abs(jv(k, R)) < tol and abs(jv(k + 1, R)) < tol):
        k += 1
    a = np.array([jv(j, R) for j in range(k)], dtype=np.float64)
    a[1:] *= 2.0
    return a


def chebyshev_step(apply, psi: np.ndarray, dt: float, emin: float, emax: float,
                   coeffs: np.ndarray | None = None, tol: float = 1e-16):
    """One step; returns (psi(t+dt), <psi|H|psi> at the start of the step)."""
    Ebar = 0.5 * (emax + emin)
    half = 0.5 * (emax - emin)
    R = half * dt
    a = chebyshev_coefficients(R, tol) if coeffs is None else coeffs
    phi0 = psi
    phi1 = -1j * (apply(psi) - Ebar * psi) / half
    energy = Ebar + half * float(np.real(np.vdot(psi, 1j * phi1)))
    acc = a[0] * phi0 + a[1] * phi1
    for kk in range(2, len(a)):
        phi2 = -2j * (apply(phi1) - Ebar * phi1) / half + phi0
        acc = acc + a[kk] * phi2
        phi0, phi1 = phi1, phi2
    return np.exp(-1j * Ebar * dt) * acc, energy


def propagate(apply, psi0: np.ndarray, dt: float, nsteps: int, emin: float,
              emax: float, check_every: int = 0, tol: float = 1e-16):
    """Runs nsteps Chebyshev steps.  Returns (psi, records) where records is a
    list of (step, norm, energy) taken every `check_every` steps."""
    a = chebyshev_coefficients(0.5 * (emax - emin) * dt, tol)
    psi = np.asarray(psi0, dtype=np.complex128)
    records = []
    for s in range(nsteps):
        new, e = chebyshev_step(apply, psi, dt, emin, emax, a)
        if check_every and s % check_every == 0:
            records.append((s, float(np.linalg.norm(psi)), e))
        psi = new
    return psi, records


def spectral_bounds_dense(H: np.ndarray, pad: float = 0.05):
    """Extreme eigenvalues of a small symmetric matrix (library eigh), padded by
    `pad` of the range on both sides."""
    ev = np.linalg.eigvalsh(np.asarray(H))
    lo, hi = float(ev[0]), float(ev[-1])
    d = hi - lo
    return lo - pad * d, hi + pad * d


def spectral_bounds_sparse(H, pad: float = 0.05):
    """Extreme eigenvalues of a large sparse symmetric matrix (library
    eigsh), padded like spectral_bounds_dense."""
    from scipy.sparse.linalg import eigsh
    lo = float(eigsh(H, k=1, which="SA", return_eigenvectors=False, tol=1e-10)[0])
    hi = float(eigsh(H, k=1, which="LA", return_eigenvectors=False, tol=1e-10)[0])
    d = hi - lo
    return lo - pad * d, hi + pad * d


def exact_propagator(H: np.ndarray, psi0: np.ndarray, t: float) -> np.ndarray:
    """exp(-i H t) psi0 through a dense eigendecomposition (small cases)."""
    ev, V = np.linalg.eigh(np.asarray(H))
    return V @ (np.exp(-1j * ev * t) * (V.T @ psi0))

