"""Taylor, Runge-Kutta, Bulirsch-Stoer and short-iterative-Lanczos propagation.

Oracle (test infrastructure only).

Besides the Chebyshev method, the paper lists n-order Runge-Kutta, n-order
Taylor expansion, short iterative Lanczos and Bulirsch-Stoer propagators
(Sec. 3, the overview of the program flow) without formulas.  Readings used
here, all for the time-independent Schroedinger equation
d psi / dt = -i H psi (hbar = 1):

* Taylor of order n: one step multiplies by sum_{k=0}^{n} (-i H dt)^k / k!.
* Runge-Kutta of order n (1..4): the explicit method with Butcher tableau
  (A, b), stages k_i = f(psi + dt sum_{j<i} A_ij k_j), psi += dt sum_i b_i k_i,
  f(y) = -i H y.  Tableaux: Euler (1), explicit midpoint (2), Heun's
  third-order method (3), the classical fourth-order method (4).
* Bulirsch-Stoer with k extrapolation columns: the modified midpoint rule
  over n_i = 2i substeps (i = 1..k) of the step, each result extrapolated to
  zero substep size by the Aitken-Neville recursion in h^2 (the textbook
  form, e.g. Stoer and Bulirsch, Introduction to Numerical Analysis).
  Fixed k and fixed step: no error control.
* Short iterative Lanczos with Krylov dimension m (Park and Light, 1986):
  Lanczos from psi / |psi| builds an orthonormal basis V of the Krylov space
  (each new vector orthogonalised against all earlier ones, twice) and the
  tridiagonal T = V^H H V; one step is psi <- |psi| V exp(-i T dt) e_1.  The
  recurrence stops early when the space becomes invariant (new norm below
  1e-13 of the start norm).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import expm

# explicit Runge-Kutta tableaux (A strictly lower triangular, b weights)
RK_TABLEAUX = {
    1: (np.zeros((1, 1)), np.array([1.0])),
    2: (np.array([[0.0, 0.0], [0.5, 0.0]]), np.array([0.0, 1.0])),
    3: (np.array([[0.0, 0.0, 0.0], [1.0 / 3.0, 0.0, 0.0], [0.0, 2.0 / 3.0, 0.0]]),
        np.array([0.25, 0.0, 0.75])),
    4: (np.array([[0.0, 0.0, 0.0, 0.0], [0.5, 0.0, 0.0, 0.0], [0.0, 0.5, 0.0, 0.0],
                  [0.0, 0.0, 1.0, 0.0]]),
        np.array([1.0, 2.0, 2.0, 1.0]) / 6.0),
}


def taylor_step(apply, psi: np.ndarray, dt: float, order: int) -> np.ndarray:
    term = np.asarray(psi, dtype=np.complex128)
    out = term.copy()
    for k in range(1, order + 1):
        term = (-1j * dt / k) * apply(term)
        out = out + term
    return out


def rk_step(apply, psi: np.ndarray, dt: float, order: int) -> np.ndarray:
    A, b = RK_TABLEAUX[order]
    y = np.asarray(psi, dtype=np.complex128)
    ks = []
    for i in range(len(b)):
        yi = y.copy()
        for j in range(i):
            if A[i, j] != 0.0:
                yi = yi + dt * A[i, j] * ks[j]
        ks.append(-1j * apply(yi))
    out = y.copy()
    for i in range(len(b)):
        if b[i] != 0.0:
            out = out + dt * b[i] * ks[i]
    return out


def modified_midpoint(apply, psi: np.ndarray, H: float, nsub: int) -> np.ndarray:
    f = lambda y: -1j * apply(y)
    h = H / nsub
    z0 = np.asarray(psi, dtype=np.complex128)
    z1 = z0 + h * f(z0)
    for _ in range(1, nsub):
        z0, z1 = z1, z0 + 2.0 * h * f(z1)
    return 0.5 * (z1 + z0 + h * f(z1))


def bs_step(apply, psi: np.ndarray, dt: float, k: int) -> np.ndarray:
    ns = [2 * (i + 1) for i in range(k)]
    rows = []
    for i, n in enumerate(ns):
        row = [modified_midpoint(apply, psi, dt, n)]
        for j in range(1, i + 1):
            r = (ns[i] / ns[i - j]) ** 2
            row.append(row[j - 1] + (row[j - 1] - rows[i - 1][j - 1]) / (r - 1.0))
        rows.append(row)
    return rows[-1][-1]


def lanczos_basis(apply, psi: np.ndarray, m: int):
    """Krylov basis V (columns), the tridiagonal T and |psi|."""
    psi = np.asarray(psi, dtype=np.complex128)
    beta0 = float(np.linalg.norm(psi))
    V = [psi / beta0]
    alpha, beta = [], []
    for j in range(m):
        w = apply(V[j])
        a_j = 0.0
        for _ in range(2):
            c = np.array([np.vdot(v, w) for v in V])
            a_j += float(np.real(c[j]))
            w = w - sum(ci * v for ci, v in zip(c, V))
        alpha.append(a_j)
        if j == m - 1:
            break
        b = float(np.linalg.norm(w))
        if b < 1e-13 * beta0:
            break
        beta.append(b)
        V.append(w / b)
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    return np.array(V[:k]).T, T, beta0


def sil_step(apply, psi: np.ndarray, dt: float, m: int) -> np.ndarray:
    V, T, beta0 = lanczos_basis(apply, psi, m)
    e1 = np.zeros(T.shape[0], dtype=np.complex128)
    e1[0] = 1.0
    return beta0 * (V @ (expm(-1j * dt * T) @ e1))


def propagate(method: str, apply, psi0: np.ndarray, dt: float, nsteps: int, order: int):
    step = {"taylor": taylor_step, "rk": rk_step, "sil": sil_step, "bs": bs_step}[method]
    psi = np.asarray(psi0, dtype=np.complex128)
    for _ in range(nsteps):
        psi = step(apply, psi, dt, order)
    return psi


def taylor_factor(z: complex, order: int) -> complex:
    """sum_{k<=order} z^k / k!: what Taylor of that order (and, for a linear
    equation, every explicit Runge-Kutta method of that order <= 4) multiplies
    an eigencomponent by, z = -i E dt."""
    return sum(z ** k / math.factorial(k) for k in range(order + 1))
