"""The Smolyak operator action H_S|psi> on the compact basis.

Oracle (test infrastructure only).

Route 1 (`apply_literal`) takes Alg. 1 (Sec. 3) step by step for every term
of R(l), as eq_action_smolyak (Sec. 2) sums them:
  1. gather the term's coefficients from the compact vector through M^B;
  2. basis -> grid along every mode (eq_transfer_b_to_g), level-0 modes
     included;
  3. the operator on the term's direct-product grid: V(Q) times the grid
     values, plus the kinetic part -1/2 omega_i d^2/dQ_i^2 evaluated at the
     grid points from the basis expansion with second-derivative tables;
  4. grid -> basis along every mode (eq_transfer_g_to_b) with weights wt_u;
  5. add D_l times the result into the compact output through M^B.
Terms are visited in Table 2 order.

Route 2 (`galerkin_masked_matrix`) is the plain definition this reaches for
the polynomial Hamiltonians used here.  Each term's product Gauss-Hermite rule
is exact for every matrix element <n|H|m> inside that term (per-mode degree at
most 4l+2 against 4l+3 for the 2l+2-point rule), so a term contributes D_l
times the exact Galerkin element, and summing D_l over the terms holding both
n and m gives 1 when sum_i max(g(n_i), g(m_i)) <= L and 0 otherwise
(combination identity).  Hence H_S[n,m] = H[n,m] * mask(n,m), with analytic
elements built from the one-mode position matrix <n|Q|m>.

`brute_force_masked` builds the full direct-product Galerkin matrix on the
largest level's basis and grid, then masks and restricts it: an independent
check of both routes at tiny D, L.

The Hamiltonian family: H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2)
+ sum_{i<j} c_ij Q_i^2 Q_j^2 + sum_{i<j} k_ij Q_i^2 Q_j, or, in Route 1, the
harmonic part plus a general coupling potential V(Q) given as a function.
For a general V the term rules are no longer exact and Route 2 does not
apply; Route 1 is then the definition.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .hermite import tables_for, hermite_functions, hermite_second_derivatives, gauss_hermite
from .smolyak import (CompactRanker, build_structure, lowest_level,
                      size_of_level)


def mode_product(T: np.ndarray, M: np.ndarray, axis: int) -> np.ndarray:
    """out[..., u, ...] = sum_k M[u, k] T[..., k, ...] along `axis`."""
    T = np.moveaxis(T, axis, 0)
    sh = T.shape
    out = (M @ T.reshape(sh[0], -1)).reshape((M.shape[0],) + sh[1:])
    return np.moveaxis(out, 0, axis)


def potential_on_grid(inst, xs: list[np.ndarray], coupling=None) -> np.ndarray:
    """V(Q) on the direct product of the one-mode grids xs (axis i = mode i):
    the harmonic part 1/2 omega_i Q_i^2 plus the couplings.  `coupling`, if
    given, replaces the polynomial couplings: a function of the list of D
    coordinate arrays (broadcasting against each other) returning the
    coupling potential at those points."""
    D = inst.D
    Q = np.meshgrid(*xs, indexing="ij", sparse=True)
    V = np.zeros(tuple(len(x) for x in xs))
    for i in range(D):
        V = V + 0.5 * inst.omega[i] * Q[i] ** 2
    if coupling is not None:
        return V + np.broadcast_to(coupling(Q), V.shape)
    for i in range(D):
        for j in range(i + 1, D):
            if inst.c[i, j] != 0.0:
                V = V + inst.c[i, j] * Q[i] ** 2 * Q[j] ** 2
            if inst.k[i, j] != 0.0:
                V = V + inst.k[i, j] * Q[i] ** 2 * Q[j]
    return V


class Oracle:
    """Holds the structure and tables for one instance.  `coupling` (a
    function of the D coordinate arrays, as in potential_on_grid) replaces the
    instance's polynomial couplings by a general potential."""

    def __init__(self, inst, structure=None, coupling=None):
        self.inst = inst
        self.coupling = coupling
        self.S = structure if structure is not None else build_structure(
            inst.D, inst.L, inst.nb_A, inst.nb_B)
        self.tab = tables_for(inst.L, inst.nb_A, inst.nb_B, inst.nq_A, inst.nq_B)

    # -- Route 1 ---------------------------------------------------------
    def term_action(self, t: int, psi: np.ndarray) -> np.ndarray:
        """Steps 1-4 of Alg. 1 for term t: returns the term's H|psi^l> on the
        term basis (flat, mode 1 fastest), not yet weighted by D_l."""
        S, tab, inst = self.S, self.tab, self.inst
        l = S.terms[t]
        idx = S.MB[S.term_offsets[t]:S.term_offsets[t + 1]]
        nbs = [tab[li].nb for li in l]
        X = psi[idx].reshape(nbs, order="F")                  # step 1 (gather)
        G = X
        for i, li in enumerate(l):                            # step 2 (B -> G)
            G = mode_product(G, tab[li].b, i)
        V = potential_on_grid(inst, [tab[li].x for li in l], self.coupling)
        HG = V * G                                            # step 3 (potential)
        for i in range(inst.D):                               # step 3 (kinetic)
            T = X
            for j, lj in enumerate(l):
                T = mode_product(T, tab[lj].d2b if j == i else tab[lj].b, j)
            HG = HG - 0.5 * inst.omega[i] * T
        R = HG
        for i, li in enumerate(l):                            # step 4 (G -> B)
            R = mode_product(R, tab[li].wtb_T, i)
        return R.reshape(-1, order="F")

    def apply_literal(self, psi: np.ndarray, terms=None) -> np.ndarray:
        """Route 1: H_S psi = sum_l D_l P_l H_l P_l psi (eq_action_smolyak)."""
        S = self.S
        psi = np.asarray(psi, dtype=np.complex128)
        out = np.zeros(S.n_cs, dtype=np.complex128)
        for t in (range(S.n_terms) if terms is None else terms):
            Dl = int(S.coeffs[t])
            if Dl == 0:
                continue
            idx = S.MB[S.term_offsets[t]:S.term_offsets[t + 1]]
            out[idx] += Dl * self.term_action(t, psi)         # step 5
        return out


# ---------------------------------------------------------------------------
# Route 2
# ---------------------------------------------------------------------------

def position_matrices(nmax: int):
    """<n|Q|m> and <n|Q^2|m> for n, m <= nmax.  Q is tridiagonal with
    <n+1|Q|n> = sqrt((n+1)/2); Q^2 is the matrix product, taken on a basis two
    functions larger than needed so that truncation does not touch n, m <=
    nmax."""
    M = nmax + 3
    Q = np.zeros((M, M))
    for n in range(M - 1):
        Q[n + 1, n] = Q[n, n + 1] = np.sqrt((n + 1) / 2.0)
    Q2 = Q @ Q
    return Q[:nmax + 1, :nmax + 1], Q2[:nmax + 1, :nmax + 1]


def galerkin_masked_matrix(inst, ranker: CompactRanker | None = None,
                           compact: np.ndarray | None = None) -> sp.csr_matrix:
    """Route 2: H_S[n, m] = <n|H|m> [sum_i max(g(n_i), g(m_i)) <= L]."""
    D, L = inst.D, inst.L
    for l in range(L + 1):
        nb = size_of_level(l, inst.nb_A, inst.nb_B)
        nq = size_of_level(l, inst.nq_A, inst.nq_B)
        if nq < nb + 1:
            raise ValueError("masked-Galerkin route needs nq(l) >= nb(l)+1")
    rk = ranker if ranker is not None else CompactRanker(D, L, inst.nb_A, inst.nb_B)
    N = compact if compact is not None else rk.enumerate()
    ncs = N.shape[0]
    nmax = rk.nmax
    Q1, Q2 = position_matrices(nmax + 2)
    g = lowest_level(np.arange(nmax + 3), inst.nb_A, inst.nb_B)
    gsum = g[N].sum(axis=1)
    rows_l, cols_l, vals_l = [], [], []
    diag = (inst.omega[None, :] * (N + 0.5)).sum(axis=1)
    rows_l.append(np.arange(ncs))
    cols_l.append(np.arange(ncs))
    vals_l.append(diag)
    ar = np.arange(ncs)

    def add_pair(i, j, di, dj, coef, Mi, Mj):
        m_i = N[:, i] + di
        m_j = N[:, j] + dj
        ok = (m_i >= 0) & (m_j >= 0) & (m_i <= nmax) & (m_j <= nmax)
        if not ok.any():
            return
        r = ar[ok]
        ni, nj, mi, mj = N[ok, i], N[ok, j], m_i[ok], m_j[ok]
        jl = gsum[ok] - g[ni] - g[nj] + np.maximum(g[ni], g[mi]) + np.maximum(g[nj], g[mj])
        keep = jl <= L
        if not keep.any():
            return
        r, ni, nj, mi, mj = r[keep], ni[keep], nj[keep], mi[keep], mj[keep]
        M = N[r].copy()
        M[:, i] = mi
        M[:, j] = mj
        cols = rk.rank(M)
        vals = coef * Mi[ni, mi] * Mj[nj, mj]
        rows_l.append(r)
        cols_l.append(cols)
        vals_l.append(vals)

    for i in range(D):
        for j in range(i + 1, D):
            if inst.c[i, j] != 0.0:
                for di in (-2, 0, 2):
                    for dj in (-2, 0, 2):
                        add_pair(i, j, di, dj, inst.c[i, j], Q2, Q2)
            if inst.k[i, j] != 0.0:
                for di in (-2, 0, 2):
                    for dj in (-1, 1):
                        add_pair(i, j, di, dj, inst.k[i, j], Q2, Q1)
    rows = np.concatenate(rows_l)
    cols = np.concatenate(cols_l)
    vals = np.concatenate(vals_l)
    H = sp.coo_matrix((vals, (rows, cols)), shape=(ncs, ncs)).tocsr()
    H.sum_duplicates()
    return H


def galerkin_masked_apply(inst, psi: np.ndarray, compact: np.ndarray) -> np.ndarray:
    """Route 2 applied without assembling the matrix: the same sums as
    galerkin_masked_matrix, H_S[n, m] = <n|H|m> [sum_i max(g(n_i), g(m_i)) <= L],
    taken row-wise over the coupling's pair shifts.  A shifted tuple's column
    is found by binary search of its base-(nmax+1) code among the codes of
    the compact tuples, which increase in the lexicographic compact order.
    compact: [N_cs, D] tuples in compact order."""
    D, L = inst.D, inst.L
    N = np.asarray(compact, dtype=np.int64)
    ncs = N.shape[0]
    nmax = int(N.max()) if ncs else 0
    base = nmax + 1
    weights = base ** np.arange(D - 1, -1, -1, dtype=np.int64)
    codes = N @ weights
    if ncs > 1 and not np.all(np.diff(codes) > 0):
        raise ValueError("compact tuples are not in lexicographic order")
    Q1, Q2 = position_matrices(nmax + 2)
    g = lowest_level(np.arange(nmax + 3), inst.nb_A, inst.nb_B)
    gsum = g[N].sum(axis=1)
    psi = np.asarray(psi, dtype=np.complex128)
    out = (inst.omega[None, :] * (N + 0.5)).sum(axis=1) * psi
    # per mode and shift d: is n_i + d a one-mode index, the rise of the
    # joint level max(g(n_i), g(n_i + d)) - g(n_i), and <n_i|Q|n_i+d>,
    # <n_i|Q^2|n_i+d>
    shifts = (-2, -1, 0, 1, 2)
    ok, rise, q1, q2 = {}, {}, {}, {}
    for i in range(D):
        ni = N[:, i]
        for d in shifts:
            m = ni + d
            v = (m >= 0) & (m <= nmax)
            mc = np.clip(m, 0, nmax)
            ok[i, d] = v
            rise[i, d] = np.maximum(g[ni], g[mc]) - g[ni]
            q1[i, d] = np.where(v, Q1[ni, mc], 0.0)
            q2[i, d] = np.where(v, Q2[ni, mc], 0.0)
    ar = np.arange(ncs)

    def add_pair(i, j, di, dj, coef, qi, qj):
        keep = ok[i, di] & ok[j, dj] & (gsum + rise[i, di] + rise[j, dj] <= L)
        if not keep.any():
            return
        r = ar[keep]
        c = codes[r] + di * weights[i] + dj * weights[j]
        cols = np.searchsorted(codes, c)
        assert np.array_equal(codes[cols], c)
        out[r] += coef * qi[i, di][r] * qj[j, dj][r] * psi[cols]

    for i in range(D):
        for j in range(i + 1, D):
            if inst.c[i, j] != 0.0:
                for di in (-2, 0, 2):
                    for dj in (-2, 0, 2):
                        add_pair(i, j, di, dj, inst.c[i, j], q2, q2)
            if inst.k[i, j] != 0.0:
                for di in (-2, 0, 2):
                    for dj in (-1, 1):
                        add_pair(i, j, di, dj, inst.k[i, j], q2, q1)
    return out


def galerkin_rows(inst, ranker: CompactRanker, tuples: np.ndarray):
    """Rows of H_S for a few compact tuples (for sampled checks at full size):
    returns a list of (cols, vals)."""
    D, L = inst.D, inst.L
    nmax = ranker.nmax
    Q1, Q2 = position_matrices(nmax + 2)
    g = lowest_level(np.arange(nmax + 3), inst.nb_A, inst.nb_B)
    out = []
    for n in np.asarray(tuples, dtype=np.int64):
        entries = {}

        def add(m, v):
            key = tuple(m)
            entries[key] = entries.get(key, 0.0) + v

        add(n, float((inst.omega * (n + 0.5)).sum()))
        for i in range(D):
            for j in range(i + 1, D):
                opts = []
                if inst.c[i, j] != 0.0:
                    opts += [(di, dj, inst.c[i, j], Q2, Q2) for di in (-2, 0, 2) for dj in (-2, 0, 2)]
                if inst.k[i, j] != 0.0:
                    opts += [(di, dj, inst.k[i, j], Q2, Q1) for di in (-2, 0, 2) for dj in (-1, 1)]
                for di, dj, coef, Mi, Mj in opts:
                    m = n.copy()
                    m[i] += di
                    m[j] += dj
                    if m[i] < 0 or m[j] < 0 or m[i] > nmax or m[j] > nmax:
                        continue
                    if np.maximum(g[n], g[m]).sum() > L:
                        continue
                    add(m, coef * Mi[n[i], m[i]] * Mj[n[j], m[j]])
        ms = np.array(list(entries.keys()), dtype=np.int64)
        vs = np.array(list(entries.values()))
        out.append((ranker.rank(ms), vs))
    return out


# ---------------------------------------------------------------------------
# Brute force on the full direct product (tiny D, L)
# ---------------------------------------------------------------------------

def brute_force_masked(inst, compact: np.ndarray, mask: bool = True) -> np.ndarray:
    """Dense H_S on the compact basis from the full direct-product Galerkin
    matrix (basis nb(L)^D, grid nq(L)^D, quadrature exact) masked by the joint
    level.  Independent of the term set."""
    D, L = inst.D, inst.L
    nb = size_of_level(L, inst.nb_A, inst.nb_B)
    nq = size_of_level(L, inst.nq_A, inst.nq_B)
    x, w, wt = gauss_hermite(nq)
    b = hermite_functions(nb, x)
    d2 = hermite_second_derivatives(nb, x)
    # full-basis tuple -> position (mode 1 fastest in this dense layout)
    V = potential_on_grid(inst, [x] * D).reshape(-1, order="F")
    W = np.ones(1)
    Phi = np.ones((1, 1))
    for _ in range(D):
        W = np.kron(wt, W)
        Phi = np.kron(b, Phi)
    H = Phi.T @ ((W * V)[:, None] * Phi)
    for i in range(D):
        Pi = np.ones((1, 1))
        for j in range(D):
            Pi = np.kron(d2 if j == i else b, Pi)
        H += -0.5 * inst.omega[i] * (Phi.T @ (W[:, None] * Pi))
    pos = np.zeros(compact.shape[0], dtype=np.int64)
    stride = 1
    for i in range(D):
        pos += compact[:, i] * stride
        stride *= nb
    Hc = H[np.ix_(pos, pos)]
    if not mask:
        return Hc
    g = lowest_level(np.arange(nb), inst.nb_A, inst.nb_B)
    gn = g[compact]                                        # [N_cs, D]
    joint = np.maximum(gn[:, None, :], gn[None, :, :]).sum(axis=2)
    return np.where(joint <= L, Hc, 0.0)
