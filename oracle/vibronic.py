"""The Smolyak operator action for a two-state (vibronic) Hamiltonian.

Oracle (test infrastructure only).

Sec. 5 propagates the pyrazine vibronic model: two electronic states, a
2 x 2 operator matrix at every nuclear configuration, with the harmonic part
on the diagonal, the energy gap 2 Delta, a linear interstate coupling
lambda Q_1 off the diagonal and state-dependent linear terms k_i^s Q_i
(i >= 2) on the diagonal.  Its parameters are not given; the family here
keeps that form and adds (optionally) state-dependent quartic couplings of
the anharmonic family used elsewhere, so that each surface is a coupled
anharmonic potential:

  H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2) (x) 1
      + [[V_00(Q), V_01(Q)], [V_01(Q), V_11(Q)]],
  V_ss(Q) = E_s + sum_i kappa^s_i Q_i + sum_{i<j} c^s_ij Q_i^2 Q_j^2,
  V_01(Q) = sum_i lambda_i Q_i.

The pyrazine form is E = (-Delta, Delta), lambda = (lambda, 0, ..., 0),
kappa^s_1 = 0, c = 0.

The wave packet carries an electronic index: psi[s, n] for s = 0, 1 and n in
the compact Smolyak basis.  The Smolyak operator is Sec. 2's
eq_action_smolyak with each term's operator acting on (electronic state) x
(the term's direct-product grid): H_S = sum_l D_l (1 (x) P_l)^T H_l (1 (x) P_l).

Route 1 (`apply_literal`): Alg. 1 per term, both states gathered, both
transformed basis -> grid along every mode, the 2 x 2 potential matrix and the
kinetic part applied on the grid, grid -> basis, D_l times the result added.
Route 2 (`masked_matrix`, `masked_apply`): every term's product rule is exact
for the matrix elements of this family (per-mode degree at most 4l+2 against
4l+3), so, as for one state, H_S[(s,n),(t,m)] = H[(s,n),(t,m)] times the
joint-level mask [sum_i max(g(n_i), g(m_i)) <= L], the same mask for all four
blocks.  `brute_force_masked` checks both on the full direct product at tiny
D, L.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .action import mode_product, position_matrices
from .hermite import gauss_hermite, hermite_functions, hermite_second_derivatives, tables_for
from .smolyak import CompactRanker, build_structure, lowest_level, size_of_level


def surface_potentials(inst, xs: list[np.ndarray]):
    """V_00, V_11 and V_01 on the direct product of the one-mode grids xs
    (axis i = mode i), without the harmonic part."""
    D = inst.D
    Q = np.meshgrid(*xs, indexing="ij", sparse=True)
    shape = tuple(len(x) for x in xs)
    V = [np.full(shape, float(inst.E[s])) for s in range(2)]
    V01 = np.zeros(shape)
    for i in range(D):
        for s in range(2):
            if inst.kappa[s, i] != 0.0:
                V[s] = V[s] + inst.kappa[s, i] * Q[i]
        if inst.lam[i] != 0.0:
            V01 = V01 + inst.lam[i] * Q[i]
    for s in range(2):
        for i in range(D):
            for j in range(i + 1, D):
                if inst.c2[s, i, j] != 0.0:
                    V[s] = V[s] + inst.c2[s, i, j] * Q[i] ** 2 * Q[j] ** 2
    return V[0], V[1], V01


def harmonic_on_grid(inst, xs):
    Q = np.meshgrid(*xs, indexing="ij", sparse=True)
    V = np.zeros(tuple(len(x) for x in xs))
    for i in range(inst.D):
        V = V + 0.5 * inst.omega[i] * Q[i] ** 2
    return V


class VibronicOracle:
    """Structure and tables for one two-state instance."""

    def __init__(self, inst, structure=None):
        self.inst = inst
        self.S = structure if structure is not None else build_structure(
            inst.D, inst.L, inst.nb_A, inst.nb_B)
        self.tab = tables_for(inst.L, inst.nb_A, inst.nb_B, inst.nq_A, inst.nq_B)

    def term_action(self, t: int, psi: np.ndarray) -> np.ndarray:
        """Steps 1-4 of Alg. 1 for term t on both states: returns [2, n_t]
        (term basis, mode 1 fastest), not yet weighted by D_l."""
        S, tab, inst = self.S, self.tab, self.inst
        l = S.terms[t]
        idx = S.MB[S.term_offsets[t]:S.term_offsets[t + 1]]
        nbs = [tab[li].nb for li in l]
        X = [psi[s, idx].reshape(nbs, order="F") for s in range(2)]      # step 1
        G = []
        for s in range(2):                                               # step 2
            g = X[s]
            for i, li in enumerate(l):
                g = mode_product(g, tab[li].b, i)
            G.append(g)
        xs = [tab[li].x for li in l]
        V00, V11, V01 = surface_potentials(inst, xs)                     # step 3
        Vh = harmonic_on_grid(inst, xs)
        HG = [(Vh + V00) * G[0] + V01 * G[1], V01 * G[0] + (Vh + V11) * G[1]]
        for s in range(2):
            for i in range(inst.D):
                T = X[s]
                for j, lj in enumerate(l):
                    T = mode_product(T, tab[lj].d2b if j == i else tab[lj].b, j)
                HG[s] = HG[s] - 0.5 * inst.omega[i] * T
        out = np.empty((2, idx.size), dtype=np.complex128)
        for s in range(2):                                               # step 4
            R = HG[s]
            for i, li in enumerate(l):
                R = mode_product(R, tab[li].wtb_T, i)
            out[s] = R.reshape(-1, order="F")
        return out

    def apply_literal(self, psi: np.ndarray, terms=None) -> np.ndarray:
        """Route 1: psi [2, N_cs] -> H_S psi [2, N_cs]."""
        S = self.S
        psi = np.asarray(psi, dtype=np.complex128).reshape(2, S.n_cs)
        out = np.zeros((2, S.n_cs), dtype=np.complex128)
        for t in (range(S.n_terms) if terms is None else terms):
            Dl = int(S.coeffs[t])
            if Dl == 0:
                continue
            idx = S.MB[S.term_offsets[t]:S.term_offsets[t + 1]]
            r = self.term_action(t, psi)
            for s in range(2):
                out[s, idx] += Dl * r[s]                                  # step 5
        return out


def _one_mode_elements(nmax: int):
    Q1, Q2 = position_matrices(nmax + 2)
    return Q1, Q2


def masked_matrix(inst, compact: np.ndarray | None = None) -> sp.csr_matrix:
    """Route 2 assembled: [[H00, H01], [H01, H11]] on the compact basis,
    2 N_cs square, state-major (row s N_cs + n)."""
    D, L = inst.D, inst.L
    rk = CompactRanker(D, L, inst.nb_A, inst.nb_B)
    N = compact if compact is not None else rk.enumerate()
    ncs = N.shape[0]
    nmax = rk.nmax
    Q1, Q2 = _one_mode_elements(nmax)
    g = lowest_level(np.arange(nmax + 3), inst.nb_A, inst.nb_B)
    gsum = g[N].sum(axis=1)
    h0 = (inst.omega[None, :] * (N + 0.5)).sum(axis=1)
    rows, cols, vals = [], [], []
    for s in range(2):
        rows.append(s * ncs + np.arange(ncs))
        cols.append(s * ncs + np.arange(ncs))
        vals.append(h0 + inst.E[s])
    ar = np.arange(ncs)

    def shifted(mods, shifts):
        M = N.copy()
        ok = np.ones(ncs, dtype=bool)
        jl = gsum.copy()
        for i, d in zip(mods, shifts):
            m = N[:, i] + d
            ok &= (m >= 0) & (m <= nmax)
            mc = np.clip(m, 0, nmax)
            jl = jl - g[N[:, i]] + np.maximum(g[N[:, i]], g[mc])
            M[:, i] = mc
        keep = ok & (jl <= L)
        return ar[keep], M[keep]

    def add(block_rows, block_cols, r, M, v):
        rows.append(block_rows * ncs + r)
        cols.append(block_cols * ncs + rk.rank(M))
        vals.append(v)

    for i in range(D):
        for d in (-1, 1):
            r, M = shifted([i], [d])
            if r.size == 0:
                continue
            q = Q1[N[r, i], M[:, i]]
            for s in range(2):
                if inst.kappa[s, i] != 0.0:
                    add(s, s, r, M, inst.kappa[s, i] * q)
            if inst.lam[i] != 0.0:
                add(0, 1, r, M, inst.lam[i] * q)
                add(1, 0, r, M, inst.lam[i] * q)
    for s in range(2):
        for i in range(D):
            for j in range(i + 1, D):
                c = inst.c2[s, i, j]
                if c == 0.0:
                    continue
                for di in (-2, 0, 2):
                    for dj in (-2, 0, 2):
                        r, M = shifted([i, j], [di, dj])
                        if r.size:
                            add(s, s, r, M, c * Q2[N[r, i], M[:, i]] * Q2[N[r, j], M[:, j]])
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(2 * ncs, 2 * ncs)).tocsr()
    H.sum_duplicates()
    return H


def masked_apply(inst, psi: np.ndarray, compact: np.ndarray) -> np.ndarray:
    """Route 2 without assembling the matrix (same sums as masked_matrix), for
    large cases: psi [2, N_cs] -> [2, N_cs].  Shifted tuples are located by
    binary search of their base-(nmax+1) codes, which increase in the
    lexicographic compact order."""
    D, L = inst.D, inst.L
    N = np.asarray(compact, dtype=np.int64)
    ncs = N.shape[0]
    nmax = int(N.max()) if ncs else 0
    weights = (nmax + 1) ** np.arange(D - 1, -1, -1, dtype=np.int64)
    codes = N @ weights
    if ncs > 1 and not np.all(np.diff(codes) > 0):
        raise ValueError("compact tuples are not in lexicographic order")
    Q1, Q2 = _one_mode_elements(nmax)
    g = lowest_level(np.arange(nmax + 3), inst.nb_A, inst.nb_B)
    gsum = g[N].sum(axis=1)
    psi = np.asarray(psi, dtype=np.complex128).reshape(2, ncs)
    h0 = (inst.omega[None, :] * (N + 0.5)).sum(axis=1)
    out = np.stack([(h0 + inst.E[s]) * psi[s] for s in range(2)])
    ar = np.arange(ncs)

    def shifted(mods, shifts):
        ok = np.ones(ncs, dtype=bool)
        jl = gsum.copy()
        code = codes.copy()
        for i, d in zip(mods, shifts):
            m = N[:, i] + d
            ok &= (m >= 0) & (m <= nmax)
            mc = np.clip(m, 0, nmax)
            jl = jl - g[N[:, i]] + np.maximum(g[N[:, i]], g[mc])
            code = code + d * weights[i]
        keep = ok & (jl <= L)
        r = ar[keep]
        cols = np.searchsorted(codes, code[keep])
        assert np.array_equal(codes[cols], code[keep])
        return r, cols

    for i in range(D):
        for d in (-1, 1):
            r, cols = shifted([i], [d])
            if r.size == 0:
                continue
            q = Q1[N[r, i], N[cols, i]]
            for s in range(2):
                if inst.kappa[s, i] != 0.0:
                    out[s, r] += inst.kappa[s, i] * q * psi[s, cols]
            if inst.lam[i] != 0.0:
                out[0, r] += inst.lam[i] * q * psi[1, cols]
                out[1, r] += inst.lam[i] * q * psi[0, cols]
    for s in range(2):
        for i in range(D):
            for j in range(i + 1, D):
                c = inst.c2[s, i, j]
                if c == 0.0:
                    continue
                for di in (-2, 0, 2):
                    for dj in (-2, 0, 2):
                        r, cols = shifted([i, j], [di, dj])
                        if r.size:
                            out[s, r] += (c * Q2[N[r, i], N[cols, i]] * Q2[N[r, j], N[cols, j]]
                                          * psi[s, cols])
    return out


def brute_force_masked(inst, compact: np.ndarray, mask: bool = True) -> np.ndarray:
    """Dense 2 N_cs x 2 N_cs H_S from the full direct-product Galerkin matrix
    (basis nb(L)^D, grid nq(L)^D, quadrature exact) of each block, masked by
    the joint level.  Independent of the term set."""
    D, L = inst.D, inst.L
    nb = size_of_level(L, inst.nb_A, inst.nb_B)
    nq = size_of_level(L, inst.nq_A, inst.nq_B)
    x, w, wt = gauss_hermite(nq)
    b = hermite_functions(nb, x)
    d2 = hermite_second_derivatives(nb, x)
    V00, V11, V01 = surface_potentials(inst, [x] * D)
    Vh = harmonic_on_grid(inst, [x] * D).reshape(-1, order="F")
    W = np.ones(1)
    Phi = np.ones((1, 1))
    for _ in range(D):
        W = np.kron(wt, W)
        Phi = np.kron(b, Phi)
    K = np.zeros((Phi.shape[1], Phi.shape[1]))
    for i in range(D):
        Pi = np.ones((1, 1))
        for j in range(D):
            Pi = np.kron(d2 if j == i else b, Pi)
        K += -0.5 * inst.omega[i] * (Phi.T @ (W[:, None] * Pi))
    blocks = {}
    for key, V in (("00", V00), ("11", V11), ("01", V01)):
        Vf = V.reshape(-1, order="F") + (Vh if key != "01" else 0.0)
        blocks[key] = Phi.T @ ((W * Vf)[:, None] * Phi) + (K if key != "01" else 0.0)
    pos = np.zeros(compact.shape[0], dtype=np.int64)
    stride = 1
    for i in range(D):
        pos += compact[:, i] * stride
        stride *= nb
    sel = {k: v[np.ix_(pos, pos)] for k, v in blocks.items()}
    if mask:
        g = lowest_level(np.arange(nb), inst.nb_A, inst.nb_B)
        gn = g[compact]
        joint = np.maximum(gn[:, None, :], gn[None, :, :]).sum(axis=2)
        sel = {k: np.where(joint <= L, v, 0.0) for k, v in sel.items()}
    return np.block([[sel["00"], sel["01"]], [sel["01"].T, sel["11"]]])
