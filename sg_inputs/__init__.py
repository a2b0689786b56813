"""Seeded synthetic workloads for the Smolyak H|psi> hot path.

This module only draws random numbers and fixes workload shapes.  It holds none
of the method's arithmetic (no term sets, tables, transforms or propagation), so
that both the CPU oracle and the GPU path can take their inputs from it without
sharing any code with each other.

The Hamiltonian family used everywhere (stand-in for the paper's Sec. 5
workloads, whose parameters the paper does not give):

    H = sum_i 0.5*omega_i*(-d^2/dQ_i^2 + Q_i^2)
        + sum_{i<j} c_ij Q_i^2 Q_j^2  [+ sum_{i<j} k_ij Q_i^2 Q_j]

omega_i ~ U(0.5, 2.0), c_ij ~ U(-0.05, 0.05), k_ij ~ U(-0.02, 0.02); the
initial state is a displaced Gaussian with shift_i ~ U(-1, 1).  The basis and
grid size maps are nb(l) = 1 + 2 l Hermite functions and nq(l) = 2 + 2 l
Gauss-Hermite points per level (the paper's N_l = A + B l, Sec. 2).

Draw order per instance, from numpy.random.default_rng(seed):
omega[D], c (i<j, row-major), k (i<j, row-major, only when the family has the
cubic term), shift[D].
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

NB_A, NB_B, NQ_A, NQ_B = 1, 2, 2, 2
DEFAULT_SEED = 0


@dataclass
class Instance:
    """One Hamiltonian + initial state.  All arrays are float64, host side."""

    D: int
    L: int
    omega: np.ndarray            # [D]
    c: np.ndarray                # [D, D], only i<j entries are non-zero
    k: np.ndarray                # [D, D], only i<j entries are non-zero
    shift: np.ndarray            # [D]
    nb_A: int = NB_A
    nb_B: int = NB_B
    nq_A: int = NQ_A
    nq_B: int = NQ_B
    meta: dict = field(default_factory=dict)


def draw_instance(rng: np.random.Generator, D: int, L: int,
                  with_k: bool = True) -> Instance:
    omega = rng.uniform(0.5, 2.0, size=D)
    c = np.zeros((D, D))
    k = np.zeros((D, D))
    iu = np.triu_indices(D, 1)
    c[iu] = rng.uniform(-0.05, 0.05, size=len(iu[0]))
    if with_k:
        k[iu] = rng.uniform(-0.02, 0.02, size=len(iu[0]))
    shift = rng.uniform(-1.0, 1.0, size=D)
    return Instance(D=D, L=L, omega=omega, c=c, k=k, shift=shift)


# ---------------------------------------------------------------------------
# The five workloads.  Index i uses seed DEFAULT_SEED + i unless overridden.
# ---------------------------------------------------------------------------

def config0(seed: int | None = None) -> Instance:
    """D=2, L=4, no cubic term; one apply + 100 Chebyshev steps of dt=0.1."""
    rng = np.random.default_rng(DEFAULT_SEED + 0 if seed is None else seed)
    inst = draw_instance(rng, 2, 4, with_k=False)
    inst.meta = dict(name="d2_l4_fp64", dt=0.1, steps=100, check_every=10,
                     precision="fp64")
    return inst


def config1(seed: int | None = None) -> Instance:
    """D=6, L=6 with cubic term; 1000 steps of dt=0.05, checks every 100."""
    rng = np.random.default_rng(DEFAULT_SEED + 1 if seed is None else seed)
    inst = draw_instance(rng, 6, 6, with_k=True)
    inst.meta = dict(name="d6_l6_fp64", dt=0.05, steps=1000, check_every=100,
                     precision="fp64")
    return inst


def config2(seed: int | None = None) -> Instance:
    """D=12, L=6 with cubic term; 500 steps of dt=0.05 in mixed precision."""
    rng = np.random.default_rng(DEFAULT_SEED + 2 if seed is None else seed)
    inst = draw_instance(rng, 12, 6, with_k=True)
    inst.meta = dict(name="d12_l6_mixed", dt=0.05, steps=500, check_every=1,
                     precision="mixed")
    return inst


def config3(seed: int | None = None, n_instances: int = 64) -> list[Instance]:
    """64 independent instances, D ~ U{4..10}, L ~ U{4..7}; 200 mixed steps."""
    rng = np.random.default_rng(DEFAULT_SEED + 3 if seed is None else seed)
    out = []
    for i in range(n_instances):
        D = int(rng.integers(4, 11))
        L = int(rng.integers(4, 8))
        inst = draw_instance(rng, D, L, with_k=True)
        inst.meta = dict(name=f"batch{i}_d{D}_l{L}", dt=0.05, steps=200,
                         precision="mixed")
        out.append(inst)
    return out


@dataclass
class Request:
    arrival_s: float
    steps: int
    inst: Instance


def config4(seed: int | None = None, rate_hz: float = 20.0,
            duration_s: float = 120.0) -> list[Request]:
    """Poisson request stream; each request draws D ~ U{3..20},
    L ~ U{3..6}, steps ~ U{50..2000}, then its Hamiltonian and shift.

    The cap on the sparse-basis size is applied by the consumer, which knows
    how to count the basis; this module only draws."""
    rng = np.random.default_rng(DEFAULT_SEED + 4 if seed is None else seed)
    t = 0.0
    reqs = []
    while True:
        t += float(rng.exponential(1.0 / rate_hz))
        if t >= duration_s:
            break
        D = int(rng.integers(3, 21))
        L = int(rng.integers(3, 7))
        steps = int(rng.integers(50, 2001))
        inst = draw_instance(rng, D, L, with_k=True)
        inst.meta = dict(name=f"req_d{D}_l{L}", dt=0.05, steps=steps,
                         precision="mixed")
        reqs.append(Request(arrival_s=t, steps=steps, inst=inst))
    return reqs


def random_state(rng: np.random.Generator, n: int) -> np.ndarray:
    """A random complex128 vector of length n with unit 2-norm."""
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    return v / np.linalg.norm(v)


def small_instance(D: int, L: int, seed: int = 123, with_k: bool = True,
                   nb=(NB_A, NB_B), nq=(NQ_A, NQ_B)) -> Instance:
    """A small seeded instance for parity tests (any D, L, size maps)."""
    rng = np.random.default_rng(seed)
    inst = draw_instance(rng, D, L, with_k=with_k)
    inst.nb_A, inst.nb_B = nb
    inst.nq_A, inst.nq_B = nq
    inst.meta = dict(name=f"small_d{D}_l{L}_s{seed}")
    return inst


# ---------------------------------------------------------------------------
# Two-state (vibronic) instances: the form of the paper's Sec. 5 pyrazine
# model (gap 2 Delta, linear interstate coupling lambda Q_1, state-dependent
# linear terms on the other modes), whose parameters the paper does not give,
# plus optional state-dependent quartic couplings of the family above.
#   H = sum_i 1/2 omega_i (-d^2/dQ_i^2 + Q_i^2) (x) 1
#       + [[V_00, V_01], [V_01, V_11]],
#   V_ss = E_s + sum_i kappa[s, i] Q_i + sum_{i<j} c2[s, i, j] Q_i^2 Q_j^2,
#   V_01 = sum_i lam[i] Q_i.
# Draw order per instance: omega[D], Delta, kappa[0, 1:], kappa[1, 1:],
# lam[0], then (quartic) c2[0] (i<j, row-major), c2[1], then shift[D].
# ---------------------------------------------------------------------------

@dataclass
class VibronicInstance:
    D: int
    L: int
    omega: np.ndarray            # [D]
    E: np.ndarray                # [2] state energies (-Delta, Delta)
    kappa: np.ndarray            # [2, D] state-dependent linear terms
    lam: np.ndarray              # [D] interstate linear coupling
    c2: np.ndarray               # [2, D, D] quartic couplings, i<j entries
    shift: np.ndarray            # [D] displacement of the initial Gaussian
    state0: int = 1              # electronic state the initial packet is on
    nb_A: int = NB_A
    nb_B: int = NB_B
    nq_A: int = NQ_A
    nq_B: int = NQ_B
    meta: dict = field(default_factory=dict)


def draw_vibronic(rng: np.random.Generator, D: int, L: int,
                  quartic: bool = True) -> VibronicInstance:
    omega = rng.uniform(0.5, 2.0, size=D)
    delta = rng.uniform(0.1, 0.5)
    kappa = np.zeros((2, D))
    kappa[0, 1:] = rng.uniform(-0.2, 0.2, size=D - 1)
    kappa[1, 1:] = rng.uniform(-0.2, 0.2, size=D - 1)
    lam = np.zeros(D)
    lam[0] = rng.uniform(0.1, 0.4)
    c2 = np.zeros((2, D, D))
    if quartic:
        iu = np.triu_indices(D, 1)
        for s in range(2):
            c2[s][iu] = rng.uniform(-0.05, 0.05, size=len(iu[0]))
    shift = rng.uniform(-1.0, 1.0, size=D)
    return VibronicInstance(D=D, L=L, omega=omega, E=np.array([-delta, delta]),
                            kappa=kappa, lam=lam, c2=c2, shift=shift)


def vibronic_small(D: int, L: int, seed: int = 321, quartic: bool = True) -> VibronicInstance:
    """A small seeded two-state instance for parity tests."""
    inst = draw_vibronic(np.random.default_rng(seed), D, L, quartic=quartic)
    inst.meta = dict(name=f"vib_d{D}_l{L}_s{seed}")
    return inst


def vibronic_pyrazine(L: int = 5, seed: int | None = None) -> VibronicInstance:
    """12 modes, the size of the paper's pyrazine propagation, with the
    pyrazine form (no quartic terms); Chebyshev steps of dt = 0.05."""
    rng = np.random.default_rng(DEFAULT_SEED + 5 if seed is None else seed)
    inst = draw_vibronic(rng, 12, L, quartic=False)
    inst.meta = dict(name=f"vib_pyrazine_d12_l{L}", dt=0.05)
    return inst


# ---------------------------------------------------------------------------
# General (non-polynomial) coupling potentials for the tabulated path.  The
# paper's systems use general potential-energy surfaces; a seeded smooth
# family of the same kind stands in for them:
#   V(Q) = sum_i a_i (1 - cos(b_i Q_i)) + sum_{i<j} g_ij exp(-(Q_i - Q_j)^2 / 2)
# with a ~ U(0.05, 0.2), b ~ U(0.5, 1.5), g ~ U(-0.05, 0.05).  Draw order:
# a[D], b[D], g (i<j, row-major).
# ---------------------------------------------------------------------------

@dataclass
class GeneralPotential:
    D: int
    a: np.ndarray
    b: np.ndarray
    g: np.ndarray                # [D, D], only i<j entries are non-zero

    def __call__(self, Q):
        """V at the points given by D coordinate arrays (broadcasting)."""
        V = 0.0
        for i in range(self.D):
            V = V + self.a[i] * (1.0 - np.cos(self.b[i] * Q[i]))
        for i in range(self.D):
            for j in range(i + 1, self.D):
                V = V + self.g[i, j] * np.exp(-0.5 * (Q[i] - Q[j]) ** 2)
        return V

    def at_points(self, P: np.ndarray) -> np.ndarray:
        """V at the rows of an (n, D) array of points."""
        return np.asarray(self([P[:, i] for i in range(self.D)]), dtype=np.float64)


def general_potential(D: int, seed: int = 777) -> GeneralPotential:
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.05, 0.2, size=D)
    b = rng.uniform(0.5, 1.5, size=D)
    g = np.zeros((D, D))
    iu = np.triu_indices(D, 1)
    g[iu] = rng.uniform(-0.05, 0.05, size=len(iu[0]))
    return GeneralPotential(D=D, a=a, b=b, g=g)


def tabulated_d8_l6(seed: int | None = None):
    """The tabulated-potential workload: D = 8, L = 6, harmonic frequencies of
    the family above and a general potential of the family above (seed
    DEFAULT_SEED + 5 for the instance, + 1005 for the potential)."""
    s = DEFAULT_SEED + 5 if seed is None else seed
    inst = draw_instance(np.random.default_rng(s), 8, 6, with_k=False)
    inst.c[:] = 0.0
    inst.meta = dict(name="tabulated_d8_l6", dt=0.05)
    return inst, general_potential(8, seed=s + 1000)
