"""Plain, slow, FP64 CPU oracle for the Smolyak operator action and Chebyshev
propagation (ElVibRot-MPI, arXiv 2111.13655).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything under this directory: only the test suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark use it.  It shares
no code with the HIP library (no kernels, headers, tables or helpers); the only
common dependency is the seeded input generator module `sg_inputs`, which holds
none of the method's arithmetic.

Modules
-------
smolyak    term set R(l), combination coefficients D_l, compact basis, M^B,
           size counts (Sec. 2, Sec. 3, Tables 1 and 2)
hermite    Hermite-function basis and Gauss-Hermite grid tables (Sec. 2,
           eq_g_to_b / eq_b_to_g; "Hm" primitive basis of the Example subsection of Sec. 4)
action     Route 1: Alg. 1 taken literally for every term; Route 2: the
           masked-Galerkin closed form; a brute-force direct-product check
propagate  initial displaced Gaussian, Chebyshev propagator, energy/norm
quadrature Smolyak quadrature (used only as a pin of R(l) and D_l)

Parity status: every function here is pinned by tests under tests/ against
the paper's printed values (Tables 1 and 2), closed forms, invariants or
brute force, except where a docstring says "parity unpinned".
"""
