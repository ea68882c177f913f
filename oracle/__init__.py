"""CPU FP64 oracle for Krylov IIF discontinuous Galerkin on sparse grids.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP library is checked against.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does,
and it shares no code with the HIP library (the only common module is the
seeded input generator, which holds none of the method's arithmetic).

Everything is float64 and written to be checked by eye against the paper
(Liu, Cheng, Chen, Zhang, "Krylov implicit integration factor discontinuous
Galerkin methods on sparse grids for high dimensional reaction-diffusion
equations", arXiv:1810.11111):

    basis       1D Legendre + Alpert multiwavelet basis      (Sec. 2.1, eqs. 2.1-2.6)
    sparsegrid  index set |l|_1 <= N, DOF count, ordering    (Sec. 2.1, eqs. 2.7-2.9)
    operator    interior-penalty operator A = -B             (Sec. 2.1, eqs. 2.10-2.11)
    project     L2 projection of initial data, L2 errors     (Sec. 2.2, Thm. 2.4)
    krylov      Arnoldi + exp(hH) e1                         (Sec. 3, eqs. 3.7-3.8)
    reaction    F(U) by finest-grid Gauss quadrature         (Sec. 4 intro; Sec. 5)
    iif         IIF2 step with implicit reaction stage       (Sec. 3, eqs. 3.3-3.5)

Every reading of a passage the paper leaves silent, ambiguous or garbled is
stated in the docstring of the function that takes it.
"""
