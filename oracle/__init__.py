"""Plain complex128 CPU oracle for the RAS-PML GMRES hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls anything in this package.  Only the
test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.

The oracle follows the paper "Massively parallel Schwarz methods for the high
frequency Helmholtz equation" (Xie, Gong, Graham, Spence, Zhang):

* ``geometry``  -- mesh, Cartesian covering, PML extension, partition of unity
                   (Section 2, "Cartesian covering").
* ``fem``       -- PML stretch, P1 element assembly of the global and local
                   operators, impedance terms (Section 1 eq. (pml)/(weak),
                   Section 2 local scaling, Section 3 (ii) eq. (impedance)).
* ``band``      -- banded LU without pivoting and triangular solves (plain C
                   core in ``bandlu.c``), the local solver.
* ``ras``       -- the RAS-PML preconditioner B^{-1} = sum_j R~_j^T A_j^{-1} R_j
                   (Section 2, discrete RAS, eq. (local-ras-discrete)/(update1)).
* ``gmres``     -- restarted right-preconditioned GMRES(m) with modified
                   Gram-Schmidt and complex Givens rotations (Section 4.1).
* ``richardson``-- the preconditioner used as a fixed-point iteration
                   (Algorithm 1).
* ``warmstart`` -- the learned warm start's convolutional encoder-decoder,
                   its hand-derived gradient and Adam (float64).

Everything is complex128 / float64 and deliberately unoptimised.
"""
