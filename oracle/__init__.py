"""CPU FP64 oracle for the hybridised Crouzeix-Raviart Stokes/Navier-Stokes solve.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import or run anything in this package.  The
solver library never calls it, shares no code with it, and must fail loudly
rather than fall back to it.

The oracle follows Chenier & Eymard, "Exact pressure elimination for the
Crouzeix-Raviart scheme applied to the Stokes and Navier-Stokes problems"
(arXiv 2101.03777):
  * Section 2 (the scheme): simplicial mesh, faces, a_{K,sigma}, the CR space,
    broken gradient/divergence, mass lumping Pi_h, the right-hand side built
    through the Raviart-Thomas reconstruction (eq. defrhs), the pinned pressure
    element K0, and the convection form b_h (eq. defbh);
  * Section 3.1: the coupled system (eq. syslin) assembled from S_K, A_K, D_K,
    R_K, solved by a sparse direct factorisation;
  * Section 3.2: the hybridised three-field system (eq. syslinhyb), the
    element-wise elimination to G W = S, and the recovery of U and P.

Everything is in float64 and written for readability, not speed.

Modules:
  cr       topology, geometry, element matrices, coupled and hybrid solves
  brute    the three-field system of eq. syslinhyb assembled densely (tiny meshes)
  norms    broken L2 / H1 error norms against a manufactured solution
  krylov   plain FP64 preconditioned CG on G (for sizes a direct solve cannot take)
  newton   Newton iterations of the nonlinear scheme (each step a coupled direct solve)

Functions whose result the tests cannot tie to the paper or to mathematics
independently of the oracle itself say "parity unpinned" in their docstring.
"""
