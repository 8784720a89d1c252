"""Plain FP64 CPU oracle for the Stokes-IB multigrid solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the HIP library and its
Python binding) imports, links or calls this package; only the tests, the
smoke check and the CPU-baseline leg of the benchmark do.  It shares no code
with the HIP path: operators are assembled as explicit SciPy sparse matrices
from the paper's definitions, the coarse immersed-boundary operators are
formed by a literal Galerkin triple product, Schwarz subdomain matrices are
sliced out of the assembled level operator and factored with LAPACK, and the
Krylov iterations solve their small least-squares problems with
``numpy.linalg.lstsq``.

Modules (each function cites the passage of the paper it follows):

* ``delta``     - Peskin's four-point kernel (App. A.3).
* ``mac``       - staggered-grid A, G, D and the Stokes-IB operator
                  (App. A.1, Eq. matrix-impib).
* ``ib``        - interpolation J_h, spreading S_h, fibre stiffness K_h
                  (App. A.2-A.3, Sec. 5 linear fibre force).
* ``transfer``  - Raviart-Thomas velocity prolongation, its adjoint
                  restriction, pressure transfers (Sec. 3.2).
* ``hierarchy`` - level operators, Galerkin coarse IB operator (Sec. 3.1).
* ``schwarz``   - restricted additive Schwarz (Alg. 2).
* ``schur``     - Schur-complement smoother (Eq. approx-fact-Stokes-IB).
* ``krylov``    - flexible GMRES and FGMRES-wrapped smoothing (Sec. 3.3).
* ``multigrid`` - recursive V-cycle (Alg. 1) and the coarsest solve.
* ``solver``    - problem set-up, outer solve, spring-stiffness gradient.

Parity status of every function is recorded in the tests under
``tests/test_oracle_*.py``; the whole-solver iteration counts are
"parity unpinned" against the paper (its convergence figures are not
available as numbers).
"""
