"""CPU FP64 oracle for inexact All-Floating IETI (AF-IETI) with Fast
Diagonalization local solvers (Bosy, Montardini, Sangalli, Tani,
arXiv 2001.09626).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the paper's definitions in NumPy/SciPy double precision.  Only
the test-suite, the smoke check and the CPU-baseline leg of the benchmark may
import it; the product library never calls into it and shares no code with it
(the two only read the same seeded problem dictionaries from ``workloads``).

Modules
  bspline   knot vectors, Cox-de Boor basis, Gauss rules (Section 2.1)
  patch     patch geometry, physical stiffness / load / mass (Sections 2.2, 3, 4)
  afieti    tearing (B, R, G), projections, FD, Schur, preconditioner,
            MINRES and recovery (Sections 4, 5.2, 5.2.1, Remark 1)
  geo       inexact local solvers with geometry inclusion: separable fit of
            the pulled-back coefficients, weighted pencils, diagonal
            scalings (Section 5.2.3, Remark 1)
  exact     the exact local solvers: sparse factorisations of A + D_H M and
            Dirichlet Schur complements (Section 5.1, Remark 1)
  nonconforming  knot insertion and the gluing rows of non-conforming
            nested interfaces (Section 2.2, the non-conforming test of
            Section 6)
  direct    the conforming Galerkin solve the method must reproduce (Section 3)
  adjoint   gradients of a scalar of the displacement w.r.t. load amplitudes
            and per-patch Lame parameters (not in the paper; follows from the
            symmetry of the saddle system of Section 4)

Parity status of every function is stated in its docstring; every function
is pinned by a test under ``tests/`` that does not re-type its formula.
"""
