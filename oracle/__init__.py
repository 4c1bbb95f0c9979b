"""CPU FP64 oracle for the preconditioned 2D TE CFIE (test infrastructure only).

This package is the plain, slow reference that the HIP path is checked against.  Only the
test-suite, the package's smoke check and the benchmark's CPU-baseline leg may import it;
the solver library never does, and the two share no code.

It computes the exact discrete solution of the paper's preconditioned equation directly:
dense Galerkin assembly of the boundary-element matrices with its own quadrature
(Sec. II, eq. (4); Sec. III, eq. (5)), the dense matrix C of eq. (6) formed with a dense
inverse of the Gram matrix, and a dense LU solve.  It does not run the low-rank/Woodbury
algorithm of Sec. V; that algorithm is an identity (eqs. (8)-(9)) whose result must agree
with the dense solve.

Modules:
  geometry  contour z(t), arc length, nodes uniform in arc length, accurate differences
  quadrature  Gauss-Legendre and tanh-sinh rules
  assembly  dense Galerkin matrices S, D, N (Maue form) and G
  system    C of eq. (6), the right-hand side of eq. (5), dense LU solve, circle counterpart
  diagnostics  singular values of C and C - C_c labelled by spatial frequency, exact rank
"""
from . import geometry, quadrature, assembly, system, diagnostics  # noqa: F401
