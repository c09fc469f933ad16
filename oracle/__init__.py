"""Plain FP64 CPU oracle for the 5-point Laplace/Poisson solvers compared in
"A Comparison of SOR, ADI and Multigrid Methods for Solving Partial
Differential Equations" (M. M. Ahmed, arXiv:2208.02427).

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and
the bench's CPU-baseline leg may import it.  The GPU library never calls it,
links it or shares code with it; the two meet only through the seeded inputs
of the ``workloads`` package.

Every function is written for a reader to check against the paper by eye:
numpy vector operations over whole colours / lines where the method updates
them simultaneously, plain Python loops where it is sequential, no blocking or
fusion.  FP64 throughout except the explicitly float32 inner cycle of the
mixed-precision defect correction, which emulates FP32 by numpy float32
arithmetic (one rounding per operation, no fused multiply-add).

Module map
  grid       operator L_h (Eq. (2)/(11)), residual (Eq. (12)), norms, Eq. (16)
  relax      Jacobi (Eq. (5)), Gauss-Seidel (Eq. (6)), SOR (Eq. (7)), red-black SOR
  lines      Thomas algorithm, SLORA (Eqs. (8)-(9)), SLORB (Eq. (10)), ADI
  multigrid  full weighting, bilinear prolongation, coarse direct solve,
             V-cycle (Eqs. (11)-(15)), mixed-precision defect correction
  direct     dense Gaussian elimination, exact DST-I solve
  solve      drivers with the stopping rules

Parity pins: every function is pinned by the tests under tests/test_oracle_*
against closed forms, invariants, brute force and the values the paper
prints; the header of each module lists its pins.  Functions that no such pin
reaches say "parity unpinned" in their docstring.
"""
from . import grid, relax, lines, multigrid, direct, solve  # noqa: F401
