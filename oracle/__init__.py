"""CPU oracle for the nonsymmetric flood GaBP solver -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct FP64 implementation of what the GPU path computes, written
from the paper (arXiv 1904.04093, "Gaussian belief propagation solvers for nonsymmetric
systems of linear equations"). Only the test-suite, the smoke check and the CPU-baseline leg
of the benchmark may import it. The product path never does, and this package imports
nothing from the product package.

Modules
-------
gabp_loops  pure-Python loops over a dict of messages (small cases), Sec. 2.3 rules
gabp        vectorized numpy form of the same iteration, plus Lambda-precompute (converged,
            and per sweep from zero messages), the error-correction smoother (Alg. 3) and
            classical FP32-message iterative refinement
mg          geometric V-cycle: full-weighting restriction, bilinear interpolation,
            dense coarse solve, red-black Gauss-Seidel comparison smoother (Sec. 4)
adjoint     transposed solve and dL/dA_ij = -lambda_i x_j, dense-LU reference gradient

Parity status: every function is pinned by the CPU tests (tests/test_oracle_*.py) against
closed forms printed in the paper, theorems it states, textbook identities or library
routines, except where a docstring says "parity unpinned".
"""
