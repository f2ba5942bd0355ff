"""CPU FP64 oracle for one Levenberg-Marquardt linear solve of multigrid bundle
adjustment (Konolige and Brown, "Multigrid for Bundle Adjustment").

THIS IS TEST INFRASTRUCTURE. Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it. The GPU library never calls it and
shares no code with it.

Modules: camera (residual, Jacobian), normal (normal blocks, Schur complement),
nullspace (16-column near-nullspace), aggregation (strength, Algorithm 2),
multigrid (QR prolongation, Galerkin, Chebyshev, Lanczos, V-cycle, PCG with the
Nash-Sofer rule), adjoint (gradient of a loss of the step), robust (Huber loss
and the reweighted step), cluster (visibility-based block Jacobi), step
(end-to-end solve), lm (the Levenberg-Marquardt outer loop).

Parity pins: every function is checked in tests/test_oracle_*.py against
closed forms, invariants, brute force or finite differences, never against a
retyped copy of itself.
"""
