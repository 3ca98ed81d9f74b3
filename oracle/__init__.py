"""FP64 CPU oracle for Coherent Point Drift and Fast Coherent Point Drift.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the test-suite, the smoke check and the benchmark's
CPU-baseline leg do.  It shares no code with the HIP path.

Modules
  cpd64   E-step (eq. 4-5), Fast M-step (eq. 17 / 20), inverse-based M-step
          (eq. 15), original CPD M-step (eq. 21), sigma^2 (eq. 18), the EM
          loops, RMSE (eq. 22), log-likelihood (eq. 3).
  eig64   Gram matrix (eq. 11), full eigendecomposition (eq. 16), randomized
          top-K eigenpairs (eq. 19).
"""
from . import cpd64, eig64  # noqa: F401
