"""Plain float64 CPU oracle for the mean-curvature hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the package's smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with
the HIP path: it never imports ``paper_2606_06329_amd`` (except nothing) and
the HIP path never imports it.

Every function here follows a definition of the paper, cited in its docstring,
written plainly and slowly in NumPy / SciPy (or PyTorch CPU float64 where a
derivative is needed).  Inputs are the float32 arrays the GPU receives,
promoted to float64, so input rounding never counts as a mismatch.

Modules:
  knn        -- k nearest neighbours by brute force (Step 1, eq. knn)
  curvature  -- patch, covariance, naive H, Theorem 1 identity, fast mode
                (Algorithm 1, both null-space readings), dense Haar
                expectation, canonical exact mode, Monte-Carlo check
  adjoint    -- float64 gradient of sum_i w_i kappa_i (autograd through the
                same definitions; pinned by finite differences and identities)
"""
from . import knn, curvature  # noqa: F401
