"""MI355X-native (gfx950) fast mean-curvature estimator (arXiv 2606.06329, Algorithm 1).

The compute path is libmecuco.so (hand-written HIP kernels behind a C ABI,
include/mecuco.h); this package only marshals torch tensors onto it.
Importing the package does not load the library; the first call does, and
fails loudly if it has not been built.
"""
from .api import (MeanCurvature, curvature, curvature_backward, curvature_exact,  # noqa: F401
                  curvature_fast, default_k, default_rerank, exact_supported, knn,
                  knn_symmetric, normalize_minmax, workspace_bytes)
