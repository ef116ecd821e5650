"""Seeded synthetic point clouds shaped like the paper's workloads.

The paper evaluates on OpenML datasets (Section "Computational Experiments and
Results"), which are not available here.  These generators stand in for them
with matching shapes (n points in R^m) and manifold structure.  They hold none
of the curvature method's arithmetic: they only draw samples.  Both the GPU
path and the CPU oracle receive the float32 arrays returned here; the oracle
promotes them to float64.

Every generator draws from ``numpy.random.default_rng(seed)`` in a fixed
order: manifold samples, then embedding parameters, then the rotation, then
the noise.  A Haar rotation is the Q factor of a QR decomposition of a
standard normal matrix with the signs of R's diagonal folded into Q.

Workloads (name, n, m, k):

* ``sphere``   500 x 20,    k=10  unit 2-sphere in R^3, padded, rotated, noise 0.01
* ``clusters`` 20000 x 784, k=11  10 latent Gaussian clusters through a quadratic chart, clipped to [0,1]
* ``torus``    100000 x 256, k=16 flat 8-torus in R^16, padded, rotated, noise 0.02
* ``swissroll`` 8192 x 128, k=12  swiss roll, padded, rotated, noise 0.01
* ``blobs``    50000 x 4096, k=32 20 Gaussian blobs on curved 16-dim charts, z-scored
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "WORKLOADS",
    "haar_rotation",
    "sphere",
    "clusters",
    "torus",
    "swissroll",
    "blobs",
    "make",
    "loss_weights",
]


def haar_rotation(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-distributed orthogonal m x m matrix (QR of a Gaussian matrix, sign-fixed)."""
    g = rng.standard_normal((m, m))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def sphere(n: int = 500, m: int = 20, seed: int = 1001, noise: float = 0.01) -> np.ndarray:
    """Uniform samples on the unit 2-sphere in R^3, zero-padded to R^m, rotated, plus noise."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n, 3))
    y = g / np.linalg.norm(g, axis=1, keepdims=True)
    ypad = np.zeros((n, m))
    ypad[:, :3] = y
    q = haar_rotation(rng, m)
    x = ypad @ q.T + noise * rng.standard_normal((n, m))
    return x.astype(np.float32)


def clusters(n: int = 20000, m: int = 784, seed: int = 2001, n_clusters: int = 10,
             d: int = 10, spread: float = 0.15) -> np.ndarray:
    """Latent Gaussian clusters in R^d mapped through a random quadratic chart into [0,1]^m.

    x_a = clip(0.5 + 0.2 * (A_a . z + 0.5 z^T B_a z), 0, 1), with A_a ~ N(0, I/d) and
    B_a = (G + G^T)/2, G_ij ~ N(0, 1/d).  Points are stored cluster after cluster.
    """
    rng = np.random.default_rng(seed)
    per = n // n_clusters
    sizes = [per] * n_clusters
    sizes[-1] += n - per * n_clusters
    centres = rng.standard_normal((n_clusters, d))
    z = np.concatenate([centres[c] + spread * rng.standard_normal((sizes[c], d))
                        for c in range(n_clusters)])
    a = rng.standard_normal((m, d)) / np.sqrt(d)
    gmat = rng.standard_normal((m, d, d)) / np.sqrt(d)
    b = 0.5 * (gmat + gmat.transpose(0, 2, 1))
    zz = (z[:, :, None] * z[:, None, :]).reshape(n, d * d)
    quad = zz @ b.reshape(m, d * d).T
    x = np.clip(0.5 + 0.2 * (z @ a.T + 0.5 * quad), 0.0, 1.0)
    return x.astype(np.float32)


def torus(n: int = 100000, m: int = 256, seed: int = 3001, d: int = 8,
          noise: float = 0.02) -> np.ndarray:
    """Flat d-torus (unit circles) in R^{2d}, zero-padded to R^m, rotated, plus noise."""
    rng = np.random.default_rng(seed)
    theta = rng.uniform(0.0, 2.0 * np.pi, size=(n, d))
    ypad = np.zeros((n, m))
    ypad[:, 0:2 * d:2] = np.cos(theta)
    ypad[:, 1:2 * d:2] = np.sin(theta)
    q = haar_rotation(rng, m)
    x = ypad @ q.T + noise * rng.standard_normal((n, m))
    return x.astype(np.float32)


def swissroll(n: int = 8192, m: int = 128, seed: int = 4001, noise: float = 0.01) -> np.ndarray:
    """Swiss roll (t in [1.5 pi, 4.5 pi], height in [0, 21]) padded to R^m, rotated, plus noise."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(1.5 * np.pi, 4.5 * np.pi, size=n)
    h = rng.uniform(0.0, 21.0, size=n)
    ypad = np.zeros((n, m))
    ypad[:, 0] = t * np.cos(t)
    ypad[:, 1] = h
    ypad[:, 2] = t * np.sin(t)
    q = haar_rotation(rng, m)
    x = ypad @ q.T + noise * rng.standard_normal((n, m))
    return x.astype(np.float32)


def blobs(n: int = 50000, m: int = 4096, seed: int = 5001, n_blobs: int = 20,
          d: int = 16) -> np.ndarray:
    """Gaussian blobs on random curved d-dimensional charts, z-scored per coordinate.

    Per blob b: x = mu_b + A_b z + 0.5 (z^T B_{b,a} z)_a with mu_b ~ N(0, I_m),
    z ~ N(0, I_d), A_b entries N(0, 1/d), B_{b,a} symmetric with entries N(0, 1/d^2).
    Every coordinate is then standardised over the whole dataset.
    """
    rng = np.random.default_rng(seed)
    per = n // n_blobs
    sizes = [per] * n_blobs
    sizes[-1] += n - per * n_blobs
    zs = [rng.standard_normal((s, d)) for s in sizes]
    x = np.empty((n, m), dtype=np.float64)
    row = 0
    for bi in range(n_blobs):
        mu = rng.standard_normal(m)
        a = rng.standard_normal((m, d)) / np.sqrt(d)
        g = rng.standard_normal((m, d, d)) / d
        bsym = 0.5 * (g + g.transpose(0, 2, 1))
        z = zs[bi]
        zz = (z[:, :, None] * z[:, None, :]).reshape(len(z), d * d)
        x[row:row + len(z)] = mu[None, :] + z @ a.T + 0.5 * (zz @ bsym.reshape(m, d * d).T)
        row += len(z)
    x -= x.mean(axis=0, keepdims=True)
    x /= x.std(axis=0, keepdims=True)
    return x.astype(np.float32)


WORKLOADS = {
    # name: (generator, n, m, k, seed)
    "sphere": (sphere, 500, 20, 10, 1001),
    "clusters": (clusters, 20000, 784, 11, 2001),
    "torus": (torus, 100000, 256, 16, 3001),
    "swissroll": (swissroll, 8192, 128, 12, 4001),
    "blobs": (blobs, 50000, 4096, 32, 5001),
}


def make(name: str, n: int | None = None, m: int | None = None, seed: int | None = None,
         rep: int = 0) -> tuple[np.ndarray, int]:
    """Generate workload ``name`` (optionally at another n, m or seed); returns (X float32, k)."""
    gen, n0, m0, k, s0 = WORKLOADS[name]
    x = gen(n=n or n0, m=m or m0, seed=(seed if seed is not None else s0) + 100 * rep)
    return np.ascontiguousarray(x), k


def loss_weights(n: int, seed: int = 4002) -> np.ndarray:
    """Weights w ~ N(0, 1) of the scalar loss sum_i w_i * kappa_i."""
    return np.random.default_rng(seed).standard_normal(n).astype(np.float32)
