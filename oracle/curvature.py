"""Float64 reference curvature estimators (test infrastructure only).

Each function restates one definition of the paper in plain NumPy/SciPy:

* ``patch``                  local centring (Step 2 and the Fast branch of Algorithm 1)
* ``covariance``             eq. cov, Sigma = X_c^T X_c / (k-1)
* ``naive_kappa``            eqs. H and curvature: |tr(-H H^T Sigma)| with H built explicitly, O(m^4)
* ``identity_kappa``         Theorem 1: |1/2 v^T (C o C) 1 + 1/2 sum v|, C = W^T (W o W)
* ``fast_terms`` / ``fast_kappa``
                             Fast branch of Algorithm 1 (truncated SVD, t_range, t_A,
                             t_B, t_null, eq. fast_curv), in two readings of the
                             null-space term (see below); ``fast_terms_with_basis`` takes
                             the range basis as given
* ``dense_haar_tnull``       eq. gnull_exp summed against Sigma directly, O(m^2)
* ``kappa_with_null_basis``  Theorem 1 with W = [V_r | a chosen null basis]
* ``canonical_exact_kappa``  the same with the Householder (LAPACK geqrf/orgqr)
                             completion of V_r as null basis
* ``lapack_exact_kappa``     the Exact branch of Algorithm 1 with LAPACK's eigh basis
* ``monte_carlo_tnull``      average of the exact null term over Haar-random null bases

Two readings of the Fast null-space term
----------------------------------------
``paper``: Algorithm 1 and eqs. tnull/tA/tB as printed:
    t_B = tau - 2 ||X_c V_r||_F^2/(k-1) + ||G||_F^2/(k-1),  t_null = (t_A + 2 t_B)/(D - p).
``haar``: the exact expectation of the null term under eq. gnull_exp.  Summing
    eq. gnull_exp against Sigma gives (d_P^T Sigma d_P + 2 sum_ab Sigma_ab P_ab^2)/(D-p+2),
    and with P o P = I - 2 diag(M) + M o M (M = V_r V_r^T) the middle term becomes
    sum_{j,a} X_c[j,a]^2 h_a/(k-1), h = (V_r o V_r) 1, instead of the printed
    ||X_c V_r||_F^2/(k-1) (which always equals tau because every row of X_c lies
    in the range of V_r), and the denominator is D-p+2.

Rank handling (the paper keeps p = k-1 columns without comment): the numerical
rank is p_eff = #{l <= p : s_l > max(k, m) * eps64 * s_1}; p_eff columns are
used and q = m - p_eff.  q = 0 means there is no null space and t_null = 0.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg

__all__ = [
    "patch", "covariance", "eig_desc", "build_H", "naive_kappa", "identity_kappa",
    "rank_eff", "fast_terms", "fast_terms_with_basis", "fast_kappa", "dense_haar_tnull", "kappa_with_null_basis",
    "householder_null_basis", "canonical_exact_kappa", "lapack_exact_kappa",
    "monte_carlo_tnull", "range_basis", "curvature_all", "minmax_normalise", "KAPPA_VARIANTS",
]

KAPPA_VARIANTS = ("paper", "haar")
EPS64 = np.finfo(np.float64).eps


def patch(X, nbr) -> np.ndarray:
    """Centred patch X_c = [x_j - xbar]_{j in N_i} (k x m), xbar the neighbour mean."""
    P = np.asarray(X, dtype=np.float64)[np.asarray(nbr)]
    return P - P.mean(axis=0, keepdims=True)


def covariance(Xc) -> np.ndarray:
    """Local covariance Sigma = X_c^T X_c / (k-1) (eq. cov)."""
    k = Xc.shape[0]
    return Xc.T @ Xc / (k - 1)


def eig_desc(S):
    """Eigenpairs of a symmetric matrix with eigenvalues in decreasing order (eq. spectral)."""
    v, W = np.linalg.eigh(S)
    order = np.argsort(v)[::-1]
    return v[order], W[:, order]


def build_H(W) -> np.ndarray:
    """Feature matrix H = [W o W | (w_j o w_l)_{j<l}] (eq. H), m x (m + m(m-1)/2)."""
    m = W.shape[1]
    sq = [W[:, l] * W[:, l] for l in range(m)]
    cross = [W[:, j] * W[:, l] for j, l in itertools.combinations(range(m), 2)]
    return np.stack(sq + cross, axis=1)


def naive_kappa(Sigma, W) -> float:
    """kappa = |tr(-H H^T Sigma)| with H formed explicitly (eq. curvature); O(m^4)."""
    H = build_H(W)
    return abs(-np.trace(H @ H.T @ Sigma))


def identity_kappa(W, v) -> float:
    """Theorem 1: kappa = |1/2 v^T (C o C) 1 + 1/2 sum(v)|, C = W^T (W o W)."""
    C = W.T @ (W * W)
    return abs(0.5 * v @ (C * C).sum(axis=1) + 0.5 * v.sum())


def rank_eff(s, k: int, m: int) -> int:
    """Numerical rank among the first p = k-1 singular values (reading of an unstated rule)."""
    p = min(k - 1, len(s))
    if p == 0 or s[0] == 0.0:
        return 0
    tol = max(k, m) * EPS64 * s[0]
    return int(np.count_nonzero(s[:p] > tol))


def range_basis(Xc):
    """Truncated SVD of the centred patch (Fast branch): (V_r m x p_eff, s_r, p_eff)."""
    k, m = Xc.shape
    _, s, Vt = np.linalg.svd(Xc, full_matrices=False)
    pe = rank_eff(s, k, m)
    return Vt[:pe].T, s[:pe], pe


def fast_terms(Xc) -> dict:
    """Every term of the Fast branch of Algorithm 1 for one centred patch.

    Returns tau, t_range, t_A, t_S (= ||X_c V_r||^2/(k-1)), g (= ||G||^2/(k-1)),
    t_D (= sum X_c^2 h/(k-1)), p_eff, q, and both kappa readings.
    """
    Vr, s, pe = range_basis(Xc)
    return fast_terms_with_basis(Xc, Vr, s)


def fast_terms_with_basis(Xc, Vr, s) -> dict:
    """The Fast branch's terms for a given orthonormal basis V_r (m x p_eff) of the patch's row
    space with singular values s.  The truncated SVD fixes V_r up to rotations inside groups of
    equal singular values; only t_range reads individual columns, the other terms depend on
    the projector V_r V_r^T alone."""
    k, m = Xc.shape
    pe = Vr.shape[1]
    lam = s ** 2 / (k - 1)                      # non-zero eigenvalues lambda_r
    tau = lam.sum()                             # tau = lambda_r^T 1
    V2 = Vr * Vr
    t_range = np.sum((Xc @ V2) ** 2) / (k - 1)  # ||X_c V_r^{o2}||_F^2/(k-1)
    h = V2.sum(axis=1)                          # (V_r o V_r) 1
    dP = 1.0 - h                                # diag of P_perp
    t_A = np.sum((Xc @ dP) ** 2) / (k - 1)      # ||X_c d_P||^2/(k-1)
    t_S = np.sum((Xc @ Vr) ** 2) / (k - 1)      # ||X_c V_r||_F^2/(k-1)
    G = np.einsum("ja,al,ab->jlb", Xc, Vr, Vr)  # G_tens, k x p x p
    g = np.sum(G * G) / (k - 1)
    t_D = np.sum(Xc * Xc * h[None, :]) / (k - 1)
    q = m - pe
    if q > 0:
        t_null_paper = (t_A + 2.0 * (tau - 2.0 * t_S + g)) / q
        t_null_haar = (t_A + 2.0 * (tau - 2.0 * t_D + g)) / (q + 2)
    else:
        t_null_paper = 0.0
        t_null_haar = 0.0
    return dict(
        tau=tau, t_range=t_range, t_A=t_A, t_S=t_S, g=g, t_D=t_D, p_eff=pe, q=q,
        s=s, t_null_paper=t_null_paper, t_null_haar=t_null_haar,
        kappa_paper=abs(0.5 * (t_range + t_null_paper) + 0.5 * tau),
        kappa_haar=abs(0.5 * (t_range + t_null_haar) + 0.5 * tau),
    )


def fast_kappa(Xc, variant: str = "paper") -> float:
    """Fast-mode curvature (eq. fast_curv) in the ``paper`` or ``haar`` reading."""
    if variant not in KAPPA_VARIANTS:
        raise ValueError(variant)
    return fast_terms(Xc)["kappa_" + variant]


def dense_haar_tnull(Xc) -> float:
    """E[t_null] = sum_ab Sigma_ab (P_aa P_bb + 2 P_ab^2)/(q+2), P = I - V_r V_r^T (eq. gnull_exp)."""
    k, m = Xc.shape
    Vr, _, pe = range_basis(Xc)
    q = m - pe
    if q == 0:
        return 0.0
    P = np.eye(m) - Vr @ Vr.T
    d = np.diag(P)
    E = (np.outer(d, d) + 2.0 * P * P) / (q + 2)
    return float(np.sum(covariance(Xc) * E))


def kappa_with_null_basis(Xc, N) -> float:
    """Theorem 1 on W = [V_r | N] with eigenvalues [lambda_r, 0, ...]; N an orthonormal null basis."""
    k, m = Xc.shape
    Vr, s, pe = range_basis(Xc)
    W = np.concatenate([Vr, N], axis=1)
    v = np.concatenate([s ** 2 / (k - 1), np.zeros(m - pe)])
    return identity_kappa(W, v)


def householder_null_basis(Vr) -> np.ndarray:
    """Trailing m - p columns of the Householder QR of V_r (LAPACK geqrf + orgqr convention)."""
    m, p = Vr.shape
    Q, _ = scipy.linalg.qr(Vr, mode="full")
    return Q[:, p:]


def canonical_exact_kappa(Xc) -> float:
    """Exact-mode curvature with the canonical (Householder) completion of V_r as null basis."""
    Vr, _, _ = range_basis(Xc)
    return kappa_with_null_basis(Xc, householder_null_basis(Vr))


def lapack_exact_kappa(Xc) -> float:
    """Exact branch of Algorithm 1: eigh of Sigma, then Theorem 1 (null basis as LAPACK returns it)."""
    v, W = eig_desc(covariance(Xc))
    return identity_kappa(W, v)


def monte_carlo_tnull(Xc, n_draws: int, rng: np.random.Generator):
    """Exact null term of Theorem 1 for Haar-random null bases N R, R ~ Haar(O(q)).

    Returns the per-draw values of t_null^W = sum_{l>p} ||X_c (w_l o w_l)||^2/(k-1).
    """
    k, m = Xc.shape
    Vr, _, pe = range_basis(Xc)
    N0 = householder_null_basis(Vr)
    q = m - pe
    out = np.empty(n_draws)
    for t in range(n_draws):
        g = rng.standard_normal((q, q))
        R, r = np.linalg.qr(g)
        R *= np.sign(np.diag(r))[None, :]
        N = N0 @ R
        out[t] = np.sum((Xc @ (N * N)) ** 2) / (k - 1)
    return out


def curvature_all(X, idx, mode: str = "fast", variant: str = "paper", rows=None) -> np.ndarray:
    """Curvature of every point (or of ``rows``) from its neighbour list idx[i] (n x k).

    mode: "fast" (Algorithm 1 Fast branch), "canonical" (Theorem 1, Householder null
    basis), "lapack" (Theorem 1, eigh basis) or "naive" (explicit H).
    """
    X = np.asarray(X, dtype=np.float64)
    idx = np.asarray(idx)
    rows = np.arange(idx.shape[0]) if rows is None else np.asarray(rows)
    out = np.empty(len(rows))
    for r, i in enumerate(rows):
        Xc = patch(X, idx[i])
        if mode == "fast":
            out[r] = fast_kappa(Xc, variant)
        elif mode == "canonical":
            out[r] = canonical_exact_kappa(Xc)
        elif mode == "lapack":
            out[r] = lapack_exact_kappa(Xc)
        elif mode == "naive":
            v, W = eig_desc(covariance(Xc))
            out[r] = naive_kappa(covariance(Xc), W)
        else:
            raise ValueError(mode)
    return out


def minmax_normalise(kappa) -> np.ndarray:
    """Per-dataset min-max normalisation of curvature scores to [0, 1] (the normalised-score
    experiment): (kappa - min) / (max - min) over the finite scores; NaN stays NaN, a constant
    vector maps to 0."""
    k = np.asarray(kappa, dtype=np.float64)
    fin = np.isfinite(k)
    out = np.full(k.shape, np.nan)
    if not fin.any():
        return out
    lo, hi = k[fin].min(), k[fin].max()
    out[fin] = 0.0 if hi == lo else (k[fin] - lo) / (hi - lo)
    return out
