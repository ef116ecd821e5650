"""Brute-force k nearest neighbours in float64 (test infrastructure only).

Definition followed: Step 1 of the method ("Local neighborhood construction",
eq. knn) and the kNN-graph step of Algorithm 1: the k Euclidean nearest
neighbours of each point.  Readings taken where the paper is silent:

* a point is not its own neighbour (the patch holds k *other* points);
* ties are broken by the smaller index, so the ordered list is unique;
* the graph is directed (each patch has exactly k rows).

Distances are the difference form sum_a (x_a - y_a)^2 evaluated in float64.
"""
from __future__ import annotations

import numpy as np

__all__ = ["knn_rows", "knn", "fp32_gap_bound"]


def _row_d2(X: np.ndarray, i: int) -> np.ndarray:
    diff = X - X[i][None, :]
    return np.einsum("ja,ja->j", diff, diff)


def knn_rows(X, rows, k: int, include_self: bool = False):
    """Exact kNN of the query rows ``rows`` against all of X.

    Returns (idx [len(rows), k] int64 ascending by (d2, j), d2 [len(rows), k],
    gap [len(rows)] = d2_(k+1) - d2_(k), d2next [len(rows)] = d2_(k+1)).
    With ``include_self`` the point itself is the first neighbour and k-1
    others follow.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.asarray(rows, dtype=np.int64)
    kk = k - 1 if include_self else k
    if kk < 1 or kk > n - 1:
        raise ValueError("k out of range")
    idx = np.empty((len(rows), k), dtype=np.int64)
    d2 = np.empty((len(rows), k), dtype=np.float64)
    gap = np.full(len(rows), np.inf)
    d2next = np.full(len(rows), np.inf)
    allj = np.arange(n)
    for r, i in enumerate(rows):
        d = _row_d2(X, int(i))
        others = allj[allj != i]
        dd = d[others]
        order = np.lexsort((others, dd))  # primary key d2, secondary key index
        sel = others[order[:kk]]
        if include_self:
            idx[r, 0] = i
            d2[r, 0] = 0.0
            idx[r, 1:] = sel
            d2[r, 1:] = d[sel]
        else:
            idx[r] = sel
            d2[r] = d[sel]
        if len(order) > kk:
            d2next[r] = dd[order[kk]]
            gap[r] = d2next[r] - dd[order[kk - 1]]
    return idx, d2, gap, d2next


def knn(X, k: int, include_self: bool = False):
    """Exact kNN of every point (n up to a few thousand: O(n^2 m) difference form)."""
    X = np.asarray(X, dtype=np.float64)
    return knn_rows(X, np.arange(X.shape[0]), k, include_self)


def fp32_gap_bound(m: int, d2next):
    """Gap below which float32 rounding may reorder the k-th and (k+1)-th neighbour.

    A difference-form distance sum_a (x_a - y_a)^2 of float32 inputs evaluated in
    float32 (any summation order) has relative error at most gamma_{m+2}, with
    gamma_j = j u / (1 - j u), u = 2^-24 (standard forward error bound of a sum of
    squares).  Two distances whose gap exceeds 2 gamma_{m+2} d2_(k+1) therefore
    keep their order.
    """
    u = 2.0 ** -24
    j = m + 2
    gam = j * u / (1.0 - j * u)
    return 2.0 * gam * np.asarray(d2next)
