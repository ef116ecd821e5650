"""Agreement statistics the paper uses to compare two curvature vectors.

The paper's Section "Computational Experiments and Results" compares score vectors by
the mean absolute error, Spearman's rank correlation and Chatterjee's xi.  Host-side
NumPy on output vectors; none of the hot path runs here.
"""
from __future__ import annotations

import numpy as np

__all__ = ["mae", "spearman", "chatterjee_xi", "agreement"]


def mae(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.mean(np.abs(a - b)))


def _ranks(v):
    """Average ranks (1-based), ties sharing the mean of their positions."""
    v = np.asarray(v, dtype=np.float64)
    order = np.argsort(v, kind="mergesort")
    r = np.empty(len(v))
    sv = v[order]
    i = 0
    while i < len(v):
        j = i
        while j + 1 < len(v) and sv[j + 1] == sv[i]:
            j += 1
        r[order[i:j + 1]] = 0.5 * (i + j) + 1.0
        i = j + 1
    return r


def spearman(a, b) -> float:
    """Pearson correlation of the average ranks."""
    ra, rb = _ranks(a), _ranks(b)
    ra -= ra.mean()
    rb -= rb.mean()
    den = np.sqrt(np.sum(ra * ra) * np.sum(rb * rb))
    return float(np.sum(ra * rb) / den) if den > 0 else float("nan")


def chatterjee_xi(x, y) -> float:
    """Chatterjee's xi_n(x, y) without ties in x: sort by x, r_i = #{j: y_j <= y_(i)},
    xi = 1 - 3 sum |r_{i+1} - r_i| / (n^2 - 1)."""
    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n = len(x)
    ys = y[np.argsort(x, kind="mergesort")]
    r = np.searchsorted(np.sort(ys), ys, side="right").astype(np.float64)
    return float(1.0 - 3.0 * np.sum(np.abs(np.diff(r))) / (n * n - 1.0))


def agreement(ref, est) -> dict:
    """MAE, Spearman rho and Chatterjee xi of `est` against `ref` (the paper's three criteria)."""
    return {"mae": mae(ref, est), "spearman": spearman(ref, est), "xi": chatterjee_xi(ref, est)}
