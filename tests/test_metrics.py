"""Pins of the agreement statistics (MAE, Spearman rho, Chatterjee xi)."""
import numpy as np
from scipy import stats

from paper_2606_06329_amd import metrics


def test_spearman_matches_scipy_with_ties():
    rng = np.random.default_rng(0)
    a = rng.integers(0, 20, 300).astype(float)
    b = a + rng.normal(0, 3, 300)
    assert abs(metrics.spearman(a, b) - stats.spearmanr(a, b)[0]) < 1e-12


def test_chatterjee_closed_forms():
    n = 1000
    x = np.arange(n, dtype=float)
    # y a strictly increasing function of x: xi = 1 - 3 (n-1)/(n^2-1) = 1 - 3/(n+1)
    assert abs(metrics.chatterjee_xi(x, x ** 3) - (1 - 3 / (n + 1))) < 1e-12
    # y a non-monotone function of x is still fully dependent: xi close to 1
    assert metrics.chatterjee_xi(x, (x - n / 2) ** 2) > 0.98
    # independent y: xi close to 0 (sd ~ sqrt(2/(5n)))
    y = np.random.default_rng(1).permutation(n).astype(float)
    assert abs(metrics.chatterjee_xi(x, y)) < 5 * np.sqrt(2 / (5 * n))


def test_mae():
    assert metrics.mae([1, 2, 3], [1, 3, 5]) == 1.0
