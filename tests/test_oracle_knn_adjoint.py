"""Pins of the oracle's kNN (Step 1, eq. knn) and of its float64 gradient."""
import numpy as np
import pytest
from scipy.spatial.distance import cdist

from oracle import adjoint as oa
from oracle import curvature as oc
from oracle import knn as ok
from paper_2606_06329_amd import synth


def test_knn_vs_full_sort():
    """Against a full distance matrix from scipy's cdist, sorted by (d2, index)."""
    X = synth.swissroll(n=1500, m=32, seed=77).astype(np.float64)
    k = 12
    idx, d2, gap, _ = ok.knn(X, k)
    D = cdist(X, X, "sqeuclidean")
    np.fill_diagonal(D, np.inf)
    for i in range(0, 1500, 7):
        order = np.lexsort((np.arange(1500), D[i]))[:k]
        if gap[i] > 1e-9 * D[i][order[-1]]:
            assert set(order) == set(idx[i])
        assert np.allclose(np.sort(D[i])[:k], d2[i], rtol=1e-9, atol=1e-12)


def test_knn_brute_force_tiny_with_ties():
    """Pure-Python brute force on a tiny grid with many exact ties: ties go to the smaller index."""
    pts = np.array([[x, y] for x in range(4) for y in range(4)], dtype=np.float64)
    k = 5
    idx, d2, gap, _ = ok.knn(pts, k)
    for i in range(len(pts)):
        cand = []
        for j in range(len(pts)):
            if j != i:
                d = sum((pts[i][a] - pts[j][a]) ** 2 for a in range(2))
                cand.append((d, j))
        cand.sort()
        assert [j for _, j in cand[:k]] == list(idx[i])


def test_knn_include_self_and_duplicates():
    X = np.array([[0.0, 0.0], [0.0, 0.0], [1.0, 0.0], [3.0, 0.0], [0.0, 2.0]])
    idx, d2, _, _ = ok.knn(X, 2)
    assert list(idx[0]) == [1, 2] and d2[0][0] == 0.0       # duplicate is a valid neighbour
    idx_s, _, _, _ = ok.knn(X, 3, include_self=True)
    assert list(idx_s[3]) == [3, 2, 0]


def test_fp32_gap_bound_is_sound():
    """Float32 difference-form distances never reorder pairs whose gap exceeds the bound."""
    rng = np.random.default_rng(0)
    m = 64
    x = rng.standard_normal(m).astype(np.float32)
    ys = (x[None, :] + 0.3 * rng.standard_normal((400, m))).astype(np.float32)
    d64 = ((ys.astype(np.float64) - x.astype(np.float64)) ** 2).sum(1)
    d32 = ((ys - x) ** 2).astype(np.float32).sum(1, dtype=np.float32)
    bound = ok.fp32_gap_bound(m, d64)
    assert np.all(np.abs(d32.astype(np.float64) - d64) <= 0.5 * bound)


@pytest.fixture(scope="module")
def small_problem():
    X = synth.swissroll(n=300, m=10, seed=99).astype(np.float64)
    k = 6
    idx, _, _, _ = ok.knn(X, k)
    w = synth.loss_weights(300, seed=5).astype(np.float64)
    return X, idx, w


@pytest.mark.parametrize("variant", ["paper", "haar"])
def test_torch_forward_matches_numpy(small_problem, variant):
    X, idx, w = small_problem
    import torch
    kt = oa.fast_kappa_torch(torch.tensor(X), idx[:40], variant).numpy()
    kn = np.array([oc.fast_kappa(oc.patch(X, idx[i]), variant) for i in range(40)])
    assert np.allclose(kt, kn, rtol=1e-11, atol=0)


@pytest.mark.parametrize("variant", ["paper", "haar"])
def test_gradient_identities(small_problem, variant):
    """Euler (degree-2 homogeneity): sum_j <x_j, dL/dx_j> = 2L; translation: sum_j dL/dx_j = 0."""
    X, idx, w = small_problem
    L, g = oa.loss_and_grad(X, idx, w, variant)
    assert abs(np.sum(X * g) - 2 * L) <= 1e-9 * np.sum(np.abs(X * g))
    assert np.linalg.norm(g.sum(0)) <= 1e-9 * np.abs(g).sum()


def test_self_gradient_zero(small_problem):
    """A point is not in its own patch, so d kappa_i / d x_i = 0 with the lists fixed."""
    X, idx, w = small_problem
    e = np.zeros(X.shape[0])
    e[17] = 1.0
    _, g = oa.loss_and_grad(X, idx, e, "haar")
    assert np.all(g[17] == 0.0)
    assert np.all(np.abs(g[idx[17]]).sum(1) > 0)


@pytest.mark.parametrize("variant", ["paper", "haar"])
def test_gradient_central_differences(small_problem, variant):
    """Central finite differences in float64 (h = 1e-6) on sampled coordinates."""
    X, idx, w = small_problem
    L, g = oa.loss_and_grad(X, idx, w, variant)
    rng = np.random.default_rng(3)
    h = 1e-6
    for _ in range(12):
        i, a = rng.integers(0, X.shape[0]), rng.integers(0, X.shape[1])
        Xp = X.copy(); Xp[i, a] += h
        Xm = X.copy(); Xm[i, a] -= h
        Lp = sum(w[r] * oc.fast_kappa(oc.patch(Xp, idx[r]), variant) for r in range(X.shape[0]))
        Lm = sum(w[r] * oc.fast_kappa(oc.patch(Xm, idx[r]), variant) for r in range(X.shape[0]))
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[i, a]) <= 1e-6 * max(1.0, abs(g[i, a])) + 1e-8 * abs(L) / h
