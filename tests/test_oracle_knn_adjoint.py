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


def near_degenerate_patch_cloud(seed=21, n=60, m=12, k=7, rel_gap=1e-7):
    """A cloud whose first k points form a patch of full rank k-1 with a prescribed spectrum
    that holds a near-degenerate pair (singular values 3, 2, 2 (1 + rel_gap), 1.5, 1.2, 1);
    every patch is the point's k successors (cyclically), so patch 0 is points 1..k and
    patch n-1 is points 0..k-1, the prescribed one."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((n, m))
    s = np.array([3.0, 2.0, 2.0 * (1.0 + rel_gap), 1.5, 1.2, 1.0])[: k - 1]
    Uc, _ = np.linalg.qr(np.column_stack([np.ones(k), rng.standard_normal((k, k - 1))]))
    Vc, _ = np.linalg.qr(rng.standard_normal((m, k - 1)))
    X[:k] = (Uc[:, 1:] * s[None, :]) @ Vc.T + rng.standard_normal(m)[None, :]
    idx = np.array([[(i + 1 + t) % n for t in range(k)] for i in range(n)])
    return X, idx


def test_regularised_adjoint_reduces_to_exact(small_problem):
    """gap_eps = 0: the regularised reading is torch's exact eigh derivative."""
    X, idx, w = small_problem
    for variant in ("paper", "haar"):
        _, g0 = oa.loss_and_grad(X, idx, w, variant)
        _, g1 = oa.loss_and_grad(X, idx, w, variant, gap_eps=0.0)
        assert np.abs(g1 - g0).max() <= 1e-8 * np.abs(g0).max()   # K^+ through an inverse


def test_reg_eigh_matches_perturbation_theory():
    """The regularised eigen adjoint is the transpose of the first-order perturbation
    du_i = sum_{j != i} u_j (u_j^T dK u_i) Delta/(Delta^2 + eta^2), Delta = sigma_i - sigma_j,
    dsigma_i = u_i^T dK u_i, written out here in NumPy: <U_bar, dU> + <s_bar, ds> = <K_bar, dK>."""
    import torch
    rng = np.random.default_rng(4)
    for eta in (0.0, 0.05, 0.7):
        A = rng.standard_normal((6, 6))
        K = A @ A.T
        Kt = torch.tensor(K, requires_grad=True)
        sig, U = oa.reg_eigh(Kt, eta)
        Ub = rng.standard_normal((6, 6))
        sb = rng.standard_normal(6)
        (Kb,) = torch.autograd.grad((sig * torch.tensor(sb)).sum() + (U * torch.tensor(Ub)).sum(), Kt)
        s, V = np.linalg.eigh(K)
        dK = rng.standard_normal((6, 6))
        dK = dK + dK.T
        dU = np.zeros((6, 6))
        for i in range(6):
            for j in range(6):
                if j != i:
                    dlt = s[i] - s[j]
                    dU[:, i] += V[:, j] * (V[:, j] @ dK @ V[:, i]) * dlt / (dlt * dlt + eta * eta)
        ds = np.array([V[:, i] @ dK @ V[:, i] for i in range(6)])
        # eigh's sign convention is shared by torch and numpy on this input; align anyway
        sgn = np.sign(np.sum(V * U.detach().numpy(), axis=0))
        lhs = np.sum(Ub * (dU * sgn[None, :])) + sb @ ds
        rhs = np.sum(Kb.numpy() * dK)
        assert abs(lhs - rhs) <= 1e-10 * (abs(lhs) + abs(rhs) + 1.0)


def test_regularised_adjoint_converges_to_exact():
    """Well-separated eigenvalues: the regularised gradient approaches the exact one as
    eta^2 (the factor Delta/(Delta^2 + eta^2) = 1/Delta (1 - eta^2/Delta^2 + ...))."""
    X, idx = near_degenerate_patch_cloud(rel_gap=0.3)      # squared gaps >= 0.44, sigma_1 = 9
    w = np.zeros(X.shape[0])
    w[-1] = 1.0
    _, g0 = oa.loss_and_grad(X, idx, w, "haar")
    d1 = np.abs(oa.loss_and_grad(X, idx, w, "haar", gap_eps=1e-3)[1] - g0).max()
    d2 = np.abs(oa.loss_and_grad(X, idx, w, "haar", gap_eps=2e-3)[1] - g0).max()
    assert d1 > 0 and 3.5 < d2 / d1 < 4.5


@pytest.mark.parametrize("gap_eps", [1e-3, 0.1])
def test_regularised_adjoint_identities_near_degenerate(gap_eps):
    """Euler and translation identities hold for the regularised reading too (scaling and
    translating X never mix eigenvectors), also on patches with a near-degenerate pair,
    where the exact derivative is dominated by the 1/gap factor."""
    X, idx = near_degenerate_patch_cloud()
    w = synth.loss_weights(X.shape[0], seed=8).astype(np.float64)
    L, g = oa.loss_and_grad(X, idx, w, "paper", gap_eps=gap_eps)
    assert abs(np.sum(X * g) - 2 * L) <= 1e-9 * np.sum(np.abs(X * g))
    assert np.linalg.norm(g.sum(0)) <= 1e-9 * np.abs(g).sum()
    _, g_exact = oa.loss_and_grad(X, idx, w, "paper")
    assert np.abs(g_exact).max() > 10 * np.abs(g).max()    # the regularisation matters here


def test_grad_contribution_scale_bounds_gradient(small_problem):
    X, idx, w = small_problem
    _, g = oa.loss_and_grad(X, idx, w, "paper")
    S = oa.grad_contribution_scale(X, idx, w, "paper")
    assert np.all(np.abs(g) <= S * (1 + 1e-12) + 1e-300)
    assert np.all(S[np.bincount(idx.ravel(), minlength=X.shape[0]) > 0].sum(1) > 0)
