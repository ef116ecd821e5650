"""GPU adjoint (mc_curvature_backward) against the float64 autograd oracle, central finite
differences of the GPU forward, and the identities of a translation-invariant, degree-2
homogeneous loss."""
import numpy as np
import pytest

from oracle import adjoint as oa
from oracle import curvature as oc
from oracle import knn as ok
from paper_2606_06329_amd import synth
from tests.gpu_common import to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _gpu_grad(X, idx, w, variant, gap_eps=0.0):
    import paper_2606_06329_amd as P
    Xd = to_dev(X)
    idd = torch.from_numpy(np.ascontiguousarray(idx, dtype=np.int32)).cuda()
    g = P.curvature_backward(Xd, idd, torch.from_numpy(w.astype(np.float32)).cuda(), variant, gap_eps)
    kap, fl = P.curvature_fast(Xd, idd, variant)
    return g.cpu().numpy().astype(np.float64), kap.cpu().numpy().astype(np.float64), fl.cpu().numpy()


CASES = [("swissroll", 300, 10, 6, 91), ("torus", 400, 24, 8, 92), ("sphere", 500, 20, 10, 93),
         ("clusters", 300, 64, 12, 94), ("torus", 300, 40, 16, 95), ("swissroll", 200, 7, 3, 96)]


def _assert_elementwise(g, go, S, what):
    """Per element: |g - g_oracle| <= 1e-4 S + 1e-12 max S, where S sums the absolute values
    of the per-patch terms each entry adds up (the float32 scatter-add's cancellation scale)."""
    err = np.abs(g - go)
    bound = 1e-4 * S + 1e-12 * S.max()
    worst = np.unravel_index(np.argmax(err / bound), g.shape)
    print(f"  {what}: max err/bound {np.max(err / bound):.3f} at {worst}, "
          f"rel norm {np.linalg.norm(g - go) / np.linalg.norm(go):.2e}", flush=True)
    assert np.all(err <= bound)


@pytest.mark.parametrize("variant", ["paper", "haar"])
@pytest.mark.parametrize("name,n,m,k,seed", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-k{c[3]}" for c in CASES])
def test_backward_vs_oracle(name, n, m, k, seed, variant):
    """Element by element against autograd through the float64 oracle (same float32 inputs)."""
    X = synth.WORKLOADS[name][0](n=n, m=m, seed=seed)
    idx, _, _, _ = ok.knn(X.astype(np.float64), k)
    w = synth.loss_weights(n, seed=seed)
    print(f"backward {name} n={n} m={m} k={k} {variant}", flush=True)
    g, kap, fl = _gpu_grad(X, idx, w, variant)
    L, go = oa.loss_and_grad(X.astype(np.float64), idx, w.astype(np.float64), variant)
    assert not np.any(fl & 4), "rank-deficient patches in a parity case"
    S = oa.grad_contribution_scale(X.astype(np.float64), idx, w.astype(np.float64), variant)
    _assert_elementwise(g, go, S, "exact derivative")
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)


@pytest.mark.parametrize("gap_eps", [1e-3, 0.1])
@pytest.mark.parametrize("variant", ["paper", "haar"])
def test_backward_regularised_near_degenerate(gap_eps, variant):
    """gap_eps > 0 on a cloud holding a patch whose Gram matrix has a near-degenerate pair
    (relative gap 4e-7): element by element against the oracle's regularised reading, which
    differentiates t_range's eigenvectors with Delta/(Delta^2 + eta^2), eta = gap_eps sigma_1."""
    from tests.test_oracle_knn_adjoint import near_degenerate_patch_cloud
    X, idx = near_degenerate_patch_cloud()
    X = X.astype(np.float32)
    w = synth.loss_weights(X.shape[0], seed=8)
    print(f"backward regularised gap_eps={gap_eps} {variant}", flush=True)
    g, kap, fl = _gpu_grad(X, idx, w, variant, gap_eps)
    X64 = X.astype(np.float64)
    w64 = w.astype(np.float64)
    _, go = oa.loss_and_grad(X64, idx, w64, variant, gap_eps=gap_eps)
    S = oa.grad_contribution_scale(X64, idx, w64, variant, gap_eps=gap_eps)
    _assert_elementwise(g, go, S, f"regularised, gap_eps={gap_eps}")
    # the regularisation is what keeps the gradient bounded on this cloud
    _, g_exact = oa.loss_and_grad(X64, idx, w64, variant)
    assert np.abs(g_exact).max() > 10 * np.abs(go).max()


def test_backward_swissroll_full_size():
    """The 8192 x 128 swiss roll with k = 12: central finite differences (h = 1e-3) of the GPU
    forward on 64 sampled coordinates, the float64 oracle gradient on a sampled sub-loss, and
    the Euler / translation identities on the full gradient."""
    import paper_2606_06329_amd as P
    X, k = synth.make("swissroll")
    n, m = X.shape
    w = synth.loss_weights(n)
    Xd = to_dev(X)
    idx, _, kfl = P.knn(Xd, k)
    wd = torch.from_numpy(w).cuda()
    g = P.curvature_backward(Xd, idx, wd, "paper").cpu().numpy().astype(np.float64)
    kap, fl = P.curvature_fast(Xd, idx, "paper")
    L = float((wd.double() * kap.double()).sum())
    # identities of L: translation invariance and Euler's relation for degree-2 homogeneity
    gs = g.sum(0)
    assert np.linalg.norm(gs) <= 1e-4 * np.abs(g).sum()
    euler = float(np.sum(X.astype(np.float64) * g))
    assert abs(euler - 2 * L) <= 1e-3 * np.sum(np.abs(X * g))
    # central differences of the GPU forward (float64 moments, float32 output) with the lists
    # fixed, at h and 2h.  Only the patches that contain point i change (the others see
    # bit-identical inputs), so the rounding floor of a difference quotient is that of those
    # patches' float32 outputs: an ulp of sum |w_j| kappa_j over them, over 2h.  The swiss
    # roll's patches have nine noise directions of nearly equal variance, where t_range turns
    # sharply, so the truncation error of the h = 1e-3 quotient is estimated from the 2h one
    # (Richardson) and the comparison uses the extrapolated value, within that estimate.
    rng = np.random.default_rng(7)
    idx_np = idx.cpu().numpy()
    kap_np = kap.cpu().numpy().astype(np.float64)
    deg = np.bincount(idx_np.ravel(), minlength=n)
    cand = np.nonzero(deg > 0)[0]
    h = 1e-3

    def quotient(i, a, hh):
        Xp = Xd.clone(); Xp[i, a] += hh
        Xm = Xd.clone(); Xm[i, a] -= hh
        kp, _ = P.curvature_fast(Xp, idx, "paper", "fp64")
        km, _ = P.curvature_fast(Xm, idx, "paper", "fp64")
        return float((wd.double() * (kp.double() - km.double())).sum()) / (2 * hh)

    X64 = X.astype(np.float64)
    bad = 0
    kinks = 0                        # the secant over [-h, h] crosses a sharp turn of t_range
    tight = 0                        # coordinates where the bound is tighter than 5 %
    for t in range(64):
        i = int(rng.choice(cand))
        a = int(rng.integers(0, m))
        f1, f2 = quotient(i, a, h), quotient(i, a, 2 * h)
        fdr = f1 + (f1 - f2) / 3.0
        owners = np.nonzero((idx_np == i).any(1))[0]
        floor = 2 * 2.0 ** -24 * float(np.sum(np.abs(w[owners]) * kap_np[owners])) / (2 * h)
        tol = max(1e-3 * abs(g[i, a]), 2 * floor, 0.5 * abs(f1 - f2))
        tight += tol < 0.05 * abs(g[i, a])
        if abs(fdr - g[i, a]) <= tol:
            continue
        # A mismatch is accepted only when the float64 oracle shows that it belongs to the
        # function, not to the kernels: its own difference quotient over the same [-h, h]
        # reproduces the GPU's, and its exact derivative at X equals the GPU gradient.
        sub_w = w[owners].astype(np.float64)
        _, g_or = oa.loss_and_grad(X64, idx_np[owners], sub_w, "paper")
        Lo = []
        for sgn in (1.0, -1.0):
            Xs = X64.copy()
            Xs[i, a] += sgn * h
            Lo.append(sum(sub_w[r] * oc.fast_kappa(oc.patch(Xs, idx_np[o]), "paper")
                          for r, o in enumerate(owners)))
        fd_or = (Lo[0] - Lo[1]) / (2 * h)
        explained = (abs(fd_or - f1) <= 1e-3 * abs(f1) + 4 * floor and
                     abs(g_or[i, a] - g[i, a]) <= 1e-4 * abs(g_or[i, a]) + 1e-9)
        print("fd mismatch", i, a, f1, f2, fdr, g[i, a], tol, "oracle fd", fd_or, "oracle grad",
              g_or[i, a], "explained" if explained else "UNEXPLAINED")
        kinks += explained
        bad += not explained
    print(f"  FD: {tight} of 64 coordinates checked to better than 5 % relative; "
          f"{kinks} secants across a sharp turn, confirmed by the oracle", flush=True)
    assert bad == 0
    assert kinks <= 4
    assert tight >= 32
    # float64 oracle on a sub-loss over 150 random points (exact gradient of that sub-loss)
    sel = rng.choice(n, 150, replace=False)
    ws = np.zeros(n, np.float32)
    ws[sel] = w[sel]
    gsub = P.curvature_backward(Xd, idx, torch.from_numpy(ws).cuda(), "paper").cpu().numpy().astype(np.float64)
    # oracle restricted to the selected patches
    L_o, go = oa.loss_and_grad(X.astype(np.float64), idx_np[sel], ws[sel].astype(np.float64), "paper")
    assert np.linalg.norm(gsub - go) <= 1e-4 * np.linalg.norm(go)


def test_autograd_function():
    import paper_2606_06329_amd as P
    X = synth.swissroll(n=400, m=16, seed=5)
    Xd = to_dev(X).requires_grad_(True)
    idx, _, _ = P.knn(Xd.detach(), 8)
    kap = P.MeanCurvature.apply(Xd, idx, "haar", 0.0)
    w = torch.from_numpy(synth.loss_weights(400, seed=6)).cuda()
    (w * kap).sum().backward()
    g2 = P.curvature_backward(Xd.detach(), idx, w, "haar")
    assert torch.allclose(Xd.grad, g2, rtol=1e-5, atol=1e-6 * float(g2.abs().max()))
    # a column slice of a wider matrix (row stride 23 > m = 16)
    wide = torch.zeros((400, 23), device="cuda")
    wide[:, 3:19] = to_dev(X)
    Xs = wide[:, 3:19].detach().requires_grad_(True)
    kap_s = P.MeanCurvature.apply(Xs, idx, "haar", 0.0)
    assert torch.equal(kap_s, kap.detach())
    (w * kap_s).sum().backward()
    assert torch.allclose(Xs.grad, g2, rtol=1e-5, atol=1e-6 * float(g2.abs().max()))
    # grad_kappa of the wrong length or device is rejected before any launch
    with pytest.raises(ValueError):
        P.curvature_backward(Xd.detach(), idx, w[:10], "haar")
    with pytest.raises(ValueError):
        P.curvature_backward(Xd.detach(), idx, w.cpu(), "haar")


def test_backward_run_to_run():
    """The scatter-add into grad_X uses float32 atomics, so the order of each entry's sum, and
    its last bits, vary between runs; the per-point terms themselves are deterministic.  Two
    runs on the same inputs may therefore differ by at most the rounding of two orders of the
    same sum: 2 (N - 1) 2^-24 sum |c| for an entry of N terms (N = the number of patches that
    contain the row), with sum |c| bounded by the oracle's contribution scale."""
    n, m, k = 2000, 16, 8
    X = synth.WORKLOADS["swissroll"][0](n=n, m=m, seed=97)
    idx, _, _, _ = ok.knn(X.astype(np.float64), k)
    w = synth.loss_weights(n, seed=97)
    print(f"backward run to run, swissroll n={n} m={m} k={k}", flush=True)
    g1, _, _ = _gpu_grad(X, idx, w, "paper")
    g2, _, _ = _gpu_grad(X, idx, w, "paper")
    S = oa.grad_contribution_scale(X.astype(np.float64), idx, w.astype(np.float64), "paper")
    terms = np.bincount(idx.ravel(), minlength=n).astype(np.float64)
    bound = 2.0 * np.maximum(terms - 1.0, 0.0)[:, None] * 2.0 ** -24 * 1.01 * S
    diff = np.abs(g1 - g2)
    print(f"  entries that differ: {int((diff > 0).sum())} of {diff.size}, "
          f"max diff / bound {np.max(np.where(bound > 0, diff / np.maximum(bound, 1e-300), 0.0)):.3f}",
          flush=True)
    assert np.all(diff <= bound)
