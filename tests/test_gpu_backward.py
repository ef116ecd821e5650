"""GPU adjoint (mc_curvature_backward) against the float64 autograd oracle, central finite
differences of the GPU forward, and the identities of a translation-invariant, degree-2
homogeneous loss."""
import numpy as np
import pytest

from oracle import adjoint as oa
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


@pytest.mark.parametrize("variant", ["paper", "haar"])
@pytest.mark.parametrize("name,n,m,k,seed", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-k{c[3]}" for c in CASES])
def test_backward_vs_oracle(name, n, m, k, seed, variant):
    """Element-by-element against autograd through the float64 oracle (same float32 inputs)."""
    X = synth.WORKLOADS[name][0](n=n, m=m, seed=seed)
    idx, _, _, _ = ok.knn(X.astype(np.float64), k)
    w = synth.loss_weights(n, seed=seed)
    print(f"backward {name} n={n} m={m} k={k} {variant}", flush=True)
    g, kap, fl = _gpu_grad(X, idx, w, variant)
    L, go = oa.loss_and_grad(X.astype(np.float64), idx, w.astype(np.float64), variant)
    assert not np.any(fl & 4), "rank-deficient patches in a parity case"
    err = np.abs(g - go)
    scale = np.abs(go).max()
    print(f"  max |dg| / max |g| = {err.max() / scale:.2e}, rel norm {np.linalg.norm(g - go) / np.linalg.norm(go):.2e}")
    assert np.linalg.norm(g - go) <= 1e-4 * np.linalg.norm(go)
    assert err.max() <= 1e-4 * scale


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
    # central differences of the float32 GPU forward with the lists fixed
    rng = np.random.default_rng(7)
    deg = np.bincount(idx.cpu().numpy().ravel(), minlength=n)
    cand = np.nonzero(deg > 0)[0]
    h = 1e-3
    bad = 0
    for t in range(64):
        i = int(rng.choice(cand))
        a = int(rng.integers(0, m))
        Xp = Xd.clone(); Xp[i, a] += h
        Xm = Xd.clone(); Xm[i, a] -= h
        kp, _ = P.curvature_fast(Xp, idx, "paper")
        km, _ = P.curvature_fast(Xm, idx, "paper")
        fd = float((wd.double() * (kp.double() - km.double())).sum()) / (2 * h)
        tol = max(1e-3 * abs(g[i, a]), 20 * 2.0 ** -24 * abs(L) / h)
        if abs(fd - g[i, a]) > tol:
            bad += 1
            print("fd mismatch", i, a, fd, g[i, a], tol)
    assert bad == 0
    # float64 oracle on a sub-loss over 150 random points (exact gradient of that sub-loss)
    sel = rng.choice(n, 150, replace=False)
    ws = np.zeros(n, np.float32)
    ws[sel] = w[sel]
    gsub = P.curvature_backward(Xd, idx, torch.from_numpy(ws).cuda(), "paper").cpu().numpy().astype(np.float64)
    idx_np = idx.cpu().numpy()
    rows = np.unique(np.concatenate([sel, idx_np[sel].ravel()]))
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
