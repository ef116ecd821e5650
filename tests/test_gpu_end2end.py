"""End-to-end GPU path (kNN then Fast curvature) against the oracle, small and full size."""
import numpy as np
import pytest

from oracle import knn as ok
from paper_2606_06329_amd import synth
from tests.gpu_common import TOL_FP32, TOL_LOW, knn_set_report, oracle_fast, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_sphere_all_points():
    """The 500-point sphere workload, every point, both readings."""
    import paper_2606_06329_amd as P
    X, k = synth.make("sphere")
    kap_p, idx, fl = P.curvature(to_dev(X), k, mode="fast", variant="paper")
    kap_h, _, _ = P.curvature(to_dev(X), k, mode="fast", variant="haar", idx=idx)
    idx = idx.cpu().numpy()
    bad_big, _, _, oidx = knn_set_report(idx, X, np.arange(500), k)
    assert bad_big == 0
    for kap, v in ((kap_p, "paper"), (kap_h, "haar")):
        want, pe = oracle_fast(X, idx, v)
        ok_rows = (fl.cpu().numpy() & 4) == 0
        assert rel_err(kap.cpu().numpy(), want)[ok_rows].max() <= TOL_FP32


@pytest.mark.parametrize("name", ["clusters", "swissroll", "torus"])
def test_full_size_sampled(name):
    """Full-size workload in the benchmark's launch configuration; 48 sampled points are
    checked against the oracle (kNN rows and curvature one by one)."""
    import paper_2606_06329_amd as P
    X, k = synth.make(name)
    n = X.shape[0]
    print(f"full size {name} n={n} m={X.shape[1]} k={k}", flush=True)
    Xd = to_dev(X)
    idx, d2, kfl = P.knn(Xd, k, precision="fp32", rerank=2)
    kap, fl = P.curvature_fast(Xd, idx, "paper", "fp32")
    idx = idx.cpu().numpy()
    kap = kap.cpu().numpy()
    fl = (fl | kfl).cpu().numpy()
    rows = np.random.default_rng(42).choice(n, 48, replace=False)
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, rows, k)
    assert bad_big == 0
    want, pe = oracle_fast(X, idx, "paper", rows=rows)
    okr = (fl[rows] & 4) == 0
    assert rel_err(kap[rows], want)[okr].max() <= TOL_FP32
    # property at every point: kappa finite and non-negative
    assert np.all(np.isfinite(kap)) and np.all(kap >= 0)
    print(f"  uncertified {(fl & 32).astype(bool).mean():.4f}, rank-deficient {(fl & 4).astype(bool).mean():.4f}")


@pytest.mark.parametrize("precision,tol,noise", [("fp64", None, 0.05), ("fp32", 1e-4, 0.05)])
def test_very_large_m_auto_mode(precision, tol, noise):
    """The paper's widest regime (n = 283, m = 54621, like its largest expression array):
    Auto mode picks the Fast branch (m >= 50), the kernels stream m in chunks, and every
    point matches the oracle; k is the default floor(log2 n).  float64 moments hold the
    float64 bar; float32 moments hold the float32 bar on every point that neither the rank test
    nor the precision estimate flags.  The float32 rank floor grows with m (eigenvalues above
    m 2^-24 sigma_1 = 3.3e-3 sigma_1 here), so a quarter of these noisy patches are declared
    rank deficient on that path, flagged and left out."""
    import paper_2606_06329_amd as P
    from tests.gpu_common import TOL_FP64
    tol = TOL_FP64 if tol is None else tol
    rng = np.random.default_rng(54621)
    n, m = 283, 54621
    # a curved 3-dimensional chart with noise, as float32
    z = rng.standard_normal((n, 3))
    A = rng.standard_normal((3, m)) / np.sqrt(3)
    B = rng.standard_normal((6, m)) / 6.0
    quad = np.stack([z[:, 0] ** 2, z[:, 1] ** 2, z[:, 2] ** 2, z[:, 0] * z[:, 1], z[:, 0] * z[:, 2],
                     z[:, 1] * z[:, 2]], axis=1)
    X = (z @ A + quad @ B + noise * rng.standard_normal((n, m))).astype(np.float32)
    k = P.default_k(n)
    print(f"very large m: n={n} m={m} k={k} {precision}", flush=True)
    kap, idx, fl = P.curvature(to_dev(X), mode="auto", precision=precision)
    idx = idx.cpu().numpy()
    bad_big, _, _, _ = knn_set_report(idx, X, np.arange(0, n, 7), k)
    assert bad_big == 0
    want, pe = oracle_fast(X, idx, "paper")
    fl = fl.cpu().numpy()
    ok_rows = ((fl & 4) == 0) & (pe == k - 1)
    unflagged = ok_rows & ((fl & 128) == 0)
    err = rel_err(kap.cpu().numpy(), want)
    print(f"  rank-full points {ok_rows.sum()}, unflagged {unflagged.sum()}, max rel err {err[unflagged].max():.2e}"
          f" (all rank-full: {err[ok_rows].max():.2e})", flush=True)
    assert ok_rows.mean() > (0.95 if precision == "fp64" else 0.6)
    assert unflagged.sum() >= 0.95 * ok_rows.sum()
    assert err[unflagged].max() <= tol


@pytest.mark.parametrize("name,kprec,cprec,nrows", [("torus", "bf16", "bf16", 100), ("blobs", "fp8", "bf16", 30)])
def test_full_size_low_precision_path(name, kprec, cprec, nrows):
    """The mixed-precision paths at the full size of the configurations they are meant for, in
    the benchmark's launch configuration: the 100000 x 256 torus with bf16 distance GEMM and
    range products (k = 16, 32 candidates), and the 50000 x 4096 blobs with the fp8 e4m3 GEMM
    and 64 candidates, bf16 range products (k = 32).  Sampled rows: neighbour sets exact
    wherever the gap exceeds the float32 bound (admissible elsewhere), curvature within 2e-2 of
    the oracle; every point certified; kappa finite and non-negative everywhere."""
    import paper_2606_06329_amd as P
    X, k = synth.make(name)
    n = X.shape[0]
    rr = P.default_rerank(k, n, kprec)
    print(f"full size {name} n={n} m={X.shape[1]} k={k} knn {kprec} x{rr}, curvature {cprec}", flush=True)
    Xd = to_dev(X)
    idx, d2, kfl = P.knn(Xd, k, precision=kprec, rerank=rr)
    kap, fl = P.curvature_fast(Xd, idx, "paper", cprec)
    idx = idx.cpu().numpy()
    kap = kap.cpu().numpy()
    kfl = kfl.cpu().numpy()
    fl = fl.cpu().numpy()
    assert int(((kfl & 32) != 0).sum()) == 0, "uncertified neighbour sets"
    rows = np.random.default_rng(43).choice(n, nrows, replace=False)
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, rows, k)
    print(f"  sets: {bad_big} wrong, {bad_small} admissible alternatives, {nbig} rows above the bound",
          flush=True)
    assert bad_big == 0
    want, pe = oracle_fast(X, idx, "paper", rows=rows)
    okr = ((fl[rows] & (4 | 128)) == 0) & (pe == k - 1)
    err = rel_err(kap[rows], want)[okr]
    print(f"  curvature: {okr.sum()} points, max rel err {err.max():.2e}", flush=True)
    assert okr.mean() > 0.9
    assert err.max() <= TOL_LOW
    assert np.all(np.isfinite(kap)) and np.all(kap >= 0)


def test_normalised_output():
    """mc_normalize_minmax against the oracle's normalisation (float64) and bit for bit against
    the same float32 arithmetic on the host; NaN scores, a constant vector, and the ragged
    block tail (n not a multiple of 256, more than 256 blocks' worth of points)."""
    import paper_2606_06329_amd as P
    from oracle import curvature as oc
    X, k = synth.make("swissroll")
    kap, idx, fl = P.curvature(to_dev(X), k)
    for vec in (kap, kap[:1001].clone(), torch.full((77,), 2.5, device="cuda")):
        v = vec.clone()
        if v.numel() > 50:
            v[13] = float("nan")
        z = P.normalize_minmax(v).cpu().numpy()
        h = v.cpu().numpy()
        want = oc.minmax_normalise(h)
        fin = np.isfinite(h)
        assert np.array_equal(np.isnan(z), ~fin)
        assert np.all(np.abs(z[fin] - want[fin]) <= 2.0 ** -22)
        lo, hi = h[fin].min(), h[fin].max()
        f32 = np.zeros_like(h[fin]) if hi == lo else (h[fin] - lo) / np.float32(hi - lo)
        assert np.array_equal(z[fin], f32.astype(np.float32))
    big = torch.rand(256 * 256 * 3 + 17, device="cuda")
    zb = P.normalize_minmax(big).cpu().numpy()
    assert zb.min() == 0.0 and zb.max() == 1.0
    # the end-to-end call with normalize=True equals normalising afterwards
    kn, _, _ = P.curvature(to_dev(X), k, normalize=True)
    assert torch.equal(kn, P.normalize_minmax(kap))
