"""GPU parity of mc_knn against the oracle's brute-force kNN.

Sets must agree exactly wherever the oracle's gap between the k-th and (k+1)-th
distance exceeds the float32 rounding bound; other rows are counted and
reported.  Distances are compared with the float64 values.
"""
import numpy as np
import pytest

from oracle import knn as ok
from paper_2606_06329_amd import synth
from tests.gpu_common import knn_set_report, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [
    # name, n, m, k, precision, rerank
    ("sphere", 500, 20, 10, "fp32", 2),
    ("swissroll", 1300, 128, 12, "fp32", 2),
    ("clusters", 1000, 784, 11, "fp32", 2),
    ("torus", 2100, 256, 16, "fp32", 2),
    ("swissroll", 777, 61, 7, "fp32", 1),    # ragged n and m, no re-rank
    ("blobs", 900, 300, 32, "fp32", 2),      # K' = 64
    ("torus", 2100, 256, 16, "bf16", 2),
    ("clusters", 1000, 784, 11, "bf16", 2),
    ("swissroll", 1300, 128, 12, "bf16", 3),
]


@pytest.mark.parametrize("name,n,m,k,prec,rr", CASES,
                         ids=[f"{c[0]}-{c[1]}x{c[2]}-k{c[3]}-{c[4]}-r{c[5]}" for c in CASES])
def test_knn_sets(name, n, m, k, prec, rr):
    import paper_2606_06329_amd as P
    gen = synth.WORKLOADS[name][0]
    X = gen(n=n, m=m, seed=77)
    print(f"knn {name} n={n} m={m} k={k} {prec} rerank={rr}", flush=True)
    idx, d2, fl = P.knn(to_dev(X), k, precision=prec, rerank=rr)
    idx = idx.cpu().numpy()
    d2 = d2.cpu().numpy()
    fl = fl.cpu().numpy()
    rows = np.arange(n)
    bad_big, bad_small, nbig, oidx = knn_set_report(idx, X, rows, k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below); "
          f"uncertified {(fl & 32).astype(bool).sum()}, ambiguous {(fl & 16).astype(bool).sum()}")
    assert bad_big == 0
    # the ordered lists agree where the whole list is well separated, distances are float32-accurate
    X64 = X.astype(np.float64)
    for i in range(0, n, 13):
        dd = ((X64[idx[i]] - X64[i]) ** 2).sum(1)
        assert np.allclose(d2[i], dd, rtol=1e-5, atol=1e-6 * dd.max())
        assert np.all(np.diff(d2[i]) >= 0)
        assert i not in idx[i]


def test_knn_include_self():
    import paper_2606_06329_amd as P
    X = synth.swissroll(n=600, m=24, seed=5)
    X[10] = X[3]                                     # a duplicate with a smaller index
    idx, d2, _ = P.knn(to_dev(X), 8, include_self=True)
    idx = idx.cpu().numpy()
    assert np.all(idx[:, 0] == np.arange(600))
    assert idx[10, 1] == 3 and idx[3, 1] == 10


def test_knn_duplicates_tie_order():
    """Exact duplicates (distance 0) are valid neighbours, ordered by index."""
    import paper_2606_06329_amd as P
    rng = np.random.default_rng(3)
    X = rng.standard_normal((300, 16)).astype(np.float32)
    X[[50, 20, 200]] = X[100]
    idx, d2, _ = P.knn(to_dev(X), 5)
    idx, d2 = idx.cpu().numpy(), d2.cpu().numpy()
    assert list(idx[100][:3]) == [20, 50, 200]
    assert np.all(d2[100][:3] == 0.0)


def test_knn_translation_invariant_sets():
    import paper_2606_06329_amd as P
    X = synth.torus(n=1500, m=64, seed=9)
    a, _, fa = P.knn(to_dev(X), 10)
    b, _, fb = P.knn(to_dev(X + np.float32(3.0)), 10)
    a, b = a.cpu().numpy(), b.cpu().numpy()
    amb = ((fa | fb).cpu().numpy() & 16) != 0
    same = np.array([set(a[i]) == set(b[i]) for i in range(1500)])
    assert np.all(same | amb)


@pytest.mark.parametrize("name,n,m,k", [("blobs", 1500, 1024, 32), ("torus", 2100, 256, 16),
                                        ("clusters", 1000, 784, 11)])
def test_knn_fp8_sets(name, n, m, k):
    """fp8 e4m3 distance GEMM with per-row scales, then the float32 re-rank of 2k candidates."""
    import paper_2606_06329_amd as P
    X = synth.WORKLOADS[name][0](n=n, m=m, seed=78)
    print(f"knn fp8 {name} n={n} m={m} k={k}", flush=True)
    idx, d2, fl = P.knn(to_dev(X), k, precision="fp8", rerank=2)
    idx = idx.cpu().numpy()
    fl = fl.cpu().numpy()
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, np.arange(0, n, 3), k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below); "
          f"uncertified {(fl & 32).astype(bool).sum()}")
    assert bad_big == 0


@pytest.mark.parametrize("name,precision", [("clusters", "bf16"), ("blobs", "fp8")])
def test_knn_low_precision_full_size(name, precision):
    """Each low-precision GEMM at the full size of the workload it is meant for (bf16: the
    20000 x 784 clusters; fp8 with per-row scales: the 50000 x 4096 blobs, k = 32, 64
    candidates): sets exact on sampled rows wherever the k-th / (k+1)-th gap exceeds the
    float32 bound."""
    import paper_2606_06329_amd as P
    X, k = synth.make(name)
    n = X.shape[0]
    print(f"knn {precision} {name} full size, rerank {P.default_rerank(k, n, precision)}", flush=True)
    idx, _, fl = P.knn(to_dev(X), k, precision=precision)
    idx = idx.cpu().numpy()
    rows = np.random.default_rng(5).choice(n, 100 if X.shape[1] < 1000 else 30, replace=False)
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, rows, k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below)", flush=True)
    assert bad_big == 0


@pytest.mark.parametrize("n", [1, 2, 100, 128, 129, 200, 256, 300, 385, 512, 650])
def test_knn_tile_counts(n):
    """One to six 128-point tiles with ragged tails: the symmetric tile-pair schedule's
    small cases (one tile; two tiles, whose second gets only the transposed pair; an even
    tile count, where half the row tiles own the pair at distance T/2)."""
    import paper_2606_06329_amd as P
    from paper_2606_06329_amd._lib import MecucoError
    X = np.ascontiguousarray(synth.swissroll(n=max(n, 3), m=19, seed=1000 + n)[:n])
    if n <= 2:                       # k >= 2 neighbours need n >= 3 points
        with pytest.raises(MecucoError):
            P.knn(to_dev(X), 2)
        return
    k = min(6, n - 1)
    print(f"knn tiles n={n} k={k}", flush=True)
    idx, d2, fl = P.knn(to_dev(X), k)
    idx = idx.cpu().numpy()
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, np.arange(n), k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below)", flush=True)
    assert bad_big == 0
    assert np.all((idx >= 0) & (idx < n))
    assert not np.any(idx == np.arange(n)[:, None])


def test_knn_symmetric_schedule_max_n():
    """n = 131072 (1024 tiles): the largest cloud the symmetric schedule takes, whose 523776
    transposed tiles fill the 32 GiB limit (tile offsets past 2^32 floats); sets exact on
    sampled rows, including both ends and tiles far apart in the schedule."""
    import paper_2606_06329_amd as P
    n = 131072
    assert P.knn_symmetric(n) and not P.knn_symmetric(n + 1)
    X = synth.swissroll(n=n, m=8, seed=4078)
    k = 8
    print(f"knn symmetric schedule n={n} m=8 k=8", flush=True)
    idx, _, fl = P.knn(to_dev(X), k)
    idx = idx.cpu().numpy()
    rows = np.random.default_rng(7).choice(n, 200, replace=False)
    rows = np.concatenate([rows, [0, 1, 127, 128, n // 2, n - 129, n - 128, n - 1]])
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, rows, k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below)", flush=True)
    assert bad_big == 0


def test_knn_full_schedule_large_n():
    """n = 140000 (1094 tiles): past the symmetric schedule's workspace limit, so every tile
    pair is scored in both orders; sets exact on sampled rows."""
    import paper_2606_06329_amd as P
    n = 140000
    assert not P.knn_symmetric(n)
    X = synth.swissroll(n=n, m=12, seed=4077)
    k = 10
    print(f"knn full schedule n={n} m=12 k=10", flush=True)
    idx, _, fl = P.knn(to_dev(X), k)
    idx = idx.cpu().numpy()
    rows = np.random.default_rng(6).choice(n, 200, replace=False)
    rows = np.concatenate([rows, [0, n - 1, n - 100]])   # first and last tiles
    bad_big, bad_small, nbig, _ = knn_set_report(idx, X, rows, k)
    print(f"  mismatches: {bad_big} (gap above bound, of {nbig}), {bad_small} (below)", flush=True)
    assert bad_big == 0


def test_knn_uncertified_flag_on_equidistant_points():
    """Points at the unit vectors of R^500 are all at distance sqrt(2) from each other: no
    candidate list can be certified, the fp8 rescan collects every point and overflows its
    buffer, so every query keeps MC_PF_KNN_UNCERTIFIED (and MC_PF_KNN_AMBIGUOUS); the sets
    still hold k distinct other points; MC_STRICT rejects the call."""
    import paper_2606_06329_amd as P
    from paper_2606_06329_amd._lib import MC_PF_KNN_AMBIGUOUS, MC_PF_KNN_UNCERTIFIED, MecucoError
    n = 500
    X = np.eye(n, dtype=np.float32)
    idx, d2, fl = P.knn(to_dev(X), 8, precision="fp8")
    idx, fl = idx.cpu().numpy(), fl.cpu().numpy()
    assert np.all(fl & MC_PF_KNN_UNCERTIFIED) and np.all(fl & MC_PF_KNN_AMBIGUOUS)
    assert all(len(set(r)) == 8 and i not in r for i, r in enumerate(idx.tolist()))
    assert np.allclose(d2.cpu().numpy(), 2.0)
    with pytest.raises(MecucoError):
        P.knn(to_dev(X), 8, precision="fp8", strict=True)
