"""GPU parity of mc_curvature_exact (Theorem 1 with the canonical Householder null basis)
against the float64 oracle's canonical exact value."""
import numpy as np
import pytest

from oracle import curvature as oc
from oracle import knn as ok
from paper_2606_06329_amd import synth
from tests.gpu_common import TOL_FP32, rel_err, to_dev

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = [("sphere", 500, 20, 10, 1001), ("swissroll", 600, 128, 12, 4041),
         ("clusters", 300, 784, 11, 2041), ("torus", 400, 96, 16, 3041), ("swissroll", 300, 9, 5, 4042)]


def _separated(Xc, rel=1e-8):
    """Range eigenvalues pairwise separated, so the canonical basis is well determined.

    The kernel centres, accumulates and eigen-solves in float64; an eigenvector's error is
    about (float64 rounding of the Gram matrix) / (relative gap), so a 1e-8 gap keeps the
    basis, and hence kappa, within the float32 bar."""
    _, s, _ = np.linalg.svd(Xc, full_matrices=False)
    s = s[: Xc.shape[0] - 1]
    return np.all(np.diff(s[::-1] ** 2) > rel * s[0] ** 2)


@pytest.mark.parametrize("name,n,m,k,seed", CASES, ids=[f"{c[0]}-{c[1]}x{c[2]}-k{c[3]}" for c in CASES])
def test_exact_parity(name, n, m, k, seed):
    import paper_2606_06329_amd as P
    X = synth.WORKLOADS[name][0](n=n, m=m, seed=seed)
    idx, _, _, _ = ok.knn(X.astype(np.float64), k)
    print(f"exact {name} n={n} m={m} k={k}", flush=True)
    kap, fl = P.curvature_exact(to_dev(X), torch.from_numpy(idx.astype(np.int32)).cuda())
    kap, fl = kap.cpu().numpy(), fl.cpu().numpy()
    X64 = X.astype(np.float64)
    rows = np.arange(0, n, max(1, n // 120))
    errs, checked, skipped = [], 0, {"flag": 0, "rank": 0, "gap": 0}
    for i in rows:
        Xc = oc.patch(X64, idx[i])
        t = oc.fast_terms(Xc)
        tau = t["tau"]
        assert 0.5 * tau * (1 - 1e-5) <= kap[i] <= tau * (1 + 1e-5)      # bracket, every point
        if fl[i] & 4:
            skipped["flag"] += 1
            continue
        if t["p_eff"] != min(k - 1, m):
            skipped["rank"] += 1
            continue
        if not _separated(Xc):
            skipped["gap"] += 1
            continue
        want = oc.canonical_exact_kappa(Xc)
        errs.append(rel_err(kap[i], want))
        checked += 1
    print(f"  checked {checked} of {len(rows)}, skipped {skipped}, "
          f"max rel err {max(errs) if errs else float('nan'):.2e}", flush=True)
    assert checked >= len(rows) // 2
    assert max(errs) <= TOL_FP32


def test_exact_equals_fast_haar_when_q_is_one():
    """m = k: one null direction, so the Haar reading is the exact value."""
    import paper_2606_06329_amd as P
    X = synth.torus(n=400, m=12, seed=3051, d=3)
    idx, _, _, _ = ok.knn(X.astype(np.float64), 12)
    idd = torch.from_numpy(idx.astype(np.int32)).cuda()
    ke, _ = P.curvature_exact(to_dev(X), idd)
    kh, _ = P.curvature_fast(to_dev(X), idd, "haar")
    ke, kh = ke.cpu().numpy(), kh.cpu().numpy()
    X64 = X.astype(np.float64)
    want = np.array([oc.fast_kappa(oc.patch(X64, idx[i]), "haar") for i in range(0, 400, 7)])
    # exact path (float64 moments) against the oracle's Haar reading
    assert rel_err(ke[::7], want).max() <= TOL_FP32
    # float64-moment Fast HAAR against the exact path, both on the GPU
    kh64, _ = P.curvature_fast(to_dev(X), idd, "haar", "fp64")
    assert rel_err(ke, kh64.cpu().numpy()).max() <= TOL_FP32
    # the float32-moment Fast path on these thin (m = k, q = 1), noisy patches: the Gram matrix
    # has condition up to ~1e4, which float32 moments and the 1/q null term amplify past the
    # 1e-4 bar, so those points carry MC_PF_PRECISION_LIMIT; every unflagged point holds 1e-4
    from paper_2606_06329_amd._lib import MC_PF_PRECISION_LIMIT
    _, fl32 = P.curvature_fast(to_dev(X), idd, "haar")
    fl32 = fl32.cpu().numpy()[::7]
    flagged = (fl32 & MC_PF_PRECISION_LIMIT) != 0
    err = rel_err(kh[::7], want)
    print(f"  float32 thin patches (Gram condition 8.6e3 .. 1.2e6): {flagged.sum()} of {len(err)} flagged, "
          f"max error {err.max():.2e}, unflagged max {err[~flagged].max() if (~flagged).any() else 0:.2e}",
          flush=True)
    # no silent miss: every point beyond the float32 bar carries the flag
    assert np.all(flagged | (err <= TOL_FP32))
    assert np.any(err > TOL_FP32)      # the case does exceed the bar where it is flagged


def test_exact_shape_limit():
    import paper_2606_06329_amd as P
    from paper_2606_06329_amd._lib import MecucoError
    X = torch.zeros((100, 4096), device="cuda")
    idx = torch.zeros((100, 32), dtype=torch.int32, device="cuda")
    with pytest.raises(MecucoError):
        P.curvature_exact(X, idx)
