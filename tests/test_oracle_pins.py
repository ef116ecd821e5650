"""Pins of the float64 oracle against facts fixed by the paper and by mathematics.

Each test names the passage it follows.  None of them retypes the formula it
checks: they compare two routes to the same quantity (explicit H vs the
closed form of Theorem 1), closed forms derived by hand for special patches,
invariants, and Monte-Carlo averages.
"""
import math

import numpy as np
import pytest

from oracle import curvature as oc
from oracle import knn as ok
from paper_2606_06329_amd import synth


@pytest.fixture(scope="module")
def sphere_data():
    X = synth.sphere().astype(np.float64)
    idx, d2, gap, d2n = ok.knn(X, 10)
    return X, idx


def _patches(X, idx, step=37):
    return [oc.patch(X, idx[i]) for i in range(0, X.shape[0], step)]


def test_naive_equals_identity(sphere_data):
    """Theorem 1 / Remark on numerical equivalence: explicit H vs closed form, same W."""
    X, idx = sphere_data
    for Xc in _patches(X, idx):
        S = oc.covariance(Xc)
        v, W = oc.eig_desc(S)
        kn = oc.naive_kappa(S, W)
        ki = oc.identity_kappa(W, v)
        assert abs(kn - ki) <= 1e-10 * ki


def test_naive_equals_identity_random_tiny():
    """Same identity on random tiny patches with any orthogonal W (the proof needs only W W^T = I)."""
    rng = np.random.default_rng(7)
    for _ in range(20):
        k, m = rng.integers(3, 8), rng.integers(3, 10)
        Xc = rng.standard_normal((k, m))
        Xc -= Xc.mean(0)
        S = oc.covariance(Xc)
        v, W = oc.eig_desc(S)
        assert abs(oc.naive_kappa(S, W) - oc.identity_kappa(W, v)) <= 1e-10 * oc.identity_kappa(W, v)


def test_HHt_collapse():
    """Boxed identity HH^T = 1/2 W2 W2^T + 1/2 I for an orthogonal W (eq. HHt_final)."""
    rng = np.random.default_rng(3)
    W = synth.haar_rotation(rng, 9)
    H = oc.build_H(W)
    assert H.shape == (9, 9 + 36)
    W2 = W * W
    assert np.linalg.norm(H @ H.T - 0.5 * W2 @ W2.T - 0.5 * np.eye(9)) <= 1e-12


def test_bracket(sphere_data):
    """1/2 tau <= kappa_exact <= tau: W o W is doubly stochastic, so its spectral norm is 1."""
    X, idx = sphere_data
    for Xc in _patches(X, idx, 11):
        t = oc.fast_terms(Xc)
        tau = t["tau"]
        for kap in (oc.canonical_exact_kappa(Xc), oc.lapack_exact_kappa(Xc), t["kappa_haar"]):
            assert 0.5 * tau - 1e-12 * tau <= kap <= tau + 1e-12 * tau


def _planar_patch(theta, v1, v2, m, offset):
    """k=3 points whose covariance has eigenvalues v1 > v2 along axes at angle theta in (e1, e2)."""
    a, b = math.sqrt(v1), math.sqrt(v2 / 3.0)
    Y = np.array([[a, b], [-a, b], [0.0, -2.0 * b]])
    c, s = math.cos(theta), math.sin(theta)
    X = np.zeros((3, m))
    X[:, 0] = c * Y[:, 0] - s * Y[:, 1]
    X[:, 1] = s * Y[:, 0] + c * Y[:, 1]
    return X + offset[None, :]


@pytest.mark.parametrize("theta_deg", [0.0, 17.0, 30.0, 45.0, 71.0])
def test_planar_closed_form(theta_deg):
    """Hand-derived closed form for a 3-point planar patch (derivation in the design doc):
    kappa = (v1+v2)(1-u^2) + 2u^3(v1-v2), u = sin(2 theta)/2, for the naive, identity,
    and both fast readings (their null term vanishes for this patch)."""
    theta = math.radians(theta_deg)
    v1, v2, m = 3.0, 1.0, 6
    off = np.linspace(-1.0, 2.0, m)
    Xp = _planar_patch(theta, v1, v2, m, off)
    Xc = Xp - Xp.mean(0)
    u = 0.5 * math.sin(2 * theta)
    want = (v1 + v2) * (1 - u * u) + 2 * u ** 3 * (v1 - v2)
    S = oc.covariance(Xc)
    v, W = oc.eig_desc(S)
    t = oc.fast_terms(Xc)
    got = [oc.naive_kappa(S, W), oc.identity_kappa(W, v), t["kappa_paper"], t["kappa_haar"],
           oc.canonical_exact_kappa(Xc)]
    for g in got:
        assert abs(g - want) <= 1e-12 * want
    # the printed check values at 45 degrees: v1 + v2/2
    if theta_deg == 45.0:
        assert abs(want - (v1 + 0.5 * v2)) < 1e-14


def test_axis_aligned_patch_gives_tau():
    """A patch supported on p coordinate axes with diagonal covariance: W is a signed
    permutation, C = I up to signs, so every estimator returns tau."""
    h = np.array([[1, 1, 1], [-1, 1, -1], [1, -1, -1], [-1, -1, 1]], dtype=float)
    Xc = np.zeros((4, 7))
    Xc[:, 1] = 2.0 * h[:, 0]
    Xc[:, 3] = 0.7 * h[:, 1]
    Xc[:, 6] = 1.3 * h[:, 2]
    tau = np.sum(Xc * Xc) / 3
    S = oc.covariance(Xc)
    v, W = oc.eig_desc(S)
    t = oc.fast_terms(Xc)
    for g in (oc.naive_kappa(S, W), oc.identity_kappa(W, v), t["kappa_paper"], t["kappa_haar"],
              oc.canonical_exact_kappa(Xc)):
        assert abs(g - tau) <= 1e-13 * tau


def test_haar_exact_when_null_space_is_one_dimensional():
    """q = m - p = 1: the null vector is unique up to sign, so the Haar expectation is
    the exact value (canonical and LAPACK bases agree); the printed reading differs."""
    rng = np.random.default_rng(11)
    for _ in range(10):
        k = 6
        Xc = rng.standard_normal((k, k))
        Xc -= Xc.mean(0)
        t = oc.fast_terms(Xc)
        assert t["q"] == 1
        ex = oc.canonical_exact_kappa(Xc)
        assert abs(oc.lapack_exact_kappa(Xc) - ex) <= 1e-12 * ex
        assert abs(t["kappa_haar"] - ex) <= 1e-12 * ex
        assert abs(t["kappa_paper"] - ex) > 1e-6 * ex


def test_factored_vs_dense_haar(sphere_data):
    """eq. gnull_exp summed densely against Sigma equals the factored O(km p^2) form."""
    X, idx = sphere_data
    for Xc in _patches(X, idx, 29):
        t = oc.fast_terms(Xc)
        d = oc.dense_haar_tnull(Xc)
        assert abs(d - t["t_null_haar"]) <= 1e-12 * abs(d)


def test_monte_carlo_haar(sphere_data):
    """The Haar reading is the mean of the exact null term over uniformly random
    orthonormal null bases (eq. gnull_exp): Monte-Carlo within 4 standard errors."""
    X, idx = sphere_data
    rng = np.random.default_rng(12345)
    for i in (7, 123):
        Xc = oc.patch(X, idx[i])
        t = oc.fast_terms(Xc)
        vals = oc.monte_carlo_tnull(Xc, 10000, rng)
        se = vals.std() / math.sqrt(len(vals))
        assert abs(vals.mean() - t["t_null_haar"]) <= 4 * se
        # the printed reading is far outside that band
        assert abs(vals.mean() - t["t_null_paper"]) > 20 * se


def test_split_range_null(sphere_data):
    """eq. split: for W = [V_r | N], Theorem 1 equals 1/2 (t_range + t_null^W) + 1/2 tau with
    t_null^W = sum_{l>p} ||X_c (w_l o w_l)||^2/(k-1)."""
    X, idx = sphere_data
    rng = np.random.default_rng(5)
    for Xc in _patches(X, idx, 53):
        k, m = Xc.shape
        Vr, s, pe = oc.range_basis(Xc)
        N0 = oc.householder_null_basis(Vr)
        R = synth.haar_rotation(rng, m - pe)
        N = N0 @ R
        t = oc.fast_terms(Xc)
        tnull = np.sum((Xc @ (N * N)) ** 2) / (k - 1)
        want = 0.5 * (t["t_range"] + tnull) + 0.5 * t["tau"]
        assert abs(oc.kappa_with_null_basis(Xc, N) - want) <= 1e-12 * want


def test_printed_tB_middle_term_equals_tau(sphere_data):
    """||X_c V_r||_F^2/(k-1) equals tau because every row of X_c lies in range(V_r)."""
    X, idx = sphere_data
    for Xc in _patches(X, idx, 19):
        t = oc.fast_terms(Xc)
        assert abs(t["t_S"] - t["tau"]) <= 1e-12 * t["tau"]
        assert abs(t["tau"] - np.sum(Xc * Xc) / (Xc.shape[0] - 1)) <= 1e-12 * t["tau"]


def test_householder_basis(sphere_data):
    """Canonical null basis: orthonormal, orthogonal to V_r, unchanged by column sign flips of V_r."""
    X, idx = sphere_data
    Xc = oc.patch(X, idx[3])
    Vr, _, pe = oc.range_basis(Xc)
    N = oc.householder_null_basis(Vr)
    m = Xc.shape[1]
    assert N.shape == (m, m - pe)
    assert np.linalg.norm(N.T @ N - np.eye(m - pe)) < 1e-13
    assert np.linalg.norm(Vr.T @ N) < 1e-13
    signs = np.where(np.arange(pe) % 2 == 0, 1.0, -1.0)
    N2 = oc.householder_null_basis(Vr * signs[None, :])
    assert np.linalg.norm(N2 - N) < 1e-13


def test_invariances(sphere_data):
    """Homogeneity of degree 2, translation, point permutation, coordinate permutation and
    global negation.  (A sign flip of a single coordinate is NOT a symmetry: it flips
    W_as but not W_al^2 in C = W^T (W o W); see test_single_sign_flip_changes_kappa.)"""
    X, idx = sphere_data
    rng = np.random.default_rng(9)
    m = X.shape[1]
    perm = rng.permutation(m)
    sg = rng.choice([-1.0, 1.0], size=m)
    for i in (0, 50, 99, 321):
        P = X[idx[i]]
        base = {v: oc.fast_kappa(P - P.mean(0), v) for v in ("paper", "haar")}
        base["canon"] = oc.canonical_exact_kappa(P - P.mean(0))
        variants = {
            "scale2": (2.0 * P, 4.0),
            "translate": (P + rng.standard_normal(m)[None, :] * 10, 1.0),
            "rowperm": (P[rng.permutation(P.shape[0])], 1.0),
            "coord_perm": (P[:, perm], 1.0),
            "negation": (-P, 1.0),
        }
        for name, (Q, fac) in variants.items():
            Qc = Q - Q.mean(0)
            for v in ("paper", "haar"):
                assert abs(oc.fast_kappa(Qc, v) - fac * base[v]) <= 1e-11 * fac * base[v], (name, v)
            if name != "coord_perm":
                # the Householder completion pivots on the coordinate order, so the
                # canonical exact value is basis (and hence order) dependent
                assert abs(oc.canonical_exact_kappa(Qc) - fac * base["canon"]) <= 1e-10 * fac * base["canon"], name


def test_rotation_invariant_parts(sphere_data):
    """Under a general rotation of ambient space the kNN sets, tau and the eigenvalues are
    invariant; kappa itself is not (the Hadamard square is coordinate dependent), so its
    drift is only bounded by the bracket."""
    X, idx = sphere_data
    rng = np.random.default_rng(21)
    Q = synth.haar_rotation(rng, X.shape[1])
    XR = X @ Q.T
    idxR, _, gapR, _ = ok.knn(XR, 10)
    assert np.array_equal(idx, idxR)
    for i in (1, 77, 400):
        a = oc.fast_terms(oc.patch(X, idx[i]))
        b = oc.fast_terms(oc.patch(XR, idx[i]))
        assert abs(a["tau"] - b["tau"]) <= 1e-12 * a["tau"]
        assert np.allclose(a["s"], b["s"], rtol=1e-10, atol=0)
        assert 0.5 * b["tau"] * (1 - 1e-12) <= oc.canonical_exact_kappa(oc.patch(XR, idx[i])) <= b["tau"] * (1 + 1e-12)


def test_fast_equals_exact_without_null_space():
    """m <= p: V_r spans R^m, there is no null space and the fast value is Theorem 1 itself."""
    rng = np.random.default_rng(4)
    Xc = rng.standard_normal((9, 5))
    Xc -= Xc.mean(0)
    t = oc.fast_terms(Xc)
    assert t["q"] == 0
    ex = oc.lapack_exact_kappa(Xc)
    assert abs(t["kappa_paper"] - ex) <= 1e-12 * ex
    assert abs(t["kappa_haar"] - ex) <= 1e-12 * ex


def test_rank_deficient_patch():
    """Duplicate points lower the rank below k-1; p_eff follows the numerical rank."""
    rng = np.random.default_rng(8)
    P = rng.standard_normal((6, 12))
    P[4] = P[1]
    P[5] = P[2]
    t = oc.fast_terms(P - P.mean(0))
    assert t["p_eff"] == 3
    assert t["q"] == 9


def test_single_sign_flip_changes_kappa():
    """Planar closed form under y -> -y: theta -> -theta, u -> -u, so kappa moves by
    4 u^3 (v1 - v2); the estimator is not invariant under coordinate reflections."""
    theta, v1, v2, m = math.radians(30.0), 3.0, 1.0, 5
    Xp = _planar_patch(theta, v1, v2, m, np.zeros(m))
    Xf = Xp.copy()
    Xf[:, 1] *= -1.0
    a = oc.canonical_exact_kappa(Xp - Xp.mean(0))
    b = oc.canonical_exact_kappa(Xf - Xf.mean(0))
    u = 0.5 * math.sin(2 * theta)
    assert abs((a - b) - 4 * u ** 3 * (v1 - v2)) <= 1e-12 * a


def _two_point_closed_form(d):
    """Every Fast-branch term of a two-point patch, derived by hand in exact rational arithmetic.

    With k = 2 the centred rows are +d/2 and -d/2, p = 1 and V_r = d/|d|, so with
    S1 = sum d_a, S3 = sum d_a^3, S4 = sum d_a^4 and D2 = |d|^2:
      tau = t_S = D2/2,  t_range = g = (S3/D2)^2/2,  t_A = (S1 - S3/D2)^2/2,  t_D = S4/(2 D2);
    the printed reading then has t_null = (t_A + 2 (g - tau))/q and the Haar reading
    t_null = (t_A + 2 (tau - 2 t_D + g))/(q + 2), q = m - 1 (Fast branch of Algorithm 1,
    eqs. tA, tB, tnull and gnull_exp)."""
    from fractions import Fraction as F
    d = [F(int(x)) for x in d]
    m = len(d)
    D2 = sum(x * x for x in d)
    S1 = sum(d)
    S3 = sum(x ** 3 for x in d)
    S4 = sum(x ** 4 for x in d)
    tau = D2 / 2
    t_range = (S3 / D2) ** 2 / 2
    g = t_range
    t_A = (S1 - S3 / D2) ** 2 / 2
    t_D = S4 / (2 * D2)
    q = m - 1
    t_null_p = (t_A + 2 * (tau - 2 * tau + g)) / q
    t_null_h = (t_A + 2 * (tau - 2 * t_D + g)) / (q + 2)
    kp = abs((t_range + t_null_p) / 2 + tau / 2)
    kh = abs((t_range + t_null_h) / 2 + tau / 2)
    return dict(tau=tau, t_range=t_range, g=g, t_A=t_A, t_S=tau, t_D=t_D, kappa_paper=kp, kappa_haar=kh)


@pytest.mark.parametrize("d,kp,kh", [
    ((1, 2, 2, 0, 0), "497/162", "215/54"),
    ((3, -1, 2, 0, 0, 0, 0, 1, 0, 0, 0), None, None),
    ((2, 1, 0, 0, -2, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 4, 0, 0), None, None),
])
def test_two_point_closed_form(d, kp, kh):
    """The Fast branch's null-space term in both readings, pinned by exact rational values.

    Unlike the planar and axis-aligned patches, a two-point patch along a generic direction
    has a non-zero null term in both readings, so a wrong denominator (q vs q + 2), a dropped
    2 t_S or a sign slip in t_B changes kappa; the first case's values are worked out by hand
    (kappa_PAPER = 497/162, kappa_HAAR = 215/54)."""
    from fractions import Fraction as F
    want = _two_point_closed_form(d)
    if kp is not None:
        assert want["kappa_paper"] == F(kp) and want["kappa_haar"] == F(kh)
    dv = np.array(d, dtype=np.float64)
    centre = np.linspace(-3.0, 5.0, len(d))           # an arbitrary offset: centring removes it
    X = np.stack([centre + 0.5 * dv, centre - 0.5 * dv])
    t = oc.fast_terms(oc.patch(X, [0, 1]))
    assert t["p_eff"] == 1 and t["q"] == len(d) - 1
    for key in ("tau", "t_range", "g", "t_A", "t_S", "t_D", "kappa_paper", "kappa_haar"):
        w = float(want[key])
        assert abs(t[key] - w) <= 1e-13 * max(abs(w), float(want["tau"])), key
    assert abs(t["kappa_paper"] - t["kappa_haar"]) > 1e-3 * float(want["tau"])


def degenerate_integer_patch(m=12):
    """Eight points whose centred Gram matrix has the eigenvalues 8 s_j^2, s = (1, 1, 2, 3, 4,
    5, 6), plus 0: rows of an 8 x 8 Hadamard matrix without its first column, column j scaled
    by s_j, zero-padded to m and shifted by 8.  Full rank 7 with an exactly degenerate pair
    (the two smallest); every value is a small integer."""
    H = np.array([[1]], np.float64)
    for _ in range(3):
        H = np.block([[H, H], [H, -H]])
    pts = np.zeros((8, m))
    pts[:, :7] = H[:, 1:] * np.array([1, 1, 2, 3, 4, 5, 6], np.float64)
    return pts + 8.0


def test_degenerate_pair_only_moves_t_range():
    """Rotating the basis inside an exactly degenerate pair of singular values (finding F6):
    tau, t_A, t_S, g and t_D depend on the projector only and stay put; t_range reads the
    individual columns and moves, so kappa spans a range."""
    Xc = degenerate_integer_patch(12)
    Xc = Xc - Xc.mean(0)
    Vr, s, pe = oc.range_basis(Xc)
    a, b = pe - 2, pe - 1                       # the degenerate pair (smallest)
    assert pe == 7 and abs(s[a] - s[b]) <= 1e-12 * s[0]
    base = oc.fast_terms(Xc)
    tr = []
    for phi in np.linspace(0.0, np.pi, 13):
        c, sn = np.cos(phi), np.sin(phi)
        V = Vr.copy()
        V[:, a], V[:, b] = c * Vr[:, a] - sn * Vr[:, b], sn * Vr[:, a] + c * Vr[:, b]
        t = oc.fast_terms_with_basis(Xc, V, s)
        for key in ("tau", "t_A", "t_S", "g", "t_D"):
            assert abs(t[key] - base[key]) <= 1e-12 * max(abs(base[key]), base["tau"]), key
        tr.append(t["t_range"])
    assert max(tr) - min(tr) > 1e-3 * base["tau"]


def test_minmax_normalise():
    """Normalised scores (the normalised-score experiment): the ranking is kept, the extremes
    map to 0 and 1, the map is affine, NaN stays NaN and a constant vector maps to 0."""
    rng = np.random.default_rng(12)
    k = rng.gamma(2.0, 3.0, 500)
    k[[7, 99]] = np.nan
    z = oc.minmax_normalise(k)
    fin = np.isfinite(k)
    assert np.all(np.isnan(z[~fin]))
    assert z[fin].min() == 0.0 and z[fin].max() == 1.0
    assert np.array_equal(np.argsort(k[fin], kind="stable"), np.argsort(z[fin], kind="stable"))
    a, b = np.polyfit(k[fin], z[fin], 1)
    assert np.allclose(a * k[fin] + b, z[fin], atol=1e-12)
    assert np.all(oc.minmax_normalise(np.full(9, 3.5)) == 0.0)
    assert np.all(np.isnan(oc.minmax_normalise(np.array([np.nan, np.inf]))))
