"""Float64 gradient of L(X) = sum_i w_i kappa_i with the neighbour lists held fixed.

Test infrastructure only.  The forward pass restates the Fast branch of
Algorithm 1 (centring, truncated SVD, t_range, t_A, t_B, t_null, eq.
fast_curv) in PyTorch float64 on the CPU so that autograd supplies the exact
derivative.  The truncated SVD is taken from the eigen-decomposition of the
k x k Gram matrix K = X_c X_c^T (its non-zero eigenpairs are s_l^2 and the left
singular vectors; V_r = X_c^T U_p diag(1/s_p)); this is the same factorisation
as SVD_p and avoids differentiating through the always-zero singular value of
a centred patch.  Pinned by central finite differences, the Euler identity of
a degree-2 homogeneous function, translation invariance and agreement of the
forward value with ``oracle.curvature.fast_kappa``.

Regularised reading (``gap_eps``).  The paper defines no derivative; the
derivative of an eigenvector of K has factors 1/(sigma_j - sigma_i) that blow up
when two eigenvalues meet.  Of the Fast terms only t_range reads individual
eigenvectors (every other term depends on the range projector alone), so the
regularised reading differentiates t_range's eigenvectors with the factor
Delta/(Delta^2 + eta^2), Delta = sigma_j - sigma_i, eta = gap_eps * sigma_1
(sigma_1 the largest eigenvalue of K, held constant), and every other term
exactly, through the projector X_c^T K^+ X_c (no eigen-gap factors at all).  gap_eps = 0 is the exact derivative.  Pinned by the exact gradient at
gap_eps = 0, by first-order perturbation theory of the regularised eigenvector
derivative, and by the Euler and translation identities, which hold for every
gap_eps because scaling and translating X never mix eigenvectors.
"""
from __future__ import annotations

import numpy as np
import torch

__all__ = ["fast_kappa_torch", "loss_and_grad", "reg_eigh", "grad_contribution_scale"]


class _RegEigh(torch.autograd.Function):
    """(sigma, U) = eigh(K), ascending; backward with regularised gap factors.

    For K = U diag(sigma) U^T the first-order change of U is dU = U (F o (U^T dK U)) with
    F_ij = 1/(sigma_j - sigma_i) off the diagonal.  The adjoint is therefore
    K_bar = U (diag(sigma_bar) + F o (U^T U_bar)) U^T (symmetrised); here F_ij is replaced by
    Delta/(Delta^2 + eta^2), Delta = sigma_j - sigma_i, and set to 0 where Delta = 0.
    """

    @staticmethod
    def forward(ctx, K, eta):
        sig, U = torch.linalg.eigh(K)
        ctx.save_for_backward(sig, U)
        ctx.eta = float(eta)
        return sig, U

    @staticmethod
    def backward(ctx, gsig, gU):
        sig, U = ctx.saved_tensors
        n = sig.shape[0]
        M = torch.zeros((n, n), dtype=sig.dtype)
        if gU is not None:
            delta = sig[None, :] - sig[:, None]               # Delta_ij = sigma_j - sigma_i
            den = delta * delta + ctx.eta * ctx.eta
            F = torch.where(den > 0, delta / torch.where(den > 0, den, torch.ones_like(den)),
                            torch.zeros_like(den))
            F.fill_diagonal_(0.0)
            M = M + F * (U.T @ gU)
        if gsig is not None:
            M = M + torch.diag(gsig)
        gK = U @ M @ U.T
        return 0.5 * (gK + gK.T), None


def reg_eigh(K: torch.Tensor, eta: float):
    """Eigenpairs of symmetric K (ascending) whose backward uses regularised gap factors."""
    return _RegEigh.apply(K, eta)


def _range_basis(Xc, sig, U, p_eff):
    """Descending eigenpairs of K truncated to p_eff; V_r = X_c^T U_p / s_p."""
    sig = sig.flip(0)[:p_eff]
    U = U.flip(1)[:, :p_eff]
    s = torch.sqrt(sig)
    return sig, (Xc.T @ U) / s[None, :]


def _kappa_one(Xc: torch.Tensor, variant: str, p_eff: int, gap_eps=None) -> torch.Tensor:
    k, m = Xc.shape
    K = Xc @ Xc.T
    if gap_eps is None:
        sig_all, U_all = torch.linalg.eigh(K)          # ascending
        sig, Vr = _range_basis(Xc, sig_all, U_all, p_eff)
        tau = (sig / (k - 1)).sum()
        V2 = Vr * Vr
        t_range = ((Xc @ V2) ** 2).sum() / (k - 1)
        h = V2.sum(dim=1)
        t_S = ((Xc @ Vr) ** 2).sum() / (k - 1)
        G = torch.einsum("ja,al,ab->jlb", Xc, Vr, Vr)
        g = (G * G).sum() / (k - 1)
    else:
        # Regularised reading.  Every term but t_range depends on the range projector
        # M = X_c^T K^+ X_c alone; with the range of full dimension k-1 the null space of K is
        # the centring direction 1, so K^+ = inv(K + 11^T/k) - 11^T/k, whose derivative has no
        # eigen-gap factors.  t_range reads the eigenvectors through reg_eigh.
        if p_eff != k - 1 or p_eff > m:
            raise ValueError("the regularised reading needs a patch of rank k-1")
        J = torch.full((k, k), 1.0 / k, dtype=Xc.dtype)
        Kp = torch.linalg.inv(K + J) - J
        M = Xc.T @ Kp @ Xc
        h = torch.diagonal(M)
        tau = torch.trace(K) / (k - 1)
        t_S = torch.trace(K @ Kp @ K) / (k - 1)
        g = ((Xc @ (M * M)) * Xc).sum() / (k - 1)        # sum_j x_j^T (M o M) x_j
        sig_all = torch.linalg.eigvalsh(K.detach())
        eta = float(gap_eps) * float(sig_all.max())
        sr, Ur = reg_eigh(K, eta)
        _, Vt = _range_basis(Xc, sr, Ur, p_eff)
        t_range = ((Xc @ (Vt * Vt)) ** 2).sum() / (k - 1)
    t_A = ((Xc @ (1.0 - h)) ** 2).sum() / (k - 1)
    t_D = (Xc * Xc * h[None, :]).sum() / (k - 1)
    q = m - p_eff
    if q <= 0:
        t_null = torch.zeros((), dtype=Xc.dtype)
    elif variant == "paper":
        t_null = (t_A + 2.0 * (tau - 2.0 * t_S + g)) / q
    else:
        t_null = (t_A + 2.0 * (tau - 2.0 * t_D + g)) / (q + 2)
    return torch.abs(0.5 * (t_range + t_null) + 0.5 * tau)


def fast_kappa_torch(X: torch.Tensor, idx, variant: str = "paper", p_eff=None, gap_eps=None) -> torch.Tensor:
    """kappa for every row of idx (n x k) from X (n x m, float64 tensor).

    gap_eps: None (or omitted) for the exact derivative through torch's eigh; a number for
    the regularised reading (identical forward values)."""
    idx = torch.as_tensor(np.asarray(idx), dtype=torch.long)
    n, k = idx.shape
    out = []
    for i in range(n):
        P = X[idx[i]]
        Xc = P - P.mean(dim=0, keepdim=True)
        pe = (k - 1 if p_eff is None else int(p_eff[i]))
        pe = min(pe, Xc.shape[1])
        out.append(_kappa_one(Xc, variant, pe, gap_eps))
    return torch.stack(out)


def loss_and_grad(X, idx, w, variant: str = "paper", p_eff=None, gap_eps=None):
    """(L, dL/dX) for L = sum_i w_i kappa_i, X and w as arrays; float64."""
    Xt = torch.tensor(np.asarray(X, dtype=np.float64), requires_grad=True)
    wt = torch.tensor(np.asarray(w, dtype=np.float64))
    kap = fast_kappa_torch(Xt, idx, variant, p_eff, gap_eps)
    L = (wt * kap).sum()
    (g,) = torch.autograd.grad(L, Xt)
    return float(L.detach()), g.numpy()


def grad_contribution_scale(X, idx, w, variant: str = "paper", gap_eps=None) -> np.ndarray:
    """S[r, a] = sum_i |w_i| |d kappa_i / d X[r, a]|: the size of the terms that the gradient
    entry sums, which bounds the cancellation a float32 accumulation of them can suffer."""
    X = np.asarray(X, dtype=np.float64)
    idx = np.asarray(idx)
    S = np.zeros_like(X)
    for i in range(idx.shape[0]):
        if w[i] == 0.0:
            continue
        P = torch.tensor(X[idx[i]], requires_grad=True)
        Xc = P - P.mean(dim=0, keepdim=True)
        kap = _kappa_one(Xc, variant, min(idx.shape[1] - 1, X.shape[1]), gap_eps)
        (gp,) = torch.autograd.grad(kap, P)
        np.add.at(S, idx[i], abs(float(w[i])) * np.abs(gp.numpy()))
    return S
