"""Float64 gradient of L(X) = sum_i w_i kappa_i with the neighbour lists held fixed.

Test infrastructure only.  The forward pass restates the Fast branch of
Algorithm 1 (centring, truncated SVD, t_range, t_A, t_B, t_null, eq.
fast_curv) in PyTorch float64 on the CPU so that autograd supplies the exact
derivative.  The truncated SVD is taken from the eigen-decomposition of the
k x k Gram matrix X_c X_c^T (its non-zero eigenpairs are s_l^2 and the left
singular vectors; V_r = X_c^T U_p diag(1/s_p)); this is the same factorisation
as SVD_p and avoids differentiating through the always-zero singular value of
a centred patch.  Pinned by central finite differences, the Euler identity of
a degree-2 homogeneous function, translation invariance and agreement of the
forward value with ``oracle.curvature.fast_kappa``.
"""
from __future__ import annotations

import numpy as np
import torch

__all__ = ["fast_kappa_torch", "loss_and_grad"]


def _kappa_one(Xc: torch.Tensor, variant: str, p_eff: int) -> torch.Tensor:
    k, m = Xc.shape
    K = Xc @ Xc.T
    sig, U = torch.linalg.eigh(K)                 # ascending
    sig = sig.flip(0)[:p_eff]
    U = U.flip(1)[:, :p_eff]
    s = torch.sqrt(sig)
    Vr = (Xc.T @ U) / s[None, :]                  # right singular vectors, m x p
    tau = (sig / (k - 1)).sum()
    V2 = Vr * Vr
    t_range = ((Xc @ V2) ** 2).sum() / (k - 1)
    h = V2.sum(dim=1)
    t_A = ((Xc @ (1.0 - h)) ** 2).sum() / (k - 1)
    t_S = ((Xc @ Vr) ** 2).sum() / (k - 1)
    G = torch.einsum("ja,al,ab->jlb", Xc, Vr, Vr)
    g = (G * G).sum() / (k - 1)
    t_D = (Xc * Xc * h[None, :]).sum() / (k - 1)
    q = m - p_eff
    if q <= 0:
        t_null = torch.zeros((), dtype=Xc.dtype)
    elif variant == "paper":
        t_null = (t_A + 2.0 * (tau - 2.0 * t_S + g)) / q
    else:
        t_null = (t_A + 2.0 * (tau - 2.0 * t_D + g)) / (q + 2)
    return torch.abs(0.5 * (t_range + t_null) + 0.5 * tau)


def fast_kappa_torch(X: torch.Tensor, idx, variant: str = "paper", p_eff=None) -> torch.Tensor:
    """kappa for every row of idx (n x k) from X (n x m, float64 tensor)."""
    idx = torch.as_tensor(np.asarray(idx), dtype=torch.long)
    n, k = idx.shape
    out = []
    for i in range(n):
        P = X[idx[i]]
        Xc = P - P.mean(dim=0, keepdim=True)
        pe = (k - 1 if p_eff is None else int(p_eff[i]))
        pe = min(pe, Xc.shape[1])
        out.append(_kappa_one(Xc, variant, pe))
    return torch.stack(out)


def loss_and_grad(X, idx, w, variant: str = "paper", p_eff=None):
    """(L, dL/dX) for L = sum_i w_i kappa_i, X and w as arrays; float64."""
    Xt = torch.tensor(np.asarray(X, dtype=np.float64), requires_grad=True)
    wt = torch.tensor(np.asarray(w, dtype=np.float64))
    kap = fast_kappa_torch(Xt, idx, variant, p_eff)
    L = (wt * kap).sum()
    (g,) = torch.autograd.grad(L, Xt)
    return float(L.detach()), g.numpy()
