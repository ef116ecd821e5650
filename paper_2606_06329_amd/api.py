"""Python surface of the mean-curvature hot path: argument marshalling onto the C ABI.

Every step runs in the HIP kernels of libmecuco.so; tensors supply device
memory and the current stream.  Names follow the paper: k neighbours, the
Fast branch of Algorithm 1 (``curvature_fast``), Theorem 1 with a canonical
null basis (``curvature_exact``), and Auto mode (exact when D < 50).
"""
from __future__ import annotations

import math

import torch

from . import _lib as L

_PREC = {"fp32": L.MC_FP32, "bf16": L.MC_BF16, "fp8": L.MC_FP8, "fp64": L.MC_FP64}
_VAR = {"paper": L.MC_FAST_PAPER, "haar": L.MC_FAST_HAAR}


def _stream(t: torch.Tensor) -> int:
    return torch.cuda.current_stream(t.device).cuda_stream


def _cloud(X: torch.Tensor):
    if not (isinstance(X, torch.Tensor) and X.is_cuda and X.dtype == torch.float32 and X.dim() == 2):
        raise TypeError("X must be a 2-D float32 CUDA tensor")
    if X.stride(1) != 1:
        raise ValueError("X rows must be contiguous (stride(1) == 1)")
    n, m = X.shape
    return n, m, X.stride(0)


def _idx(idx: torch.Tensor, n: int, k: int, device) -> torch.Tensor:
    if not (isinstance(idx, torch.Tensor) and idx.dtype == torch.int32 and idx.device == device):
        raise TypeError("idx must be an int32 tensor on the same device as X")
    if tuple(idx.shape) != (n, k) or not idx.is_contiguous():
        raise ValueError(f"idx must be contiguous with shape ({n}, {k})")
    return idx


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def workspace_bytes(op: int, n: int, m: int, k: int, precision: str = "fp32", rerank: int = 2) -> int:
    return int(L.lib().mc_workspace_bytes(op, n, m, k, _PREC[precision], rerank))


def default_rerank(k: int, n: int, precision: str = "fp32") -> int:
    """Candidates per neighbour for the float32 re-rank: 2 on the float32 and bf16 GEMMs; fp8
    keeps as many as the 64-entry lists allow (up to 4), since e4m3 scores order close
    neighbours coarsely."""
    r = 2 if precision in ("fp32", "bf16") else max(2, min(4, 64 // max(k, 1)))
    while r > 1 and r * k >= n:
        r -= 1
    return r


# the library's workspace limit for the symmetric tile-pair schedule (one 64 KiB transposed
# score tile per unordered pair of 128-point tiles)
KNN_SYM_MAX_BYTES = 32 << 30


def knn_symmetric(n: int) -> bool:
    """Whether mc_knn scores each unordered pair of 128-point tiles once (n up to 131072)
    rather than every ordered pair: its distance GEMM then does n (n + 1) m flop, not 2 n^2 m."""
    T = -(-int(n) // 128)
    return T >= 2 and (T * (T - 1) // 2) * 65536 <= KNN_SYM_MAX_BYTES


def knn(X: torch.Tensor, k: int, precision: str = "fp32", rerank: int | None = None,
        include_self: bool = False, strict: bool = False, ws: torch.Tensor | None = None):
    """k nearest neighbours of every row of X (Step 1): (idx int32 n x k, d2 float32 n x k, flags uint8 n).

    rerank: candidates per neighbour kept from the GEMM for the float32 re-rank (None: default_rerank).
    """
    n, m, ldx = _cloud(X)
    if rerank is None:
        rerank = default_rerank(k, n, precision)
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float32, device=X.device)
    fl = torch.empty((n,), dtype=torch.uint8, device=X.device)
    need = L.lib().mc_workspace_bytes(L.MC_OP_KNN, n, m, k, _PREC[precision], rerank)
    if ws is None or ws.numel() < need:
        ws = _workspace(need, X.device)
    flags = (L.MC_INCLUDE_SELF if include_self else 0) | (L.MC_STRICT if strict else 0)
    st = L.lib().mc_knn(X.data_ptr(), n, m, ldx, k, _PREC[precision], rerank, flags, idx.data_ptr(),
                        d2.data_ptr(), fl.data_ptr(), ws.data_ptr(), ws.numel(), _stream(X))
    L.check(st, "mc_knn")
    return idx, d2, fl


def curvature_fast(X: torch.Tensor, idx: torch.Tensor, variant: str = "paper",
                   precision: str = "fp32", strict: bool = False):
    """Fast branch of Algorithm 1 for every point: (kappa float32 n, flags uint8 n)."""
    n, m, ldx = _cloud(X)
    k = idx.shape[1]
    _idx(idx, n, k, X.device)
    kap = torch.empty((n,), dtype=torch.float32, device=X.device)
    fl = torch.empty((n,), dtype=torch.uint8, device=X.device)
    ws = _workspace(L.lib().mc_workspace_bytes(L.MC_OP_FAST, n, m, k, _PREC[precision], 1), X.device)
    st = L.lib().mc_curvature_fast(X.data_ptr(), n, m, ldx, idx.data_ptr(), k, _PREC[precision],
                                   _VAR[variant], L.MC_STRICT if strict else 0, kap.data_ptr(),
                                   fl.data_ptr(), ws.data_ptr(), ws.numel(), _stream(X))
    L.check(st, "mc_curvature_fast")
    return kap, fl


def exact_supported(m: int, k: int) -> bool:
    """Whether mc_curvature_exact accepts these sizes (its per-point state must fit on chip)."""
    return L.lib().mc_workspace_bytes(L.MC_OP_EXACT, k + 1, m, k, L.MC_FP32, 1) > 0


def curvature_exact(X: torch.Tensor, idx: torch.Tensor, strict: bool = False):
    """Theorem 1 with the canonical (Householder) null basis: (kappa float32 n, flags uint8 n)."""
    n, m, ldx = _cloud(X)
    k = idx.shape[1]
    _idx(idx, n, k, X.device)
    kap = torch.empty((n,), dtype=torch.float32, device=X.device)
    fl = torch.empty((n,), dtype=torch.uint8, device=X.device)
    ws = _workspace(L.lib().mc_workspace_bytes(L.MC_OP_EXACT, n, m, k, L.MC_FP32, 1), X.device)
    st = L.lib().mc_curvature_exact(X.data_ptr(), n, m, ldx, idx.data_ptr(), k, L.MC_FP32,
                                    L.MC_STRICT if strict else 0, kap.data_ptr(), fl.data_ptr(),
                                    ws.data_ptr(), ws.numel(), _stream(X))
    L.check(st, "mc_curvature_exact")
    return kap, fl


def curvature_backward(X: torch.Tensor, idx: torch.Tensor, grad_kappa: torch.Tensor,
                       variant: str = "paper", gap_eps: float = 0.0, grad_X: torch.Tensor | None = None):
    """grad_X += d(sum_i grad_kappa_i kappa_i)/dX with idx fixed (adjoint of curvature_fast, fp32)."""
    n, m, ldx = _cloud(X)
    k = idx.shape[1]
    _idx(idx, n, k, X.device)
    if grad_X is None:
        # same row stride as X (a column slice of a wider matrix keeps its ldx)
        grad_X = torch.zeros((n, ldx), dtype=torch.float32, device=X.device)[:, :m]
    if (grad_X.shape != X.shape or grad_X.stride() != X.stride() or grad_X.dtype != torch.float32
            or grad_X.device != X.device):
        raise ValueError("grad_X must match X in shape, stride, dtype and device")
    if not (isinstance(grad_kappa, torch.Tensor) and grad_kappa.device == X.device
            and grad_kappa.dim() == 1 and grad_kappa.numel() == n):
        raise ValueError(f"grad_kappa must be a length-{n} vector on X's device")
    gk = grad_kappa.contiguous().to(torch.float32)
    ws = _workspace(L.lib().mc_workspace_bytes(L.MC_OP_BACKWARD, n, m, k, L.MC_FP32, 1), X.device)
    st = L.lib().mc_curvature_backward(X.data_ptr(), n, m, ldx, idx.data_ptr(), k, _VAR[variant],
                                       gk.data_ptr(), float(gap_eps), grad_X.data_ptr(), ws.data_ptr(),
                                       ws.numel(), _stream(X))
    L.check(st, "mc_curvature_backward")
    return grad_X


class MeanCurvature(torch.autograd.Function):
    """kappa = MeanCurvature.apply(X, idx, variant, gap_eps); differentiable in X, idx fixed."""

    @staticmethod
    def forward(ctx, X, idx, variant="paper", gap_eps=0.0):
        kap, _ = curvature_fast(X, idx, variant, "fp32")
        ctx.save_for_backward(X, idx)
        ctx.variant = variant
        ctx.gap_eps = gap_eps
        return kap

    @staticmethod
    def backward(ctx, gk):
        X, idx = ctx.saved_tensors
        g = curvature_backward(X, idx, gk, ctx.variant, ctx.gap_eps)
        return g, None, None, None


def normalize_minmax(kappa: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """(kappa - min) / (max - min) over the finite scores: the per-dataset normalisation to
    [0, 1] of the paper's normalised-score experiment (NaN stays NaN, constant scores give 0)."""
    if not (isinstance(kappa, torch.Tensor) and kappa.is_cuda and kappa.dtype == torch.float32
            and kappa.dim() == 1 and kappa.is_contiguous()):
        raise TypeError("kappa must be a contiguous 1-D float32 CUDA tensor")
    n = kappa.numel()
    if out is None:
        out = torch.empty_like(kappa)
    if out.shape != kappa.shape or out.dtype != torch.float32 or out.device != kappa.device or not out.is_contiguous():
        raise ValueError("out must match kappa")
    ws = _workspace(L.lib().mc_workspace_bytes(L.MC_OP_NORMALIZE, n, 1, 2, 0, 1), kappa.device)
    st = L.lib().mc_normalize_minmax(kappa.data_ptr(), n, out.data_ptr(), ws.data_ptr(), ws.numel(),
                                     _stream(kappa))
    L.check(st, "mc_normalize_minmax")
    return out


def default_k(n: int) -> int:
    """k = floor(log2 n), the paper's default neighbourhood size (clamped to the supported range)."""
    return max(2, min(L.MC_KMAX, int(math.floor(math.log2(max(n, 2))))))


def curvature(X: torch.Tensor, k: int | None = None, mode: str = "auto", precision: str = "fp32",
              variant: str = "paper", idx: torch.Tensor | None = None, normalize: bool = False):
    """Algorithm 1 end to end: kNN graph then per-point curvature.

    mode "auto" selects the exact identity when D < 50 and the fast estimator otherwise.
    precision: "fp32" | "bf16" | "fp8" (kNN GEMM in fp8, moments in bf16) | "fp64"
    (float32 kNN, float64 moments).  normalize: min-max normalise the scores to [0, 1].
    Returns (kappa, idx, flags) with flags the OR of the kNN and curvature flags.
    """
    n, m, _ = _cloud(X)
    k = default_k(n) if k is None else int(k)
    kfl = None
    if idx is None:
        kprec = {"fp32": "fp32", "fp64": "fp32", "bf16": "bf16", "fp8": "fp8"}[precision]
        idx, _, kfl = knn(X, k, precision=kprec)
    if mode == "auto":
        mode = "exact" if m < 50 else "fast"
    if mode == "exact":
        kap, fl = curvature_exact(X, idx)
    elif mode == "fast":
        cprec = {"fp32": "fp32", "fp64": "fp64", "bf16": "bf16", "fp8": "bf16"}[precision]
        kap, fl = curvature_fast(X, idx, variant, cprec)
    else:
        raise ValueError(mode)
    if kfl is not None:
        fl = fl | kfl
    if normalize:
        kap = normalize_minmax(kap, out=kap)
    return kap, idx, fl
