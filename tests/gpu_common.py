"""Shared helpers of the GPU parity tests (inputs from the seeded generators only)."""
import numpy as np
import torch

from oracle import curvature as oc
from oracle import knn as ok

TOL_FP32 = 1e-4   # per-point relative error bound of the float32 path
TOL_LOW = 2e-2    # bf16 / fp8 paths
# float64 moments: the float32 output rounding (2^-24 = 6e-8) plus float64 error amplified by the
# Gram condition number (<= 1e8 on these workloads, so <= 1e-8): 1e-6 leaves a wide margin
TOL_FP64 = 1e-6


def to_dev(X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).cuda()


def oracle_fast(X32, idx, variant, rows=None):
    """Oracle kappa and the oracle's numerical rank for each row (float64 from float32 inputs)."""
    X64 = np.asarray(X32, dtype=np.float64)
    rows = np.arange(idx.shape[0]) if rows is None else rows
    kap = np.empty(len(rows))
    pe = np.empty(len(rows), dtype=np.int64)
    for r, i in enumerate(rows):
        t = oc.fast_terms(oc.patch(X64, idx[i]))
        kap[r] = t["kappa_" + variant]
        pe[r] = t["p_eff"]
    return kap, pe


def rel_err(got, want):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    return np.abs(got - want) / np.maximum(np.abs(want), 1e-30)


def knn_set_report(idx_gpu, X32, rows, k):
    """Compare GPU neighbour sets with the oracle on `rows`: (mismatches where the gap exceeds
    the float32 bound, mismatches elsewhere, number of rows with a large gap)."""
    X64 = np.asarray(X32, dtype=np.float64)
    oidx, od2, gap, d2n = ok.knn_rows(X64, rows, k)
    bound = ok.fp32_gap_bound(X32.shape[1], d2n)
    big = gap > bound
    bad_big = bad_small = 0
    for r, i in enumerate(rows):
        same = set(oidx[r].tolist()) == set(idx_gpu[i].tolist())
        if not same:
            if big[r]:
                bad_big += 1
            else:
                bad_small += 1
    return bad_big, bad_small, int(big.sum()), oidx
