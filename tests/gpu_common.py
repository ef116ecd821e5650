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
    the float32 bound, mismatches elsewhere, number of rows with a large gap).

    Where several sets are correct (the k-th and (k+1)-th distances lie within the float32
    rounding bound delta of each other) a differing set must still be admissible: every point
    it holds lies within d_(k) + delta, every oracle neighbour it leaves out at d_(k) - delta or
    beyond, and it holds k distinct points other than the query.  An inadmissible set counts as
    a mismatch above the bound."""
    X64 = np.asarray(X32, dtype=np.float64)
    oidx, od2, gap, d2n = ok.knn_rows(X64, rows, k)
    bound = ok.fp32_gap_bound(X32.shape[1], d2n)
    big = gap > bound
    bad_big = bad_small = 0
    for r, i in enumerate(rows):
        gset, oset = set(idx_gpu[i].tolist()), set(oidx[r].tolist())
        if gset == oset:
            continue
        if big[r]:
            bad_big += 1
            continue
        dk = od2[r][-1]
        g = np.array(sorted(gset))
        dg = ((X64[g] - X64[i]) ** 2).sum(1)
        left = np.array(sorted(oset - gset))
        dl = ((X64[left] - X64[i]) ** 2).sum(1)
        admissible = (len(gset) == k and i not in gset and np.all(dg <= dk + bound[r])
                      and np.all(dl >= dk - bound[r]))
        if admissible:
            bad_small += 1
        else:
            bad_big += 1
    return bad_big, bad_small, int(big.sum()), oidx
