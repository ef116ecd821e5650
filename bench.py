#!/usr/bin/env python3
"""Throughput of the mean-curvature hot path on one MI355X.

One step = the whole hot path over the workload: mc_knn (MFMA distance GEMM +
top-K' + float32 re-rank) followed by mc_curvature_fast (Fast branch of
Algorithm 1), inputs resident in HBM.  The headline workload is the
20000 x 784 cluster cloud (k = 11, float32 path).

Prints ONE JSON line with the metric, a roofline entry for the dominant kernel
(timed with the library's own hipEvent stage timers on the launch stream) and
the float64 oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "bf16": 2500.0}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                          # GB/s


def cpu_baseline(X, k, variant, budget_s=15.0):
    """The oracle as it stands (kNN rows + Fast curvature) on a bounded sample of points."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import curvature as oc
    from oracle import knn as ok

    X64 = X.astype(np.float64)
    n = X.shape[0]
    rng = np.random.default_rng(123)
    order = rng.permutation(n)
    done = 0
    kap = {}
    t0 = time.perf_counter()
    with threadpool_limits(limits=1):
        while done < n and time.perf_counter() - t0 < budget_s:
            rows = order[done:done + 4]
            idx, _, _, _ = ok.knn_rows(X64, rows, k)
            for r, i in enumerate(rows):
                kap[int(i)] = (oc.fast_kappa(oc.patch(X64, idx[r]), variant), idx[r])
            done += len(rows)
    el = time.perf_counter() - t0
    return {"value": done / el, "unit": "points/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} random points of the same workload: exact float64 kNN row "
                      f"(difference form over all {n} points) + Fast curvature, 1 BLAS thread, "
                      f"{el:.1f} s"}, kap


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clusters")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16"])
    ap.add_argument("--variant", default="paper", choices=["paper", "haar"])
    ap.add_argument("--rerank", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib, synth

    X, k = synth.make(args.workload)
    n, m = X.shape
    Xd = torch.from_numpy(X).cuda()
    prec = args.precision
    ws = torch.empty(P.workspace_bytes(_lib.MC_OP_KNN, n, m, k, prec, args.rerank),
                     dtype=torch.uint8, device="cuda")

    def step():
        idx, _, kfl = P.knn(Xd, k, precision=prec, rerank=args.rerank, ws=ws)
        kap, fl = P.curvature_fast(Xd, idx, args.variant, prec)
        return idx, kap, fl | kfl

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                 # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    _lib.timing_read()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    ms_step = ms_total / args.steps
    value = n * args.steps / (ms_total / 1e3)

    gemm_ms, gemm_cnt = stages.get("knn_gemm_topk", (float("nan"), 1))
    gemm_avg = gemm_ms / gemm_cnt
    flops = 2.0 * n * n * m                      # algorithmic distance-GEMM work per launch
    achieved = flops / (gemm_avg / 1e3) / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK[prec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[prec], 4), "traffic": None,
            "kernel": "knn_gemm_topk", "kernel_ms": round(gemm_avg, 4),
            "work": f"2*n*n*m = {flops:.4g} flop per launch"}

    idx, kap, fl = out
    kap_np = kap.cpu().numpy()
    fl_np = fl.cpu().numpy()
    res = {
        "metric": "curvature points/sec (kNN+SVD+identity), fast estimator",
        "value": round(value, 1),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == "fp32" else "bf16",
        "data": "synthetic",
        "config": {"workload": f"{args.workload} n={n} m={m} k={k}", "n": n, "m": m, "k": k,
                   "precision": prec, "variant": args.variant, "rerank": args.rerank,
                   "mode": "fast"},
        "roofline": roof,
        "stages_ms": {s: round(v[0] / v[1], 4) for s, v in stages.items()},
        "flags": {"rank_deficient": int(((fl_np & 4) != 0).sum()),
                  "knn_uncertified": int(((fl_np & 32) != 0).sum()),
                  "knn_ambiguous": int(((fl_np & 16) != 0).sum())},
    }
    if not args.no_cpu_baseline:
        cb, kap_o = cpu_baseline(X, k, args.variant)
        res["cpu_baseline"] = cb
        idx_np = idx.cpu().numpy()
        errs = []
        for i, (kv, oi) in kap_o.items():
            if set(oi.tolist()) == set(idx_np[i].tolist()) and not (fl_np[i] & 4):
                errs.append(abs(kap_np[i] - kv) / kv)
        if errs:
            res["error_vs_oracle"] = {"points": len(errs), "max_rel": float(np.max(errs)),
                                      "median_rel": float(np.median(errs))}
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
