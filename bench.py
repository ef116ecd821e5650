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

PEAK = {"fp32": 157.3, "bf16": 2500.0, "fp8": 5000.0}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                                          # GB/s
# precision option -> (kNN GEMM precision, curvature moment precision, reported dtype)
PRECISIONS = {"fp32": ("fp32", "fp32", "f32"), "bf16": ("bf16", "bf16", "bf16"),
              "fp8": ("fp8", "bf16", "fp8/bf16"), "fp64": ("fp32", "fp64", "f32/f64")}
KNN_SOURCES = ("paper_2606_06329_amd/csrc/knn.hip", "paper_2606_06329_amd/csrc/mc_device.h")


HOST_MARK = b"// host side"   # knn.hip's launch code starts here; it does not change the kernels


def source_digest(paths=KNN_SOURCES):
    """sha256 over the device code the distance-GEMM kernel is built from (each file up to
    its host section)."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            data = f.read()
        cut = data.find(HOST_MARK)
        h.update(data if cut < 0 else data[:cut])
    return h.hexdigest()[:16]


def profiled_traffic(workload, prec):
    """HBM bytes per launch of knn_gemm_topk from the committed counter summary, or None when
    there is none for this workload or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"knn_gemm_topk_{workload}_{prec}.md")
    if not os.path.exists(path):
        return None, "no counter summary"
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            key, val = line[2:].split(": ", 1)
            fields[key.strip().strip("`")] = val.strip().strip("`")
    if fields.get("source_digest") != source_digest():
        return None, "kernel changed since the counters were taken"
    try:
        return int(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    except (KeyError, ValueError):
        return None, "summary has no traffic line"


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


def time_path(P, _lib, torch, Xd, k, prec, mode, variant, rerank, steps, warmup):
    """Run `steps` timed passes of the hot path (kNN + curvature) after `warmup` untimed ones.
    Returns (ms per step, library stage timers {name: (ms, launches)}, last outputs)."""
    kprec, cprec, _ = PRECISIONS[prec]
    n, m = Xd.shape
    if rerank is None:
        rerank = P.default_rerank(k, n, kprec)
    ws = torch.empty(P.workspace_bytes(_lib.MC_OP_KNN, n, m, k, kprec, rerank),
                     dtype=torch.uint8, device="cuda")

    def step():
        idx, _, kfl = P.knn(Xd, k, precision=kprec, rerank=rerank, ws=ws)
        if mode == "exact":
            kap, fl = P.curvature_exact(Xd, idx)
        else:
            kap, fl = P.curvature_fast(Xd, idx, variant, cprec)
        return idx, kap, fl | kfl

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    _lib.timing_enable(True)
    _lib.timing_read()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        out = step()
    ev1.record()
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    stages = _lib.timing_read()
    _lib.timing_enable(False)
    return ms_total / steps, stages, out, rerank


def errors_vs_oracle(kap_o, idx_np, kap_np, fl_np):
    """Per-point relative error on the oracle's sample, over points whose neighbour set equals
    the oracle's and whose patch has full numerical rank; plus the count of differing sets."""
    import numpy as np
    errs, diff_sets = [], 0
    for i, (kv, oi) in kap_o.items():
        if set(oi.tolist()) != set(idx_np[i].tolist()):
            diff_sets += 1
            continue
        if not (fl_np[i] & 4):
            errs.append(abs(float(kap_np[i]) - kv) / kv)
    out = {"points": len(errs), "knn_sets_differing": diff_sets}
    if errs:
        out.update(max_rel=float(np.max(errs)), median_rel=float(np.median(errs)))
    return out


def oracle_sample(X, k, rows, variant):
    """Oracle neighbour lists and Fast kappa of the sampled rows (float64 from the float32 input)."""
    import numpy as np

    from oracle import curvature as oc
    from oracle import knn as ok

    X64 = X.astype(np.float64)
    idx, _, _, _ = ok.knn_rows(X64, rows, k)
    kap = {int(i): (oc.fast_kappa(oc.patch(X64, idx[r]), variant), idx[r]) for r, i in enumerate(rows)}
    return kap


def suite(args):
    """Secondary configurations, one JSON line each: the other workloads at their own sizes and
    precision paths, errors against the oracle on a sampled set of points."""
    import numpy as np
    import torch

    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib, synth

    # (workload, precisions, exact mode too, n override, k override); the last entry is the
    # cluster cloud at the paper's MNIST_784 shape (n = 70000, k = log2 n = 16), for context
    plan = [("sphere", ("fp32",), True, None, None), ("torus", ("fp32", "bf16"), False, None, None),
            ("swissroll", ("fp32",), False, None, None), ("blobs", ("fp32", "fp8"), False, None, None),
            ("clusters", ("fp32", "bf16"), False, 70000, 16)]
    for name, precs, with_exact, n_over, k_over in plan:
        X, k = synth.make(name, n=n_over)
        k = k_over or k
        n, m = X.shape
        Xd = torch.from_numpy(X).cuda()
        rows = np.random.default_rng(11).choice(n, min(n, 120 if m < 1000 else 40), replace=False)
        t0 = time.perf_counter()
        kap_o = oracle_sample(X, k, rows, args.variant)
        t_or = (time.perf_counter() - t0) / len(rows)
        for prec in precs:
            steps = 2 if n * n * m > 1e12 else 5
            ms, st, out, rr = time_path(P, _lib, torch, Xd, k, prec, "fast", args.variant, None, steps, 1)
            idx, kap, fl = out
            line = {"suite": name, "n": n, "m": m, "k": k, "precision": prec, "mode": "fast",
                    "dtype": PRECISIONS[prec][2], "rerank": rr, "points_per_s": round(n / (ms / 1e3), 1),
                    "ms_per_step": round(ms, 4),
                    "stages_ms": {a: round(v[0] / v[1], 4) for a, v in st.items()},
                    "error_vs_oracle": errors_vs_oracle(kap_o, idx.cpu().numpy(), kap.cpu().numpy(),
                                                        fl.cpu().numpy()),
                    "eigen_fp64_points": int(((fl.cpu().numpy() & 64) != 0).sum()),
                    "oracle_s_per_point_1core": round(t_or, 4)}
            if name == "swissroll":
                # forward + adjoint of sum_i w_i kappa_i, neighbour lists fixed
                w = torch.from_numpy(synth.loss_weights(n)).cuda()
                g = torch.zeros_like(Xd)
                for _ in range(2):
                    P.curvature_backward(Xd, idx, w, args.variant, 0.0, g)
                torch.cuda.synchronize()
                _lib.timing_enable(True)
                _lib.timing_read()
                for _ in range(steps):
                    P.curvature_backward(Xd, idx, w, args.variant, 0.0, g)
                torch.cuda.synchronize()
                bt = _lib.timing_read()
                _lib.timing_enable(False)
                b_ms, b_cnt = bt.get("curv_backward", (float("nan"), 1))
                line["backward_ms"] = round(b_ms / b_cnt, 4)
            print(json.dumps(line), flush=True)
        if with_exact:
            ms, st, out, rr = time_path(P, _lib, torch, Xd, k, "fp32", "exact", args.variant, None, 5, 1)
            print(json.dumps({"suite": name, "n": n, "m": m, "k": k, "precision": "fp32", "mode": "exact",
                              "points_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                              "stages_ms": {a: round(v[0] / v[1], 4) for a, v in st.items()}}), flush=True)
        del Xd
        torch.cuda.empty_cache()


def sweep(args):
    """Fast-vs-exact agreement against m/k on synthetic manifolds: one JSON line per case with
    the relative error of both Fast readings against the exact value (canonical basis), the
    paper's three agreement criteria, and on a small sample the oracle's exact value with the
    LAPACK eigenbasis (the Exact branch as printed) against the canonical one."""
    import numpy as np
    import torch

    import paper_2606_06329_amd as P
    from oracle import curvature as oc
    from paper_2606_06329_amd import metrics, synth

    n = 2000
    cases = [("torus", m, 8) for m in (16, 32, 64, 128, 256, 512, 800)]
    cases += [("swissroll", m, 8) for m in (16, 64, 256, 800)]
    cases += [("torus", m, 16) for m in (32, 128, 512, 1000)]
    for name, m, k in cases:
        if not P.exact_supported(m, k):
            continue
        X = synth.WORKLOADS[name][0](n=n, m=m, seed=7000 + m + k)
        Xd = torch.from_numpy(X).cuda()
        idx, _, kfl = P.knn(Xd, k)
        ex, efl = P.curvature_exact(Xd, idx)
        line = {"sweep": name, "n": n, "m": m, "k": k, "m_over_k": round(m / k, 2)}
        ex_np = ex.cpu().numpy().astype(np.float64)
        ok = ((efl | kfl).cpu().numpy() & 0x0E) == 0        # no degenerate / rank / sweep flags
        for variant in ("paper", "haar"):
            fa, _ = P.curvature_fast(Xd, idx, variant)
            fa = fa.cpu().numpy().astype(np.float64)
            rel = np.abs(fa - ex_np)[ok] / ex_np[ok]
            ag = metrics.agreement(ex_np[ok], fa[ok])
            line[variant] = {"median_rel": float(np.median(rel)), "p90_rel": float(np.quantile(rel, 0.9)),
                             "mae": ag["mae"], "spearman": ag["spearman"], "xi": ag["xi"]}
        # the printed Exact branch (LAPACK eigenbasis of the m x m covariance) on a sample
        X64 = X.astype(np.float64)
        idx_np = idx.cpu().numpy()
        rows = [i for i in range(0, n, n // 40) if ok[i]][:30]
        lap = np.array([oc.lapack_exact_kappa(oc.patch(X64, idx_np[i])) for i in rows])
        line["lapack_vs_canonical_median_rel"] = float(np.median(np.abs(lap - ex_np[rows]) / ex_np[rows]))
        for variant in ("paper", "haar"):
            fa, _ = P.curvature_fast(Xd, idx, variant)
            fa = fa.cpu().numpy().astype(np.float64)[rows]
            rel = np.abs(fa - lap) / lap
            line[variant]["vs_lapack_median_rel"] = float(np.median(rel))
            line[variant]["vs_lapack_max_rel"] = float(np.max(rel))
        line["points"] = int(ok.sum())
        print(json.dumps(line), flush=True)
        del Xd


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clusters")
    ap.add_argument("--precision", default="fp32", choices=list(PRECISIONS))
    ap.add_argument("--variant", default="paper", choices=["paper", "haar"])
    ap.add_argument("--rerank", type=int, default=None,
                    help="candidates per neighbour for the float32 re-rank (default: per precision)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the secondary measurements (other precisions, exact mode)")
    ap.add_argument("--sweep", action="store_true",
                    help="instead of the headline line, the Fast-vs-exact agreement sweep over m/k")
    ap.add_argument("--suite", action="store_true",
                    help="instead of the headline line, one line per secondary configuration")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (counter calibration for rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(multi-GPU sharding is design-only)", file=sys.stderr)
        sys.exit(2)

    if args.suite:
        suite(args)
        return
    if args.sweep:
        sweep(args)
        return

    import numpy as np
    import torch

    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib, synth

    X, k = synth.make(args.workload)
    n, m = X.shape
    Xd = torch.from_numpy(X).cuda()
    prec = args.precision
    kprec, cprec, dtype = PRECISIONS[prec]

    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)                 # reads and writes exactly 256 MiB
        torch.cuda.synchronize()
        del src, dst

    ms_step, stages, out, rerank = time_path(P, _lib, torch, Xd, k, prec, "fast", args.variant,
                                             args.rerank, args.steps, args.warmup)
    value = n / (ms_step / 1e3)

    gemm_ms, gemm_cnt = stages.get("knn_gemm_topk", (float("nan"), 1))
    gemm_avg = gemm_ms / gemm_cnt
    # algorithmic distance-GEMM work per launch: every unordered pair (self included) once
    # under the symmetric tile-pair schedule, every ordered pair otherwise
    sym = P.knn_symmetric(n)
    flops = float(n) * (n + 1) * m if sym else 2.0 * n * n * m
    achieved = flops / (gemm_avg / 1e3) / 1e12
    traffic, traffic_src = profiled_traffic(args.workload, kprec)
    roof = {"bound": "mfma", "achieved": round(achieved, 2), "peak": PEAK[kprec], "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[kprec], 4), "traffic": traffic,
            "kernel": "knn_gemm_topk", "kernel_ms": round(gemm_avg, 4),
            "work": (f"n*(n+1)*m = {flops:.4g} flop per launch (symmetric schedule)" if sym
                     else f"2*n*n*m = {flops:.4g} flop per launch"),
            "traffic_source": traffic_src}

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
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": f"{args.workload} n={n} m={m} k={k}", "n": n, "m": m, "k": k,
                   "precision": prec, "variant": args.variant, "rerank": rerank,
                   "mode": "fast"},
        "roofline": roof,
        "stages_ms": {s: round(v[0] / v[1], 4) for s, v in stages.items()},
        "flags": {"rank_deficient": int(((fl_np & 4) != 0).sum()),
                  "knn_uncertified": int(((fl_np & 32) != 0).sum()),
                  "knn_ambiguous": int(((fl_np & 16) != 0).sum()),
                  "eigen_fp64": int(((fl_np & 64) != 0).sum())},
    }
    kap_o = None
    if not args.no_cpu_baseline:
        cb, kap_o = cpu_baseline(X, k, args.variant)
        res["cpu_baseline"] = cb
        res["error_vs_oracle"] = errors_vs_oracle(kap_o, idx.cpu().numpy(), kap_np, fl_np)

    if not args.no_modes:
        # the same workload through the other precisions and the exact mode, timed the same way
        modes = []
        for mprec, mmode in (("bf16", "fast"), ("fp8", "fast"), ("fp64", "fast"), ("fp32", "exact")):
            if (mprec, mmode) == (prec, "fast"):
                continue
            if mmode == "exact" and not P.exact_supported(m, k):
                continue
            steps = max(2, args.steps // 2)
            mms, mst, mout, mrr = time_path(P, _lib, torch, Xd, k, mprec, mmode, args.variant,
                                            args.rerank, steps, 1)
            entry = {"precision": mprec, "mode": mmode, "dtype": PRECISIONS[mprec][2], "rerank": mrr,
                     "points_per_s": round(n / (mms / 1e3), 1), "ms_per_step": round(mms, 4),
                     "stages_ms": {s: round(v[0] / v[1], 4) for s, v in mst.items()}}
            if kap_o is not None:
                midx, mkap, mfl = mout
                if mmode == "fast":
                    entry["error_vs_oracle"] = errors_vs_oracle(kap_o, midx.cpu().numpy(),
                                                                mkap.cpu().numpy(), mfl.cpu().numpy())
            modes.append(entry)
        res["modes"] = modes
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
