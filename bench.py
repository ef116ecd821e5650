#!/usr/bin/env python3
"""Throughput of the mean-curvature hot path on one MI355X.

One step = the whole hot path over the workload: mc_knn (MFMA distance GEMM +
top-K' + float32 re-rank + certificate, and the rescan of uncertified queries)
followed by mc_curvature_fast (Fast branch of Algorithm 1), inputs resident in
HBM.  The headline workload is the largest configuration, the 50000 x 4096 blob
mixture with k = 32: fp8 e4m3 distance GEMM with per-row scales and a float32
re-rank of 64 candidates, Gram from split bf16 products (x = hi + lo), float32
eigen-solve, range GEMM on binary16 operands (the bf16 curvature path).

Prints ONE JSON line with the metric, a roofline entry for the dominant kernel
(timed with the library's hipEvent stage timers on the launch stream), the
float64 oracle timed on a bounded sample on the host's cores, and the other
precision paths (float32 and bf16 on the same workload; bf16 vs float32 on the
100000 x 256 torus) as `modes`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32": 157.3, "bf16": 2500.0, "f16": 2500.0, "fp8": 5000.0, "fp64": 78.6}   # dense MFMA TFLOP/s, MI355X
HBM_PEAK = 8000.0                                                      # GB/s
# precision option -> (kNN GEMM precision, curvature moment precision, reported dtype)
# (the bf16 curvature path's two-pass form, k >= 13, runs its range GEMM on binary16)
PRECISIONS = {"fp32": ("fp32", "fp32", "f32"), "bf16": ("bf16", "bf16", "bf16/f16"),
              "fp8": ("fp8", "bf16", "fp8/bf16/f16"), "fp64": ("fp32", "fp64", "f32/f64")}
# device sources of each kernel whose counters a profile summary records
KERNEL_SOURCES = {
    "knn_gemm_topk": ("paper_2606_06329_amd/csrc/knn.hip", "paper_2606_06329_amd/csrc/mc_device.h"),
    "curv_range": ("paper_2606_06329_amd/csrc/curv_fast2.hip", "paper_2606_06329_amd/csrc/curv_core.h",
                   "paper_2606_06329_amd/csrc/mc_device.h"),
    "curv_gram": ("paper_2606_06329_amd/csrc/curv_fast2.hip", "paper_2606_06329_amd/csrc/curv_core.h",
                  "paper_2606_06329_amd/csrc/mc_device.h"),
}
HOST_MARK = b"// host side"   # knn.hip's launch code starts here; it does not change the kernels
MAX_CPU_WORKERS = 16          # the host share of one GPU


def source_digest(paths):
    """sha256 over the device code a kernel is built from (each file up to its host section)."""
    import hashlib
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            data = f.read()
        cut = data.find(HOST_MARK)
        h.update(data if cut < 0 else data[:cut])
    return h.hexdigest()[:16]


def profiled_traffic(kernel, workload, prec):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None when there
    is none for this workload or the kernel's sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{prec}.md")
    if not os.path.exists(path) or kernel not in KERNEL_SOURCES:
        return None, "no counter summary"
    fields = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            key, val = line[2:].split(": ", 1)
            fields[key.strip().strip("`")] = val.strip().strip("`")
    if fields.get("source_digest") != source_digest(KERNEL_SOURCES[kernel]):
        return None, "kernel changed since the counters were taken"
    try:
        return int(fields["traffic_bytes_per_launch"]), os.path.relpath(path, ROOT)
    except (KeyError, ValueError):
        return None, "summary has no traffic line"


# ---- CPU baseline: the oracle on the host cores ------------------------------------------
_CPU_X = None
_CPU_ARGS = None


def _cpu_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _cpu_work(rows):
    from oracle import curvature as oc
    from oracle import knn as ok
    k, variant = _CPU_ARGS
    idx, _, gap, d2n = ok.knn_rows(_CPU_X, rows, k)
    return [(int(i), float(oc.fast_kappa(oc.patch(_CPU_X, idx[r]), variant)), idx[r], float(gap[r]), float(d2n[r]))
            for r, i in enumerate(rows)]


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(X, k, variant, budget_s=20.0):
    """The oracle as it stands (exact float64 kNN row + Fast curvature) on random points of the
    workload, one worker process per core (forked before the GPU is touched), for about
    budget_s seconds.  Returns (baseline entry, {point: (kappa, idx, gap, d2_(k+1))})."""
    import multiprocessing as mp

    import numpy as np
    global _CPU_X, _CPU_ARGS
    _CPU_X = X.astype(np.float64)
    _CPU_ARGS = (k, variant)
    n = X.shape[0]
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(MAX_CPU_WORKERS, avail))
    order = np.random.default_rng(123).permutation(n)
    chunks = (order[s:s + 2] for s in range(0, n, 2))
    res = {}
    t0 = time.perf_counter()
    pool = mp.get_context("fork").Pool(workers, initializer=_cpu_init)
    try:
        for out in pool.imap_unordered(_cpu_work, chunks):
            for i, kap, idx, gap, d2n in out:
                res[i] = (kap, idx, gap, d2n)
            if time.perf_counter() - t0 > budget_s:
                break
        el = time.perf_counter() - t0
    finally:
        pool.terminate()
        pool.join()
    _CPU_X = None
    return {"value": round(len(res) / el, 3), "unit": "points/s", "cores": workers, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": f"{len(res)} random points of the same workload in {el:.1f} s: exact float64 kNN "
                      f"row (difference form over all {n} points) + Fast curvature per point, NumPy/SciPy, "
                      f"{workers} worker processes with one BLAS thread each"}, res


# ---- GPU timing -------------------------------------------------------------------------
def time_path(P, _lib, torch, Xd, k, prec, mode, variant, rerank, steps, warmup):
    """Run `steps` timed passes of the hot path (kNN + curvature) after `warmup` untimed ones.
    Returns (ms per step, library stage timers {name: (ms, launches)}, last outputs, rerank)."""
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
    del ws
    return ms_total / steps, stages, out, rerank


def stage_ms(stages):
    return {s: round(v[0] / v[1], 4) for s, v in stages.items()}


def curvature_ms(stages):
    return sum(v[0] / v[1] for s, v in stages.items() if s in ("curv_fast", "curv_gram", "curv_eigen", "curv_range"))


def roofline(P, stages, n, m, k, prec, workload):
    """Roofline entry of the kernel with the largest average launch time among those with a
    stated algorithmic work: the distance GEMM (n (n+1) m flop under the symmetric tile-pair
    schedule, 2 n^2 m otherwise, at its precision's MFMA peak), the range pass of the two-pass
    Fast form (per point 2 k (k-1) m flop for V_r^T = Ut^T X_c and 2 k m ((k-1) k / 2 + 2) flop
    for the G_tens / trace / row-sum GEMM, each at the peak of the MFMA it runs on; the peak
    reported is the work over its shortest possible time) and the Gram pass (k (k+1) m flop per
    point at the peak of its MFMA: float32, float64 for float64 moments, bf16 for the split bf16
    products of the bf16 path)."""
    kprec, cprec, _ = PRECISIONS[prec]
    cand = {}
    if "knn_gemm_topk" in stages:
        sym = P.knn_symmetric(n)
        f = float(n) * (n + 1) * m if sym else 2.0 * n * n * m
        cand["knn_gemm_topk"] = (f, f / (PEAK[kprec] * 1e12),
                                 f"n*(n+1)*m = {f:.4g} flop per launch (symmetric schedule), {kprec} MFMA"
                                 if sym else f"2*n*n*m = {f:.4g} flop per launch, {kprec} MFMA")
    if "curv_range" in stages:
        p = k - 1
        fv = 2.0 * k * p * m * n
        fg = 2.0 * k * m * (p * k / 2 + 2) * n
        # the G_tens GEMM: float32, float64, or binary16 operands on the bf16 path (the f16
        # MFMA's dense peak equals bf16's)
        gprec = cprec if cprec in ("fp32", "fp64") else "f16"
        gp = PEAK[gprec]
        # the V_r^T product: float32 MFMA, float64 for float64 moments, and bf16 MFMA (high/low
        # parts) on the bf16 path with several waves per point (k > 16)
        vprec = "fp64" if cprec == "fp64" else ("bf16" if cprec == "bf16" and k > 16 else "fp32")
        vp = PEAK[vprec]
        tmin = fv / (vp * 1e12) + fg / (gp * 1e12)
        cand["curv_range"] = (fv + fg, tmin,
                              f"per point 2k(k-1)m = {fv / n:.4g} flop ({vprec} MFMA) "
                              f"+ 2km((k-1)k/2+2) = {fg / n:.4g} flop ({gprec} MFMA), x n = {fv + fg:.4g} per launch")
    if "curv_gram" in stages:
        f = float(k) * (k + 1) * m * n
        gprec = cprec if cprec in ("fp64", "bf16") else "fp32"
        cand["curv_gram"] = (f, f / (PEAK[gprec] * 1e12),
                             f"k(k+1)m per point x n = {f:.4g} flop per launch, {gprec} MFMA")
    if not cand:
        return None
    name = max(cand, key=lambda s: stages[s][0] / stages[s][1])
    flops, tmin, work = cand[name]
    ms = stages[name][0] / stages[name][1]
    achieved = flops / (ms / 1e3) / 1e12
    peak = flops / tmin / 1e12
    traffic, src = profiled_traffic(name, workload, prec)
    return {"bound": "mfma", "achieved": round(achieved, 2), "peak": round(peak, 1), "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": traffic, "kernel": name, "kernel_ms": round(ms, 4),
            "work": work, "traffic_source": src}


def errors_vs_oracle(kap_o, idx_np, kap_np, fl_np, m):
    """Per-point relative error on the oracle's sample over points whose neighbour set equals
    the oracle's and whose patch has full numerical rank; differing neighbour sets are
    classified against the float32 rounding bound of the k-th/(k+1)-th gap."""
    import numpy as np

    from oracle import knn as ok
    errs, diff_big, diff_small, big = [], 0, 0, 0
    for i, (kv, oi, gap, d2n) in kap_o.items():
        gap_ok = gap > float(ok.fp32_gap_bound(m, d2n))
        big += gap_ok
        if set(oi.tolist()) != set(idx_np[i].tolist()):
            if gap_ok:
                diff_big += 1
            else:
                diff_small += 1
            continue
        if not (fl_np[i] & 4):
            errs.append(abs(float(kap_np[i]) - kv) / kv)
    out = {"points": len(errs), "knn_sets_differing_gap_above_bound": diff_big,
           "knn_sets_differing_gap_below_bound": diff_small, "rows_gap_above_bound": int(big)}
    if errs:
        out.update(max_rel=float(np.max(errs)), median_rel=float(np.median(errs)))
    return out


def flag_counts(fl_np):
    return {"rank_deficient": int(((fl_np & 4) != 0).sum()), "knn_uncertified": int(((fl_np & 32) != 0).sum()),
            "knn_ambiguous": int(((fl_np & 16) != 0).sum()), "eigen_fp64": int(((fl_np & 64) != 0).sum()),
            "precision_limit": int(((fl_np & 128) != 0).sum())}


def oracle_sample(X, k, rows, variant):
    """Oracle neighbour lists and Fast kappa of the sampled rows (float64 from the float32 input)."""
    import numpy as np

    from oracle import curvature as oc
    from oracle import knn as ok

    X64 = X.astype(np.float64)
    idx, _, gap, d2n = ok.knn_rows(X64, rows, k)
    return {int(i): (oc.fast_kappa(oc.patch(X64, idx[r]), variant), idx[r], float(gap[r]), float(d2n[r]))
            for r, i in enumerate(rows)}


def suite(args):
    """Secondary configurations, one JSON line each: the other workloads at their own sizes and
    precision paths, errors against the oracle on a sampled set of points."""
    import numpy as np
    import torch

    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib, synth

    # (workload, precisions, exact mode too, n override, k override); the last entry is the
    # cluster cloud at the paper's MNIST_784 shape (n = 70000, k = log2 n = 16), for context
    plan = [("sphere", ("fp32",), True, None, None), ("clusters", ("fp32", "bf16", "fp8"), True, None, None),
            ("torus", ("fp32", "bf16"), False, None, None),
            ("swissroll", ("fp32",), False, None, None), ("blobs", ("fp32", "bf16", "fp8"), False, None, None),
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
            fl_np = fl.cpu().numpy()
            line = {"suite": name, "n": n, "m": m, "k": k, "precision": prec, "mode": "fast",
                    "dtype": PRECISIONS[prec][2], "rerank": rr, "points_per_s": round(n / (ms / 1e3), 1),
                    "ms_per_step": round(ms, 4), "stages_ms": stage_ms(st),
                    "error_vs_oracle": errors_vs_oracle(kap_o, idx.cpu().numpy(), kap.cpu().numpy(), fl_np, m),
                    "flags": flag_counts(fl_np), "oracle_s_per_point_1core": round(t_or, 4)}
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
        if with_exact and P.exact_supported(m, k):
            ms, st, out, rr = time_path(P, _lib, torch, Xd, k, "fp32", "exact", args.variant, None, 3, 1)
            print(json.dumps({"suite": name, "n": n, "m": m, "k": k, "precision": "fp32", "mode": "exact",
                              "points_per_s": round(n / (ms / 1e3), 1), "ms_per_step": round(ms, 4),
                              "stages_ms": stage_ms(st)}), flush=True)
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
    ap.add_argument("--workload", default="blobs")
    ap.add_argument("--precision", default="fp8", choices=list(PRECISIONS))
    ap.add_argument("--variant", default="paper", choices=["paper", "haar"])
    ap.add_argument("--rerank", type=int, default=None,
                    help="candidates per neighbour for the float32 re-rank (default: per precision)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="wall-clock budget of the oracle's CPU baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-modes", action="store_true",
                    help="skip the secondary measurements (other precision paths)")
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

    from paper_2606_06329_amd import synth

    X, k = synth.make(args.workload)
    n, m = X.shape
    # the oracle's worker processes are forked before anything touches the GPU
    cb, kap_o = (None, None)
    if not args.no_cpu_baseline:
        cb, kap_o = cpu_baseline(X, k, args.variant, args.cpu_seconds)

    import torch

    import paper_2606_06329_amd as P
    from paper_2606_06329_amd import _lib

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
    idx, kap, fl = out
    kap_np = kap.cpu().numpy()
    fl_np = fl.cpu().numpy()
    idx_np = idx.cpu().numpy()
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
                   "precision": prec, "knn_gemm": kprec,
                   "range_products": "f16" if cprec == "bf16" and k >= 13 else cprec, "variant": args.variant,
                   "rerank": rerank, "candidates": rerank * k, "mode": "fast"},
        "roofline": roofline(P, stages, n, m, k, prec, args.workload),
        "stages_ms": stage_ms(stages),
        "knn_ms": round(sum(v[0] / v[1] for s, v in stages.items() if s.startswith("knn_")), 4),
        "curvature_ms": round(curvature_ms(stages), 4),
        "flags": flag_counts(fl_np),
    }
    if cb is not None:
        res["cpu_baseline"] = cb
        res["error_vs_oracle"] = errors_vs_oracle(kap_o, idx_np, kap_np, fl_np, m)

    if not args.no_modes:
        # the same workload through the other precision paths, and bf16 vs float32 on the torus
        modes = []
        runs = [(args.workload, Xd, X, mp_, kap_o) for mp_ in ("bf16", "fp32") if mp_ != prec]
        del idx, kap, fl
        for wl, Xm, Xh, mprec, ko in runs:
            mms, mst, mout, mrr = time_path(P, _lib, torch, Xm, k, mprec, "fast", args.variant, args.rerank,
                                            max(2, args.steps // 2), 1)
            midx, mkap, mfl = mout
            entry = {"workload": f"{wl} n={n} m={m} k={k}", "precision": mprec, "mode": "fast",
                     "dtype": PRECISIONS[mprec][2], "rerank": mrr, "points_per_s": round(n / (mms / 1e3), 1),
                     "ms_per_step": round(mms, 4), "stages_ms": stage_ms(mst),
                     "knn_ms": round(sum(v[0] / v[1] for s, v in mst.items() if s.startswith("knn_")), 4),
                     "curvature_ms": round(curvature_ms(mst), 4), "flags": flag_counts(mfl.cpu().numpy()),
                     "roofline": roofline(P, mst, n, m, k, mprec, wl)}
            if ko is not None:
                entry["error_vs_oracle"] = errors_vs_oracle(ko, midx.cpu().numpy(), mkap.cpu().numpy(),
                                                            mfl.cpu().numpy(), m)
            modes.append(entry)
            del midx, mkap, mfl
        del Xd
        torch.cuda.empty_cache()
        # the 100000 x 256 torus (k = 16): bf16 distance GEMM and range products against float32
        Xt, kt = synth.make("torus")
        nt, mt = Xt.shape
        Xtd = torch.from_numpy(Xt).cuda()
        rows = np.random.default_rng(11).choice(nt, 60, replace=False)
        ko_t = oracle_sample(Xt, kt, rows, args.variant)
        for mprec in ("bf16", "fp32"):
            mms, mst, mout, mrr = time_path(P, _lib, torch, Xtd, kt, mprec, "fast", args.variant, None,
                                            max(2, args.steps // 2), 1)
            midx, mkap, mfl = mout
            modes.append({"workload": f"torus n={nt} m={mt} k={kt}", "precision": mprec, "mode": "fast",
                          "dtype": PRECISIONS[mprec][2], "rerank": mrr, "points_per_s": round(nt / (mms / 1e3), 1),
                          "ms_per_step": round(mms, 4), "stages_ms": stage_ms(mst),
                          "flags": flag_counts(mfl.cpu().numpy()),
                          "roofline": roofline(P, mst, nt, mt, kt, mprec, "torus"),
                          "error_vs_oracle": errors_vs_oracle(ko_t, midx.cpu().numpy(), mkap.cpu().numpy(),
                                                              mfl.cpu().numpy(), mt)})
            del midx, mkap, mfl
        res["modes"] = modes
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
