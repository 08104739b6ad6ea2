"""Benchmark of the FastMuyGPs posterior-mean path on one MI355X.

One step = one pass of the whole path over the workload, inputs already in
HBM: build (ingest, kNN screen + FP64 re-rank + certificate, coefficient
precompute with refinement) of n=1,000,000 training points in 40-D (k=50,
RBF, ell=10, mixed precision), then prediction (nearest training point +
gather-dot) of 200,000 queries.  `value` = queries predicted per second of
whole-step time.  Extra fields report the predict-only rate, the plain FP32
path on the same workload, RMSEs, the screen kernel's MFMA roofline, and the
FP64 CPU oracle timed on a bounded sample on this host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 MFMA
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--m", type=int, default=200_000)
    ap.add_argument("--cpu-rows", type=int, default=8192, help="oracle sample: training rows")
    ap.add_argument("--cpu-queries", type=int, default=8192, help="oracle sample: queries")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--serve-seconds", type=float, default=8.0,
                    help="length of each served (Poisson stream) run; 0 skips serving")
    ap.add_argument("--serve-qps", type=float, default=2.0e6, help="offered queries per second")
    ap.add_argument("--no-muygps", action="store_true",
                    help="skip the MuyGPs prediction beside FastMuyGPs")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (scale for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs the FastMuyGPs path on one GPU only; "
              "--gpus %d is not supported (sharding is described in the design notes)"
              % max(args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2205_10879_amd as fmg
    import synth

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 3}))
        return
    log("generating workload n=%d m=%d" % (args.n, args.m))
    w = synth.cfg3(n=args.n, m=args.m)
    X = torch.from_numpy(w.X).to(dev)
    Y = torch.from_numpy(w.Y).to(dev)
    Z = torch.from_numpy(w.Z).to(dev)
    out = torch.empty((args.m, w.Y.shape[1]), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def step(prec="mixed"):
        model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision=prec,
                                     flags=fmg.FLAG_TIMING, stream=stream)
        model.predict(Z, out=out, stream=stream)
        t = model.timings()  # waits for the predict's last event
        info = model.info()
        model.free()
        return t, info

    for i in range(args.warmup):
        t, info = step()
        log("warmup %d: build %.1f ms predict %.1f ms" % (i, t["build_total_ms"],
                                                          t["predict_total_ms"]))
    torch.cuda.synchronize()
    timings = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        t, info = step()
        timings.append(t)
        log("step %d: build %.1f ms (screen %.1f) predict %.1f ms (screen %.1f)" % (
            i, t["build_total_ms"], t["build_screen_ms"], t["predict_total_ms"],
            t["predict_screen_ms"]))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    value = args.m / (ms_per_step / 1000.0)

    def avg(key):
        return sum(t[key] for t in timings) / len(timings)

    mu_mixed = out.cpu().numpy()
    rmse_mixed = float(np.sqrt(np.mean((mu_mixed - w.Yz) ** 2)))
    acc_mixed = float(np.mean(np.argmax(mu_mixed, 1) == w.extra["labels_test"]))

    # Dominant kernel: the build's BF16 MFMA distance screen (n x n pairs, 2d
    # flops per pair).
    screen_ms = avg("build_screen_ms")
    flops = 2.0 * args.n * args.n * w.X.shape[1]
    achieved_tflops = flops / (screen_ms / 1000.0) / 1e12
    roofline = {"bound": "mfma", "kernel": "screen_kernel<OpBF16,2> (build)",
                "achieved": round(achieved_tflops, 2), "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_BF16_TFLOPS, 4),
                "traffic": screen_traffic(args.n), "avg_launch_ms": round(screen_ms, 3),
                "algorithmic_flops_per_launch": flops}

    result = {
        "metric": "predictions/s + p99 latency (n=1M,k=50) vs plain FP32 path at equal RMSE",
        "value": round(value, 1),
        "unit": "predictions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-screen/f64-rerank/f32-solve+f64-residual",
        "data": "synthetic",
        "config": {"workload": "cfg3 10-cluster 40-D Gaussian mixture, one-hot +-0.5 ell=10",
                   "n_train": args.n, "n_test": args.m, "d": int(w.X.shape[1]), "k": w.k,
                   "kernel": "rbf", "length_scale": w.rho, "noise_var": w.noise,
                   "precision": "mixed", "step": "build(all n) + predict(all m)"},
        "build_ms": round(avg("build_total_ms"), 3),
        "predict_ms": round(avg("predict_total_ms"), 3),
        "predict_only_predictions_per_s": round(args.m / (avg("predict_total_ms") / 1000.0), 1),
        "phases_ms": {k: round(avg(k), 3) for k in timings[0]},
        "build_fallback_rows": int(info["build_fallback_rows"]),
        "rmse_mixed": rmse_mixed,
        "accuracy_mixed": acc_mixed,
        "roofline": roofline,
    }

    if not args.no_fp32:
        log("plain FP32 path, one step")
        t32, info32 = step("fp32")
        mu32 = out.cpu().numpy()
        rmse32 = float(np.sqrt(np.mean((mu32 - w.Yz) ** 2)))
        result["fp32_plain"] = {
            "build_ms": round(t32["build_total_ms"], 3),
            "predict_ms": round(t32["predict_total_ms"], 3),
            "whole_step_predictions_per_s": round(
                args.m / ((t32["build_total_ms"] + t32["predict_total_ms"]) / 1000.0), 1),
            "predict_only_predictions_per_s": round(
                args.m / (t32["predict_total_ms"] / 1000.0), 1),
            "rmse": rmse32,
            "rmse_ratio_mixed_over_fp32": rmse_mixed / rmse32,
            "max_abs_mean_diff_vs_mixed": float(np.max(np.abs(mu32 - mu_mixed))),
        }

    # The paper's own comparison (Section 4): MuyGPs prediction (each query
    # solving over its own neighbourhood, Section 2.1) against FastMuyGPs
    # prediction on the same model and queries.
    if not args.no_muygps:
        muygps_run(fmg, np, torch, w, X, Y, Z, out, stream, args, result)

    if args.serve_seconds > 0:
        result["served"] = {}
        for prec in ("mixed", "fp32"):
            log("served run (%s): Poisson stream, %.0f queries/s offered, %.1f s" % (
                prec, args.serve_qps, args.serve_seconds))
            model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise,
                                         precision=prec, stream=stream)
            result["served"][prec] = serve_run(fmg, synth, np, model, args.serve_qps,
                                               args.serve_seconds)
            model.free()
            log("served %s: %s" % (prec, result["served"][prec]))
        result["p99_ms_served_mixed"] = result["served"]["mixed"]["p99_ms"]
        result["p99_ms_served_fp32"] = result["served"]["fp32"]["p99_ms"]

    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        rs = synth.rng(3, 4)
        rows = np.sort(rs.choice(args.n, args.cpu_rows, replace=False))
        qs = np.sort(rs.choice(args.m, args.cpu_queries, replace=False))
        X64 = w.X.astype(np.float64)
        Y64 = w.Y.astype(np.float64)
        log("cpu baseline: oracle on %d rows + %d queries, %d threads" % (
            len(rows), len(qs), threads))
        c0 = time.perf_counter()
        oracle.build_model(X64, Y64, w.k, w.kernel, w.nu, w.rho, w.noise, rows=rows,
                           nthreads=threads)
        c1 = time.perf_counter()
        mu_o, _, _ = oracle.predict(X64, Y64, w.Z[qs].astype(np.float64), w.k, w.kernel, w.nu,
                                    w.rho, w.noise, nthreads=threads)
        c2 = time.perf_counter()
        per_row = (c1 - c0) / len(rows)
        per_query = (c2 - c1) / len(qs)
        # whole job at the same shape: build all n rows, predict all m queries
        est = per_row * args.n + per_query * args.m
        result["cpu_baseline"] = {
            "value": round(args.m / est, 3), "unit": "predictions/s", "cores": threads,
            "kind": "oracle",
            "sample": "FP64 oracle on %d seeded training rows and %d seeded queries of the "
                      "same workload (%.1f s); per-item times extrapolated to build(n=%d) + "
                      "predict(m=%d) = %.0f s" % (len(rows), len(qs), c2 - c0, args.n, args.m,
                                                   est)}
        err = float(np.max(np.abs(mu_mixed[qs] - mu_o)) / max(
            float(np.sqrt(np.mean(mu_o ** 2))), 1e-300))
        result["oracle_sample_max_rel_err_mixed"] = err

    print(json.dumps(result), flush=True)


def muygps_run(fmg, np, torch, w, X, Y, Z, out, stream, args, result):
    log("MuyGPs prediction of the same queries")
    model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision="mixed",
                                 stream=stream)
    mu_fast = model.predict(Z, stream=stream)
    mg_out = torch.empty_like(out)
    model.predict_muygps(Z, out=mg_out, stream=stream)  # warm-up
    torch.cuda.synchronize()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    e0.record(stream)
    model.predict(Z, out=out, stream=stream)
    e1.record(stream)
    model.predict_muygps(Z, out=mg_out, stream=stream)
    e2.record(stream)
    torch.cuda.synchronize()
    model.free()
    mu_mg = mg_out.cpu().numpy()
    rmse_mg = float(np.sqrt(np.mean((mu_mg - w.Yz) ** 2)))
    result["muygps_predict"] = {
        "predict_ms": round(e1.elapsed_time(e2), 3),
        "predictions_per_s": round(args.m / (e1.elapsed_time(e2) / 1000.0), 1),
        "fastmuygps_predict_ms": round(e0.elapsed_time(e1), 3),
        "fastmuygps_speedup": round(e1.elapsed_time(e2) / e0.elapsed_time(e1), 3),
        "rmse": rmse_mg, "rmse_fastmuygps": float(np.sqrt(np.mean(
            (mu_fast.cpu().numpy() - w.Yz) ** 2))),
        "accuracy": float(np.mean(np.argmax(mu_mg, 1) == w.extra["labels_test"]))}
    log("MuyGPs predict: %s" % result["muygps_predict"])


def screen_traffic(n):
    """HBM bytes per launch of the build screen, from the committed counter
    record (FETCH_SIZE + WRITE_SIZE, scaled by a plain copy's reading); None
    when the record is missing, for another n, or taken on other kernel
    source than the one built now."""
    import hashlib
    rec = os.path.join(ROOT, "profiles", "screen_build_traffic.txt")
    src = os.path.join(ROOT, "paper_2205_10879_amd", "csrc", "fmg_screen.hip")
    try:
        fields = {}
        for line in open(rec):
            if ":" in line and not line.startswith("#"):
                key, val = line.split(":", 1)
                fields[key.strip()] = val.strip()
        digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
        if fields.get("source_sha256") != digest or int(fields.get("n", -1)) != n:
            return None
        return float(fields["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def serve_run(fmg, synth, np, model, qps, seconds, bmax=4096):
    """Open-loop served run: requests arrive as a Poisson stream with batch
    sizes log-uniform in [1, bmax] (mean offered load `qps` queries/s); latency
    runs from each request's scheduled arrival to its results in host memory."""
    import queue
    import threading
    mean_b = (bmax + 1) / math.log(bmax + 1) - 1.0  # E[floor(exp(U ln(bmax+1)))] ~
    rate = qps / mean_b
    t_arr, B = synth.poisson_stream(rate, seconds, bmax)
    pool = synth.cfg3_queries(1 << 20)
    offs = np.concatenate([[0], np.cumsum(B)[:-1]]) % (len(pool) - bmax)
    srv = fmg.Server(slots=3, max_batch=16384)
    mid, _ = srv.add_model(model)
    # warm-up: one request per batch-size bucket the stream can form
    for b in (1, 300, 600, 1000, 2000, 4000, 8000, 16000):
        for _ in range(3):
            srv.submit(mid, pool[:b]).wait()
    srv.reset_stats()
    tickets = queue.Queue()
    lat = []

    def waiter():
        while True:
            t = tickets.get()
            if t is None:
                return
            lat.append(t.wait()[1])

    th = threading.Thread(target=waiter)
    th.start()
    t0 = time.monotonic_ns() + 20_000_000
    for i in range(len(t_arr)):
        due = t0 + int(t_arr[i] * 1e9)
        while True:
            now = time.monotonic_ns()
            if now >= due:
                break
            if due - now > 200_000:
                time.sleep((due - now - 100_000) * 1e-9)
        o = int(offs[i])
        tickets.put(srv.submit(mid, pool[o:o + int(B[i])], arrival_ns=due))
    tickets.put(None)
    th.join()
    st = srv.stats()
    srv.close()
    return {"requests": int(st["requests"]), "queries": int(st["queries"]),
            "batches": int(st["batches"]), "offered_qps": qps,
            "predictions_per_s": round(st["queries_per_s"], 1),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
            "hbm_peak_bytes": int(st["hbm_peak"])}


if __name__ == "__main__":
    main()
