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
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="length of the served (Poisson stream) run of the mixed-precision "
                         "model; 0 skips serving")
    ap.add_argument("--serve-seconds-fp32", type=float, default=8.0,
                    help="length of the plain FP32 served run (it falls behind the offered "
                         "load, so its backlog grows with the length)")
    ap.add_argument("--cfg5-seconds", type=float, default=10.0,
                    help="length of each multi-model served run (9 models); 0 skips it")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the cfg-1 and cfg-2 build and predict lines")
    ap.add_argument("--serve-qps", type=float, default=2.0e6, help="offered queries per second")
    ap.add_argument("--serve-qps-equal", type=float, default=5.0e5,
                    help="offered load of the equal-load served runs (both precisions at a "
                         "rate the plain FP32 path sustains)")
    ap.add_argument("--serve-seconds-equal", type=float, default=8.0,
                    help="length of each equal-load served run; 0 skips them")
    ap.add_argument("--no-muygps", action="store_true",
                    help="skip the MuyGPs prediction beside FastMuyGPs")
    ap.add_argument("--no-borehole", action="store_true",
                    help="skip the borehole emulator and its MCMC calibration")
    ap.add_argument("--no-training", action="store_true",
                    help="skip the leave-one-out loss and gradient timings")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy 3 times (scale for HBM counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: the FastMuyGPs path runs on one GPU only; "
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
    # One more (untimed) build + predict whose neighbour lists and nearest
    # points the oracle leg checks.
    model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision="mixed",
                                 stream=stream)
    nn_d = torch.empty(args.m, dtype=torch.int32, device=dev)
    model.predict(Z, out=out, nn_out=nn_d, stream=stream)
    N_mixed = model.neighbors(stream=stream).cpu().numpy()
    nn_mixed = nn_d.cpu().numpy()
    assert np.array_equal(out.cpu().numpy(), mu_mixed), "repeated prediction differs"
    model.free()
    rmse_mixed = float(np.sqrt(np.mean((mu_mixed - w.Yz) ** 2)))
    acc_mixed = float(np.mean(np.argmax(mu_mixed, 1) == w.extra["labels_test"]))

    # Dominant kernel: the build's BF16 MFMA distance screen (n x n pairs, 2d
    # flops per pair: the brute-force work the screen answers for, whether it
    # computes a pair or proves it unnecessary by tile pruning).
    screen_ms = avg("build_screen_ms")
    flops = 2.0 * args.n * args.n * w.X.shape[1]
    achieved_tflops = flops / (screen_ms / 1000.0) / 1e12
    roofline = {"bound": "mfma", "kernel": "screen_kernel<OpBF16,2,256,true> (build, pruned)",
                "achieved": round(achieved_tflops, 2), "peak": PEAK_BF16_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_BF16_TFLOPS, 4),
                "traffic": screen_traffic(args.n), "avg_launch_ms": round(screen_ms, 3),
                "algorithmic_flops_per_launch": flops}

    # The prediction gather-dot (HBM-bound): per query it must read the query
    # row, j, N(j), the k neighbour rows, C[j] and write ell means.
    d_, k_, ell_ = int(w.X.shape[1]), w.k, int(w.Y.shape[1])
    gbytes = args.m * (4 * d_ + 4 + 4 * k_ + 4 * k_ * d_ + 4 * k_ * ell_ + 4 * ell_)
    gather_ms = avg("predict_gather_ms")
    gather_gbs = gbytes / (gather_ms / 1000.0) / 1e9
    gather_roofline = {"bound": "hbm", "kernel": "gather_vec_kernel<float,10,10>",
                       "achieved": round(gather_gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                       "frac": round(gather_gbs / PEAK_HBM_GBS, 4),
                       "avg_launch_ms": round(gather_ms, 4),
                       "algorithmic_bytes_per_launch": gbytes}

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
        "builds_per_s": round(1000.0 / avg("build_total_ms"), 3),
        "training_points_per_s": round(args.n / (avg("build_total_ms") / 1000.0), 1),
        "predict_ms": round(avg("predict_total_ms"), 3),
        "predict_only_predictions_per_s": round(args.m / (avg("predict_total_ms") / 1000.0), 1),
        "phases_ms": {k: round(avg(k), 3) for k in timings[0]},
        "build_fallback_rows": int(info["build_fallback_rows"]),
        "rmse_mixed": rmse_mixed,
        "accuracy_mixed": acc_mixed,
        "roofline": roofline,
        "gather_roofline": gather_roofline,
    }

    if not args.no_fp32:
        log("plain FP32 path, one step")
        t32, info32 = step("fp32")
        mu32 = out.cpu().numpy()
        log("plain FP32: build %.1f ms predict %.1f ms" % (t32["build_total_ms"],
                                                         t32["predict_total_ms"]))
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

    # MuyGPs hyperparameter training on the same model (Algorithm 1): the loss
    # Q(theta) in the model's precision and its FP64 gradient, on a batch.
    if not args.no_training:
        training_run(fmg, np, torch, w, X, Y, stream, result)

    # The borehole emulator (Section 4.2): k = 150 in FP64, its single-query
    # latency and an MCMC calibration driven by its predictions.
    bh_sample = None
    if not args.no_borehole:
        bh_sample = borehole_run(fmg, np, torch, synth, stream, result)

    # Build and predict lines of the cfg-1 (FP64) and cfg-2 (FP32) workloads.
    cfg_sample = None
    if not args.no_configs:
        cfg_sample = configs_run(fmg, np, torch, synth, result)

    if args.serve_seconds > 0:
        result["served"] = {}
        for prec, secs in (("mixed", args.serve_seconds), ("fp32", args.serve_seconds_fp32)):
            if secs <= 0:
                continue
            log("served run (%s): Poisson stream, %.0f queries/s offered, %.1f s" % (
                prec, args.serve_qps, secs))
            model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise,
                                         precision=prec, stream=stream)
            result["served"][prec] = serve_run(fmg, synth, np, torch, model, args.serve_qps,
                                               secs)
            model.free()
            log("served %s: %s" % (prec, result["served"][prec]))
        for prec in result["served"]:
            result["p99_ms_served_" + prec] = result["served"][prec]["p99_ms"]

    # The same comparison at an offered load that both paths sustain, so that
    # the p99 latencies compare service times rather than a growing backlog.
    if args.serve_seconds_equal > 0:
        eq = {"offered_qps": args.serve_qps_equal}
        for prec in ("mixed", "fp32"):
            log("equal-load served run (%s): %.0f queries/s offered, %.1f s" % (
                prec, args.serve_qps_equal, args.serve_seconds_equal))
            model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise,
                                         precision=prec, stream=stream)
            eq[prec] = serve_run(fmg, synth, np, torch, model, args.serve_qps_equal,
                                 args.serve_seconds_equal)
            model.free()
            log("equal-load served %s: %s" % (prec, eq[prec]))
        result["served_equal_load"] = eq
        for prec in ("mixed", "fp32"):
            result["p99_ms_equal_load_" + prec] = eq[prec]["p99_ms"]

    # Several resident models admitted by HBM budget (multi-model serving).
    cfg5_sample = None
    if args.cfg5_seconds > 0:
        result["served_cfg5"], cfg5_sample = cfg5_run(fmg, np, torch, synth, args.cfg5_seconds,
                                                      args.serve_qps)

    if not args.no_cpu_baseline:
        cpu_baseline_run(np, synth, w, args, result, N_mixed, nn_mixed, mu_mixed,
                         mu32 if not args.no_fp32 else None)
        oracle_samples(np, result, bh_sample, cfg_sample, cfg5_sample)

    print(json.dumps(result), flush=True)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_run(np, synth, w, args, result, N_gpu, nn_gpu, mu_gpu, mu32):
    """The FP64 oracle on a seeded sample of the same workload, on this host's
    cores: its rate (all threads, and one thread on a smaller sample) and the
    GPU results checked against it (neighbour lists and nearest points bit
    for bit, means by the relative error max |dmu| / max(|mu_o|, RMS(mu_o)))."""
    import oracle
    threads = oracle.max_threads()
    rs = synth.rng(3, 4)
    rows = np.sort(rs.choice(args.n, args.cpu_rows, replace=False))
    qs = np.sort(rs.choice(args.m, args.cpu_queries, replace=False))
    X64 = w.X.astype(np.float64)
    Y64 = w.Y.astype(np.float64)
    Zs = w.Z[qs].astype(np.float64)
    log("cpu baseline: oracle on %d rows + %d queries, %d threads" % (
        len(rows), len(qs), threads))
    c0 = time.perf_counter()
    N_o, _, _ = oracle.build_model(X64, Y64, w.k, w.kernel, w.nu, w.rho, w.noise, rows=rows,
                                   nthreads=threads)
    c1 = time.perf_counter()
    mu_o, nn_o, _ = oracle.predict(X64, Y64, Zs, w.k, w.kernel, w.nu, w.rho, w.noise,
                                   nthreads=threads)
    c2 = time.perf_counter()
    per_row = (c1 - c0) / len(rows)
    per_query = (c2 - c1) / len(qs)
    # whole job at the same shape: build all n rows, predict all m queries
    est = per_row * args.n + per_query * args.m
    # one thread, on a smaller sample
    r1, q1 = rows[:128], Zs[:128]
    d0 = time.perf_counter()
    oracle.build_model(X64, Y64, w.k, w.kernel, w.nu, w.rho, w.noise, rows=r1, nthreads=1)
    d1 = time.perf_counter()
    oracle.predict(X64, Y64, q1, w.k, w.kernel, w.nu, w.rho, w.noise, nthreads=1)
    d2 = time.perf_counter()
    est1 = (d1 - d0) / len(r1) * args.n + (d2 - d1) / len(q1) * args.m
    result["cpu_baseline"] = {
        "value": round(args.m / est, 3), "unit": "predictions/s", "cores": threads,
        "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
        "value_1_thread": round(args.m / est1, 3),
        "sample": "FP64 oracle on %d seeded training rows and %d seeded queries of the "
                  "same workload (%.1f s, %d threads); per-item times extrapolated to "
                  "build(n=%d) + predict(m=%d) = %.0f s; 1-thread rate from 128 rows + 128 "
                  "queries (%.1f s)" % (len(rows), len(qs), c2 - c0, threads, args.n, args.m,
                                         est, d2 - d0)}

    def rel_err(got, ref):
        rms = max(float(np.sqrt(np.mean(ref * ref))), 1e-300)
        return float(np.max(np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), rms)))

    def rmse_ratio(got):
        return float(np.sqrt(np.mean((got - w.Yz[qs]) ** 2)) /
                     np.sqrt(np.mean((mu_o - w.Yz[qs]) ** 2)))

    chk = {"rows": int(len(rows)), "queries": int(len(qs)),
           "neighbor_list_mismatches": int(np.count_nonzero(np.any(N_gpu[rows] != N_o, axis=1))),
           "nearest_mismatches": int(np.count_nonzero(nn_gpu[qs] != nn_o)),
           "mean_rel_err_mixed": rel_err(mu_gpu[qs], mu_o),
           "rmse_ratio_mixed": rmse_ratio(mu_gpu[qs])}
    if mu32 is not None:
        chk["mean_rel_err_fp32"] = rel_err(mu32[qs], mu_o)
        chk["rmse_ratio_fp32"] = rmse_ratio(mu32[qs])
    result["oracle_check"] = chk
    log("oracle check: %s" % chk)


def oracle_samples(np, result, bh_sample, cfg_sample, cfg5_sample):
    """The FP64 oracle on seeded samples of the other workloads' outputs:
    neighbour lists and nearest points bit for bit, means by the relative
    error max |dmu| / max(|mu_o|, RMS(mu_o))."""
    import oracle
    threads = oracle.max_threads()

    def rel_err(got, ref):
        rms = max(float(np.sqrt(np.mean(ref * ref))), 1e-300)
        return float(np.max(np.abs(got.astype(np.float64) - ref) / np.maximum(np.abs(ref), rms)))

    def check(w, qs_means, nn_gpu, Zq, rows=None, N_gpu=None):
        X64, Y64 = w.X.astype(np.float64), w.Y.astype(np.float64)
        out = {"queries": int(len(Zq))}
        if rows is not None:
            N_o, _, _ = oracle.build_model(X64, Y64, w.k, w.kernel, w.nu, w.rho, w.noise,
                                           rows=rows, nthreads=threads)
            out["rows"] = int(len(rows))
            out["neighbor_list_mismatches"] = int(np.count_nonzero(np.any(N_gpu != N_o, axis=1)))
        mu_o, nn_o, _ = oracle.predict(X64, Y64, Zq.astype(np.float64), w.k, w.kernel, w.nu,
                                       w.rho, w.noise, nthreads=threads)
        out["nearest_mismatches"] = int(np.count_nonzero(nn_gpu != nn_o))
        out["mean_rel_err"] = rel_err(qs_means, mu_o)
        return out

    c0 = time.perf_counter()
    if bh_sample is not None:
        w, qs, mu, nn = bh_sample
        result["borehole"]["oracle_check"] = check(w, mu, nn, w.Z[qs])
        log("borehole oracle check: %s" % result["borehole"]["oracle_check"])
    if cfg_sample is not None:
        for w, rows, N_g, qs, mu, nn in cfg_sample:
            result["configs"][w.name]["oracle_check"] = check(w, mu, nn, w.Z[qs], rows, N_g)
            log("%s oracle check: %s" % (w.name, result["configs"][w.name]["oracle_check"]))
    if cfg5_sample is not None:
        for j, (w, qs, mu, nn) in enumerate(cfg5_sample):
            result["served_cfg5"]["models"][j]["oracle_check"] = check(w, mu, nn, w.Z[qs])
        log("cfg5 oracle checks: %s" % [m["oracle_check"] for m in
                                        result["served_cfg5"]["models"]])
    result["oracle_samples_seconds"] = round(time.perf_counter() - c0, 1)


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


def training_run(fmg, np, torch, w, X, Y, stream, result, b=65536):
    log("leave-one-out loss and gradient on %d rows" % b)
    model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision="mixed",
                                 stream=stream)
    rows = torch.from_numpy(np.sort(np.random.default_rng(9).choice(
        X.shape[0], b, replace=False)).astype(np.int32)).cuda()
    model.loo_loss(rows, w.kernel, w.nu, w.rho, w.noise, stream=stream)  # warm-up
    model.loo_loss_grad(rows, w.kernel, w.nu, w.rho, w.noise, stream=stream)
    t0 = time.perf_counter()
    q = model.loo_loss(rows, w.kernel, w.nu, w.rho, w.noise, stream=stream)
    t1 = time.perf_counter()
    qg, g = model.loo_loss_grad(rows, w.kernel, w.nu, w.rho, w.noise, stream=stream)
    t2 = time.perf_counter()
    model.free()
    result["training"] = {
        "batch_rows": b, "loo_loss_ms": round((t1 - t0) * 1e3, 3),
        "loo_loss_grad_fp64_ms": round((t2 - t1) * 1e3, 3), "loss_mixed": q, "loss_fp64": qg,
        "grad_length_scale": float(g[0]), "grad_noise_var": float(g[1])}
    log("training: %s" % result["training"])


def borehole_run(fmg, np, torch, synth, stream, result, chains=4096, steps=300, burn=100,
                 latency_reps=300):
    w = synth.borehole()
    log("borehole emulator: n=%d m=%d k=%d, RBF rho=%g, FP64" % (
        w.X.shape[0], w.Z.shape[0], w.k, w.rho))
    X = torch.from_numpy(w.X).cuda()
    Y = torch.from_numpy(w.Y).cuda()
    Z = torch.from_numpy(w.Z).cuda()
    for rep in range(2):  # the first build warms up the kernels
        model = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise, precision="fp64",
                                     flags=fmg.FLAG_TIMING, stream=stream)
        mu = model.predict(Z, stream=stream)
        t = model.timings()
        if rep == 0:
            model.free()
    rm = float(np.sqrt(np.mean((mu.cpu().numpy() - w.Yz) ** 2)))
    # single-query predictions, one after another (the MCMC use of an emulator)
    one = torch.empty((1, 1), dtype=torch.float64, device="cuda")
    lat = []
    for r in range(latency_reps):
        z = Z[r:r + 1]
        c0 = time.perf_counter()
        model.predict(z, out=one, stream=stream)
        stream.synchronize()
        lat.append((time.perf_counter() - c0) * 1e3)
    lat = np.sort(np.array(lat[10:]))
    mc = borehole_mcmc(fmg, np, torch, synth, w, model, chains, steps, burn)
    qs = np.sort(synth.rng(6, 4).choice(w.Z.shape[0], 64, replace=False))
    nn = torch.empty(len(qs), dtype=torch.int32, device="cuda")
    mu_s = model.predict(Z[torch.from_numpy(qs).cuda()], nn_out=nn, stream=stream)
    sample = (w, qs, mu_s.cpu().numpy(), nn.cpu().numpy())
    model.free()
    result["borehole"] = {
        "workload": w.name, "n": int(w.X.shape[0]), "m": int(w.Z.shape[0]), "k": w.k,
        "noise_var": w.noise, "build_ms": round(t["build_total_ms"], 3),
        "build_search_ms": round(t["build_prep_ms"] + t["build_screen_ms"], 3),
        "build_precompute_ms": round(t["build_precompute_ms"], 3),
        "predict_ms": round(t["predict_total_ms"], 3),
        "predictions_per_s": round(w.Z.shape[0] / (t["predict_total_ms"] / 1e3), 1),
        "rmse": rm, "single_query_p50_ms": round(float(np.percentile(lat, 50)), 4),
        "single_query_p99_ms": round(float(np.percentile(lat, 99)), 4), "mcmc": mc}
    log("borehole: %s" % result["borehole"])
    return sample


def borehole_mcmc(fmg, np, torch, synth, w, model, chains, steps, burn, step_sd=0.01,
                  like_sd=1.0):
    """Metropolis calibration of the borehole radius r_w with the emulator
    (Section 4.2): the observed flow is the borehole function at r_w = 0.09
    (unit coordinate 0.4) with the other parameters at mid-range, the
    likelihood Gaussian with standard deviation 1 on the flow, the prior
    uniform on the r_w range, random-walk proposals in the unit coordinate.
    `chains` independent chains advance together, each step one batched
    prediction of all their proposals."""
    truth = np.full(8, synth.BOREHOLE_FIXED_U)
    truth[0] = 0.4
    y_obs = float(synth.borehole_flow(synth.BOREHOLE_LO + truth * (
        synth.BOREHOLE_HI - synth.BOREHOLE_LO))) - w.extra["response_mean"]
    base = torch.from_numpy(synth.borehole_inputs(truth)).cuda()
    g = torch.Generator(device="cuda")
    g.manual_seed(42)
    u = torch.rand(chains, generator=g, dtype=torch.float64, device="cuda")
    Zc = base.repeat(chains, 1)
    Zc[:, 0] = u / synth.BOREHOLE_SCALE[0]
    mu = model.predict(Zc)[:, 0]
    acc = torch.zeros((), dtype=torch.float64, device="cuda")
    tot = torch.zeros((), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    c0 = time.perf_counter()
    for s in range(burn + steps):
        up = u + step_sd * torch.randn(chains, generator=g, dtype=torch.float64, device="cuda")
        inside = (up >= 0.0) & (up <= 1.0)
        Zc[:, 0] = up.clamp(0.0, 1.0) / synth.BOREHOLE_SCALE[0]
        mup = model.predict(Zc)[:, 0]
        logr = ((mu - y_obs) ** 2 - (mup - y_obs) ** 2) / (2.0 * like_sd * like_sd)
        lu = torch.log(torch.rand(chains, generator=g, dtype=torch.float64, device="cuda"))
        take = inside & (lu < logr)
        u = torch.where(take, up, u)
        mu = torch.where(take, mup, mu)
        if s >= burn:
            acc += take.sum()
            tot += u.sum()
    torch.cuda.synchronize()
    el = time.perf_counter() - c0
    n_s = chains * steps
    return {"chains": chains, "steps": steps, "burn_in": burn, "samples": n_s,
            "posterior_mean_rw_unit": float(tot) / n_s, "truth_rw_unit": 0.4,
            "acceptance": float(acc) / n_s, "seconds": round(el, 3),
            "samples_per_s": round(chains * (burn + steps) / el, 1)}


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


def mean_batch(bmax):
    """E[floor(exp(U ln(bmax + 1)))], the mean of the log-uniform batch sizes."""
    return (bmax + 1) / math.log(bmax + 1) - 1.0


def drive(srv, ids, pools, events, keep=6):
    """Submit `events` [(time_s, model index, B)] open loop, each at its
    scheduled time (latency runs from that time, so a server that falls
    behind is charged for it); a waiter thread collects every request's
    latency per model and keeps the first `keep` results of each model (with
    their pool offsets) for a check against direct prediction."""
    import queue
    import threading
    tickets = queue.Queue()
    lat = [[] for _ in ids]
    kept = [[] for _ in ids]

    def waiter():
        while True:
            item = tickets.get()
            if item is None:
                return
            j, o, b, t = item
            out, ms = t.wait()
            lat[j].append(ms)
            if len(kept[j]) < keep:
                kept[j].append((o, b, out.copy()))

    th = threading.Thread(target=waiter)
    th.start()
    offs = [0] * len(ids)
    t0 = time.monotonic_ns() + 20_000_000
    for ta, j, b in events:
        due = t0 + int(ta * 1e9)
        while True:
            now = time.monotonic_ns()
            if now >= due:
                break
            if due - now > 200_000:
                time.sleep((due - now - 100_000) * 1e-9)
        pool = pools[j]
        o = offs[j] % (len(pool) - b + 1)
        offs[j] += b
        tickets.put((j, o, b, srv.submit(ids[j], pool[o:o + b], arrival_ns=due)))
    tickets.put(None)
    th.join()
    return lat, kept


def served_equals_direct(torch, models, pools, kept):
    """Kept served results against fastmuygps_predict of the same queries:
    the number of requests compared and of those bit-identical."""
    n = same = 0
    for j, lst in enumerate(kept):
        for o, b, out in lst:
            ref = models[j].predict(torch.from_numpy(pools[j][o:o + b]).cuda()).cpu().numpy()
            n += 1
            same += int(ref.shape == out.shape and (ref == out).all())
    return n, same


def pct(v, p):
    """Nearest-rank percentile."""
    v = sorted(v)
    if not v:
        return None
    r = max(1, int(math.ceil(p / 100.0 * len(v))))
    return v[r - 1]


def serve_run(fmg, synth, np, torch, model, qps, seconds, bmax=4096):
    """One resident model (the cfg-3 model) under an open-loop Poisson stream
    of requests with batch sizes log-uniform in [1, bmax] (mean offered load
    `qps` queries/s); latency runs from each request's scheduled arrival to
    its results in host memory."""
    t_arr, B = synth.poisson_stream(qps / mean_batch(bmax), seconds, bmax)
    pool = synth.cfg3_queries(1 << 20)
    srv = fmg.Server(slots=3, max_batch=16384)
    mid, _ = srv.add_model(model)
    # warm-up: one request per batch-size bucket the stream can form
    for b in (1, 300, 600, 1000, 2000, 4000, 8000, 16000):
        for _ in range(3):
            srv.submit(mid, pool[:b]).wait()
    srv.reset_stats()
    events = [(float(t), 0, int(b)) for t, b in zip(t_arr, B)]
    _, kept = drive(srv, [mid], [pool], events)
    st = srv.stats()
    srv.close()
    n, same = served_equals_direct(torch, [model], [pool], kept)
    return {"seconds": seconds, "requests": int(st["requests"]), "queries": int(st["queries"]),
            "batches": int(st["batches"]), "offered_qps": qps,
            "predictions_per_s": round(st["queries_per_s"], 1),
            "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
            "mean_ms": round(st["mean_ms"], 3), "max_ms": round(st["max_ms"], 3),
            "hbm_peak_bytes": int(st["hbm_peak"]),
            "served_checked_against_direct": n, "served_bit_identical": same}


def cfg5_run(fmg, np, torch, synth, seconds, qps, bmax=8192):
    """Several resident models admitted by HBM budget: model A (n = 5M, d = 3,
    Matern 1/2, FP32) and eight models of the cfg-1/2/3 kinds (synth.cfg5_models),
    each with its own Poisson stream (batch sizes log-uniform in [1, 8192],
    the total offered load split equally), interleaved.  Two runs: (i) the
    whole device, (ii) a budget of the slot workspaces plus 60 % of the sum of
    the model footprints, where the server swaps idle models out to host
    memory for models with waiting requests.  Returns the block and, for the
    oracle leg, a seeded sample of every model's direct predictions."""
    ws = synth.cfg5_models()
    models, build_ms = [], []
    for w in ws:
        dt = torch.float64 if w.precision == "fp64" else torch.float32
        X = torch.from_numpy(w.X).to("cuda", dt)
        Y = torch.from_numpy(w.Y).to("cuda", dt)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        models.append(fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise,
                                           precision=w.precision))
        torch.cuda.synchronize()
        build_ms.append((time.perf_counter() - c0) * 1e3)
        del X, Y
        log("cfg5 model %s built in %.1f ms" % (w.name, build_ms[-1]))
    fps = [int(m.info()["device_bytes"]) for m in models]
    pools = [np.ascontiguousarray(w.Z) for w in ws]
    rate = qps / len(ws) / mean_batch(bmax)
    events = []
    for j in range(len(ws)):
        t_arr, B = synth.poisson_stream(rate, seconds, bmax, cfg=60 + j)
        events += [(float(t), j, int(b)) for t, b in zip(t_arr, B)]
    events.sort()
    with fmg.Server(slots=3, max_batch=bmax) as probe:
        wsb = int(probe.stats()["hbm_resident"])
    block = {"offered_qps": qps, "seconds": seconds, "batch_max": bmax,
             "slot_workspace_bytes": wsb, "sum_footprints_bytes": sum(fps),
             "models": [{"name": w.name, "n": int(w.X.shape[0]), "d": int(w.X.shape[1]),
                         "k": w.k, "ell": int(w.Y.shape[1]), "precision": w.precision,
                         "kernel": w.kernel, "nu": w.nu, "build_ms": round(b, 2),
                         "footprint_bytes": f,
                         "rmse": float(np.sqrt(np.mean((models[j].predict(
                             torch.from_numpy(pools[j]).cuda()).cpu().numpy() - w.Yz) ** 2)))}
                        for j, (w, b, f) in enumerate(zip(ws, build_ms, fps))],
             "builds_per_s": round(len(ws) / (sum(build_ms) / 1e3), 3)}
    for label, budget, swap in (("whole_device", 0, False),
                                ("budget_60pct", wsb + int(0.6 * sum(fps)), True)):
        log("cfg5 served run (%s): 9 models, %.0f queries/s offered, %.1f s" % (
            label, qps, seconds))
        srv = fmg.Server(hbm_budget=budget, slots=3, max_batch=bmax, swap_idle=swap)
        ids = [srv.add_model(m)[0] for m in models]
        for j in range(len(ws)):
            for b in (1, 300, 1000, 4000, bmax):
                srv.submit(ids[j], pools[j][:b]).wait()
        srv.reset_stats()
        lat, kept = drive(srv, ids, pools, events)
        st = srv.stats()
        srv.close()
        n, same = served_equals_direct(torch, models, pools, kept)
        run = {"hbm_budget_bytes": budget if budget else None, "swap_idle": swap,
               "requests": int(st["requests"]), "queries": int(st["queries"]),
               "batches": int(st["batches"]),
               "predictions_per_s": round(st["queries_per_s"], 1),
               "p50_ms": round(st["p50_ms"], 3), "p99_ms": round(st["p99_ms"], 3),
               "hbm_peak_bytes": int(st["hbm_peak"]), "swaps": int(st["swaps"]),
               "per_model": [{"name": w.name, "requests": len(lat[j]),
                              "p50_ms": round(pct(lat[j], 50), 3) if lat[j] else None,
                              "p99_ms": round(pct(lat[j], 99), 3) if lat[j] else None}
                             for j, w in enumerate(ws)],
               "served_checked_against_direct": n, "served_bit_identical": same}
        block[label] = run
        log("cfg5 %s: %s" % (label, {k: v for k, v in run.items() if k != "per_model"}))
    # seeded sample of each model's direct predictions for the oracle leg
    sample = []
    rs = synth.rng(5, 4)
    for j, w in enumerate(ws):
        q = np.sort(rs.choice(len(pools[j]), 24, replace=False))
        nn = torch.empty(len(q), dtype=torch.int32, device="cuda")
        mu = models[j].predict(torch.from_numpy(pools[j][q]).cuda(), nn_out=nn)
        sample.append((w, q, mu.cpu().numpy(), nn.cpu().numpy()))
        models[j].free()
    return block, sample


def configs_run(fmg, np, torch, synth, result):
    """Build and predict rates of the full-size cfg-1 (FP64) and cfg-2 (FP32)
    workloads with the bound of their dominant kernel.  Returns a seeded
    sample of their outputs for the oracle leg."""
    out, sample = {}, []
    for w, peak, unit in ((synth.cfg1(), 78.6, "FP64 TFLOP/s"),
                          (synth.cfg2(), PEAK_FP32_MFMA_TFLOPS, "FP32 MFMA TFLOP/s")):
        dt = torch.float64 if w.precision == "fp64" else torch.float32
        X = torch.from_numpy(w.X).to("cuda", dt)
        Y = torch.from_numpy(w.Y).to("cuda", dt)
        Z = torch.from_numpy(w.Z).to("cuda", dt)
        ts = []
        for rep in range(3):
            m = fmg.fastmuygps_build(X, Y, w.k, w.kernel, w.nu, w.rho, w.noise,
                                     precision=w.precision, flags=fmg.FLAG_TIMING)
            nn = torch.empty(Z.shape[0], dtype=torch.int32, device="cuda")
            mu = m.predict(Z, nn_out=nn)
            ts.append(m.timings())
            if rep < 2:
                m.free()
        t = ts[-1]
        n, d, mq = w.X.shape[0], w.X.shape[1], w.Z.shape[0]
        # dominant kernel: the build's neighbour search over n^2 pairs; its
        # algorithmic work is 3d FP64 operations per pair (exact FP64 search)
        # or 2d flops per pair (FP32 MFMA screen)
        per_pair = 3 * d if w.precision == "fp64" else 2 * d
        search_ms = t["build_screen_ms"]
        achieved = per_pair * float(n) * n / (search_ms / 1e3) / 1e12
        rmse = float(np.sqrt(np.mean((mu.cpu().numpy() - w.Yz) ** 2)))
        out[w.name] = {
            "n_train": int(n), "n_test": int(mq), "d": int(d), "k": w.k,
            "precision": w.precision, "build_ms": round(t["build_total_ms"], 3),
            "predict_ms": round(t["predict_total_ms"], 3),
            "builds_per_s": round(1e3 / t["build_total_ms"], 3),
            "training_points_per_s": round(n / (t["build_total_ms"] / 1e3), 1),
            "predictions_per_s": round(mq / (t["predict_total_ms"] / 1e3), 1),
            "phases_ms": {k: round(v, 3) for k, v in t.items()},
            "search_roofline": {"achieved": round(achieved, 2), "peak": peak, "unit": unit,
                                "frac": round(achieved / peak, 4),
                                "algorithmic_ops_per_launch": per_pair * float(n) * n},
            "rmse": rmse}
        rs = synth.rng(7, 4)
        rows = np.sort(rs.choice(n, 256, replace=False))
        qs = np.sort(rs.choice(mq, min(1024, mq), replace=False))
        sample.append((w, rows, m.neighbors().cpu().numpy()[rows], qs, mu.cpu().numpy()[qs],
                       nn.cpu().numpy()[qs]))
        m.free()
        del X, Y, Z
        log("%s: %s" % (w.name, {k: v for k, v in out[w.name].items() if k != "phases_ms"}))
    result["configs"] = out
    return sample


if __name__ == "__main__":
    main()
