#!/usr/bin/env python3
"""Throughput of the fused single-V NLL + gradient on one MI355X.

Workload: K = 16 waves, FP32 amplitudes, 10^6 data events and 5 x 10^6 MC
events (Breit-Wigner x Y_J^0 stand-in amplitudes, seeded), one production
vector V; a step is one synchronous NLL + gradient evaluation (V in, NLL and
gradient back on the host), i.e. one pass over all 6 x 10^6 event rows.

Prints ONE JSON line: throughput in event-evaluations per second, the HBM
roofline of the likelihood kernel (kernel time from HIP events on the stream
it runs on), and the FP64 CPU oracle timed on the host as a reported baseline.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "NLL+grad event-evals/s, batched vs single-V at 1e-6 rel err; %HBM / %MFMA peak"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_nll_stream_k16.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1108_5882_amd", "csrc", "nll_stream_impl.hpp")


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def stored_traffic(units_per_launch):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha256_16") != kernel_hash() or t.get("units_per_launch") != units_per_launch:
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(sample, V, budget_s: float):
    import oracle
    evals, t0 = 0, time.perf_counter()
    while True:
        oracle.nll_grad(sample.A_data, sample.A_mc, V)
        evals += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    units = evals * (sample.A_data.shape[0] + sample.A_mc.shape[0])
    return {"value": units / dt, "unit": "event-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{evals} FP64 NLL+grad evaluations of the full workload "
                      f"({sample.A_data.shape[0]} data + {sample.A_mc.shape[0]} MC rows), "
                      f"{dt:.1f} s, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe", action="store_true",
                    help="for HBM counter runs: a few evaluations plus a plain device copy of the "
                         "same byte count (the counter scale reference); prints no JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the likelihood path has no multi-GPU mode "
              "(events would shard with one FP64 all-reduce per evaluation); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_1108_5882_amd import Context

    t0 = time.perf_counter()
    s = synth.make_sample(1)
    V = synth.eval_vectors(1, 1, s.k)[0]
    nd, nm, k = s.A_data.shape[0], s.A_mc.shape[0], s.k
    units = nd + nm
    log(f"sample: {nd} data + {nm} MC rows, K={k}, generated in {time.perf_counter() - t0:.1f}s")

    stream = torch.cuda.Stream()
    ctx = Context(0, "f32", stream=stream)
    ctx.set_amplitudes("data", s.A_data)
    ctx.set_amplitudes("mc", s.A_mc)
    cfg, tune_ms = ctx.autotune(reps=5)
    log(f"autotuned stream configuration {cfg}: {tune_ms * 1e3:.1f} us")
    for _ in range(args.warmup):
        ctx.nll_grad(V)
    torch.cuda.synchronize()
    if args.probe:
        nbytes = units * 8 * k
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
            ctx.nll_grad(V)
        torch.cuda.synchronize()
        log(f"probe: 5 evaluations and 5 copies of {nbytes} bytes")
        return

    ctx.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    w0 = time.perf_counter()
    for _ in range(args.steps):
        nll, grad = ctx.nll_grad(V)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_step = max(ev0.elapsed_time(ev1), wall * 1e3) / args.steps
    k_ms, k_count = ctx.kernel_time()
    ctx.set_timing(False)
    log(f"steps={args.steps} ms/step={ms_step:.4f} kernel avg={k_ms:.4f} ms over {k_count} launches "
        f"nll={nll:.10g}")

    alg_bytes = units * 8 * k            # FP32 complex amplitudes read once per event
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    traffic = stored_traffic(units)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": "nll_stream_kernel<float, L=%d, C=%d, U=%d>, %d blocks/CU"
                      % (cfg["lanes_per_row"], cfg["complex_per_lane"], cfg["rows_per_stage"],
                         cfg["blocks_per_cu"]),
            "kernel_ms": k_ms,
            "alg_bytes_per_launch": alg_bytes}

    rec = {
        "metric": METRIC,
        "value": units / (ms_step * 1e-3),
        "unit": "event-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "single-V NLL+grad, K=16 FP32, 1e6 data + 5e6 MC events",
                   "k": k, "n_data": nd, "n_mc": nm, "n_v": 1, "mc_mode": "stream"},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle ...")
        rec["cpu_baseline"] = cpu_baseline(s, V, args.cpu_seconds)
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
