#!/usr/bin/env python3
"""Throughput of the fused single-V NLL + gradient on one MI355X.

Workload: K = 16 waves, FP32 amplitudes, 10^6 data events and 5 x 10^6 MC
events (Breit-Wigner x Y_J^0 stand-in amplitudes, seeded), one production
vector V; a step is one synchronous NLL + gradient evaluation (V in, NLL and
gradient back on the host), i.e. one pass over all 6 x 10^6 event rows.

Prints ONE JSON line: throughput in event-evaluations per second, the HBM
roofline of the likelihood kernel (kernel time from HIP events on the stream
it runs on), and the FP64 CPU oracle timed on the host as a reported baseline.

The line's "extras" object holds the extended forms, each on its own
workload: "batched" (K = 32, 2e6 data + 1e7 MC events, 256 vectors in one
matrix-core pass, against the single-V kernel on the same sample),
"surrogate" (the K = 16 sample above: 1e5 exact pairs, network training,
screening of 1e5 starts, refinement of the best 256, against random starts)
and, with --extras multifit, the 64-fit uneven family.
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
# committed counter summaries of the single-V kernel, one per launch configuration
TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "traffic_nll_stream_k16*.json")
# the files the streaming kernel's code comes from: its loop, and the in-launch
# combine of the block partials
KERNEL_SRCS = [os.path.join(ROOT, "paper_1108_5882_amd", "csrc", f) for f in ("nll_stream_impl.hpp", "block_reduce.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    """SHA-256 prefix of the kernel's source files, concatenated in order."""
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(units_per_launch, kernel: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary taken on
    this kernel source, launch configuration and rows per launch, or None when
    there is none."""
    import glob
    for path in sorted(glob.glob(TRAFFIC_GLOB)):
        try:
            with open(path) as f:
                t = json.load(f)
        except (OSError, ValueError):
            continue
        if (t.get("kernel_sha256_16") == kernel_hash() and t.get("units_per_launch") == units_per_launch
                and t.get("kernel") == kernel):
            return t.get("hbm_bytes_per_launch")
    return None


def host_threads() -> int:
    """Threads the OpenMP oracle runs on: OMP_NUM_THREADS, else the CPUs this process may use."""
    try:
        n = int(os.environ.get("OMP_NUM_THREADS", "0"))
    except ValueError:
        n = 0
    return n if n > 0 else len(os.sched_getaffinity(0))


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sample, V, budget_s: float):
    """The FP64 oracle on the host: its chunked form (fixed 65536-row chunks, the
    result independent of the thread count) on one thread and on all the threads
    this process may use, each for about budget_s / 2 seconds."""
    import numpy as np

    import oracle
    Ad = np.ascontiguousarray(sample.A_data, dtype=np.complex128)
    Am = np.ascontiguousarray(sample.A_mc, dtype=np.complex128)
    rows = Ad.shape[0] + Am.shape[0]
    out = {}
    for threads in (1, host_threads()):
        oracle.nll_grad_chunked(Ad, Am, V, threads=threads)
        evals, t0 = 0, time.perf_counter()
        while True:
            oracle.nll_grad_chunked(Ad, Am, V, threads=threads)
            evals += 1
            if time.perf_counter() - t0 >= budget_s / 2:
                break
        dt = time.perf_counter() - t0
        out[threads] = (evals * rows / dt, evals, dt)
    n = host_threads()
    v1, e1, d1 = out[1]
    vn, en, dn = out[n]
    return {"value": vn, "unit": "event-evals/s", "cores": n, "kind": "oracle",
            "sample": f"FP64 NLL+grad evaluations of the full workload ({Ad.shape[0]} data + {Am.shape[0]} MC "
                      f"rows): {en} in {dn:.1f} s on {n} threads, {e1} in {d1:.1f} s on one thread",
            "single_thread": {"value": v1, "cores": 1},
            "host": {"cpu": cpu_model(), "threads_available": len(os.sched_getaffinity(0))}}


def kernel_name(cfg) -> str:
    return "nll_stream_kernel<float, L=%d, C=%d, U=%d>, %d blocks/CU" % (
        cfg["lanes_per_row"], cfg["complex_per_lane"], cfg["rows_per_stage"], cfg["blocks_per_cu"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--extras", default="batched,surrogate,hessian,kinematic,multifit",
                    help="comma list of batched, surrogate, hessian, kinematic, multifit (or none)")
    ap.add_argument("--probe", action="store_true",
                    help="for HBM counter runs: a few evaluations plus a plain device copy of the "
                         "same byte count (the counter scale reference); prints no JSON")
    ap.add_argument("--cfg", default="",
                    help="lanes_per_row,complex_per_lane,rows_per_stage,blocks_per_cu of the single-V kernel "
                         "instead of autotuning (for counter runs on the configuration a bench run chose)")
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
    if args.cfg:
        ctx.set_stream_cfg(*[int(x) for x in args.cfg.split(",")])
        cfg = ctx.stream_cfg()
        log(f"stream configuration {cfg} (given)")
    else:
        cfg, tune_ms = ctx.autotune(reps=20)
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
        log(f"probe: 5 evaluations of {kernel_name(cfg)} and 5 copies of {nbytes} bytes")
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
    kernel = kernel_name(cfg)
    traffic = stored_traffic(units, kernel)
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": kernel,
            "kernel_ms": k_ms,
            "alg_bytes_per_launch": alg_bytes,
            "per_evaluation_frac": alg_bytes / (ms_step * 1e-3) / 1e9 / HBM_PEAK_GBS}

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
    extras = [e for e in args.extras.split(",") if e and e != "none"]
    rec["extras"] = {}
    if "hessian" in extras:
        rec["extras"]["hessian"] = extra_hessian(ctx, V, nd, k)
        rec["extras"]["hessian"]["k48"] = extra_hessian_k48()
    if "surrogate" in extras:
        rec["extras"]["surrogate"] = extra_surrogate(ctx, k)
    ctx.close()
    del s
    if "kinematic" in extras:
        rec["extras"]["kinematic"] = extra_kinematic()
    if "batched" in extras:
        rec["extras"]["batched"] = extra_batched()
    if "multifit" in extras:
        rec["extras"]["multifit"] = extra_multifit()
    print(json.dumps(rec), flush=True)


MFMA_PEAK_TFS = 2500.0       # dense FP16 / BF16 matrix-core peak of the MI355X


def extra_batched(nv: int = 256, reps: int = 10):
    """256 vectors in one matrix-core pass (K = 32, 2e6 data + 1e7 MC) against one
    single-V streaming pass per vector on the same sample."""
    import torch

    import synth
    from paper_1108_5882_amd import Context

    t0 = time.perf_counter()
    s = synth.make_sample(2)
    Vs = synth.eval_vectors(2, nv, s.k)
    nd, nm, k = s.A_data.shape[0], s.A_mc.shape[0], s.k
    rows = nd + nm
    log(f"batched: sample {nd} + {nm} rows, K={k}, {time.perf_counter() - t0:.1f}s")
    ctx = Context(0, "f32")
    ctx.set_amplitudes("data", s.A_data)
    ctx.set_amplitudes("mc", s.A_mc)
    cfg, _ = ctx.autotune(reps=3)
    ctx.set_timing(True)
    for _ in range(5):
        ctx.nll_grad(Vs[0])
    ctx.kernel_time()
    w0 = time.perf_counter()
    for b in range(20):
        ctx.nll_grad(Vs[b])
    single_wall = (time.perf_counter() - w0) / 20
    single_ms, _ = ctx.kernel_time()
    timed = {}
    for split in (2, 3):
        for _ in range(2):
            ctx.nll_batch(Vs, split=split)
        ctx.batch_kernel_time()
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(reps):
            ctx.nll_batch(Vs, split=split)
        wall = (time.perf_counter() - w0) / reps
        b_ms, b_n = ctx.batch_kernel_time()
        timed[split] = (wall, b_ms, b_n)
        log(f"batched split {split}: {wall * 1e3:.3f} ms per call, kernels {b_ms:.3f} ms")
    ctx.set_timing(False)
    ctx.close()
    ks = 2 * k
    alg_flops = 2 * (2.0 * rows * ks * 2 * nv)           # forward GEMM and adjoint GEMM
    exec_flops = 3 * alg_flops                           # three split products each
    wall, b_ms, b_n = timed[3]
    w2, b2_ms, _ = timed[2]
    return {
        "workload": f"batched NLL+grad, K={k} FP32, {nd} data + {nm} MC events, {nv} vectors, split 3 "
                    "(matrix cores, small coherent sums recomputed exactly: 1e-6 for every vector)",
        "value": nv * rows / wall,
        "unit": "event-evals/s",
        "ms_per_call": wall * 1e3,
        "kernel_ms": b_ms,
        "kernel_launches": b_n,
        "single_v": {"value": rows / single_wall, "kernel_ms": single_ms, "ms_per_call": single_wall * 1e3,
                     "config": cfg},
        "speedup_vs_single_v_loop": (nv * single_wall) / wall,
        "roofline": {"bound": "mfma", "achieved": alg_flops / (b_ms * 1e-3) / 1e12, "peak": MFMA_PEAK_TFS,
                     "unit": "TFLOP/s", "frac": alg_flops / (b_ms * 1e-3) / 1e12 / MFMA_PEAK_TFS,
                     "traffic": None,
                     "kernel": "nll_batch_kernel (v_mfma_f32_16x16x32 f16 forward, bf16 adjoint) + exact refinement",
                     "alg_flops_per_launch": alg_flops,
                     "executed_mfma_tflops": exec_flops / (b_ms * 1e-3) / 1e12},
        "split2": {"value": nv * rows / w2, "ms_per_call": w2 * 1e3, "kernel_ms": b2_ms,
                   "executed_mfma_frac": exec_flops / (b2_ms * 1e-3) / 1e12 / MFMA_PEAK_TFS,
                   "error": "NLL below 2e-7 for every vector; gradient median below 1e-6, 95th percentile "
                            "below 1e-4, maximum below 1e-3 on small samples"},
    }


def extra_surrogate(ctx, k: int, n_train: int = 100000, n_screen: int = 100000, top: int = 256,
                    epochs: int = 30, batch: int = 1024, budgets=(5, 10, 20, 50, 100, 200)):
    """Surrogate-screened multi-start against random starts on the single-V sample.

    Both arms refine their starts for each iteration budget in `budgets` (from the
    starts, one batched fit per budget) and are judged by the exact NLL; the target
    is the lowest NLL any run reached, and each arm reports the smallest budget and
    the wall time (pipeline included for the surrogate arm) at which its best start
    came within 1 unit of NLL of it.
    """
    import math

    import numpy as np
    import torch

    import synth
    from paper_1108_5882_amd import Mlp, surrogate

    ctx.set_mc_mode("gram")
    V_train = synth.eval_vectors(4, n_train, k, stream=1)
    V_screen = synth.eval_vectors(4, n_screen, k, stream=2)
    V_plain = synth.eval_vectors(4, top, k, stream=3)
    perm = synth.permutations(n_train, epochs, batch, seed=1)
    mlp = Mlp(2 * k, 256, max_batch=8192)
    # warm-up of every stage on a small slice (graph capture, allocations)
    surrogate.multistart(ctx, mlp, V_train[:4096], V_screen[:4096], V_plain[:8], perm[:4 * batch] % 4096, batch,
                         iters=2, top=8, init=synth.mlp_init(2 * k, 256, seed=1))
    res = surrogate.multistart(ctx, mlp, V_train, V_screen, V_plain, perm, batch, iters=budgets[-1], top=top,
                               init=synth.mlp_init(2 * k, 256, seed=1))
    sec = res["seconds"]
    t_pipe = sec["pairs"] + sec["train"] + sec["screen"]
    starts = {"surrogate": V_screen[res["surrogate"]["sel"]], "random": V_plain}
    curve = {a: [] for a in starts}
    for T in budgets:
        for a, V0 in starts.items():
            torch.cuda.synchronize()
            w0 = time.perf_counter()
            r = surrogate.refine_and_judge(ctx, V0, T)
            torch.cuda.synchronize()
            curve[a].append((T, float(r["nll"].min()), float(np.median(r["nll"])), time.perf_counter() - w0))
    target = min(b for a in curve for _, b, _, _ in curve[a])
    reach = {}
    for a in curve:
        hit = [(T, t) for T, b, _, t in curve[a] if b <= target + 1.0]
        reach[a] = None if not hit else {"iterations": hit[0][0],
                                         "seconds": hit[0][1] + (t_pipe if a == "surrogate" else 0.0)}
    # random starts given the surrogate arm's whole wall time at the largest budget
    t_sur = t_pipe + curve["surrogate"][-1][3]
    n_eq = int(min(4096, top * max(1, math.ceil(t_sur / max(curve["random"][-1][3], 1e-9)))))
    V_eq = synth.eval_vectors(4, n_eq, k, stream=5)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    eq = surrogate.refine_and_judge(ctx, V_eq, budgets[-1])
    torch.cuda.synchronize()
    t_eq = time.perf_counter() - w0
    # screening throughput (features + inference + selection of the candidates)
    Vd = torch.from_numpy(np.stack([V_screen.real, V_screen.imag], -1).reshape(n_screen, -1)).cuda()
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(5):
        mlp.select(mlp.predict(mlp.features(Vd)), top)
    torch.cuda.synchronize()
    t_scr = (time.perf_counter() - w0) / 5
    mlp.close()
    ctx.set_mc_mode("stream")
    f_start = {a: float(np.median(ctx.nll_batch(V0, grad=False, split=0))) for a, V0 in starts.items()}
    out = {
        "workload": f"K={k}, {n_train} exact pairs (matrix-core pass, MC by the Gram matrix), network "
                    f"{2 * k}-256-256-1 trained {epochs} epochs of batch {batch}, {n_screen} candidates "
                    f"screened, best {top} refined by batched L-BFGS; {top} random starts refined alike",
        "median_start_nll": f_start,
        "best_and_median_nll_by_iterations": {a: [{"iterations": T, "best": b, "median": m, "seconds": t}
                                                  for T, b, m, t in curve[a]] for a in curve},
        "target_nll": target,
        "first_within_1_of_target": reach,
        f"random_{n_eq}_starts_equal_time": {"best": float(eq["nll"].min()), "median": float(np.median(eq["nll"])),
                                             "seconds": t_eq},
        "pipeline_seconds": {"pairs": sec["pairs"], "train": sec["train"], "screen": sec["screen"]},
        "train_ms_per_step": res["ms_per_train_step"],
        "train_loss_first_last": [float(res["losses"][:50].mean()), float(res["losses"][-50:].mean())],
        "screen_candidates_per_s": n_screen / t_scr,
    }
    log(f"surrogate: {json.dumps(out)}")
    return out


FP64_PEAK_TFS = 78.6         # FP64 peak of the MI355X (vector and matrix cores alike)


def hessian_flops(nd: int, k: int) -> float:
    """Algorithmic FP64 flops of the Hessian's data pass: per data event, z (8 K),
    u = 1 / z (about 12), B = A u (6 K) and the K (K + 1) / 2 distinct entries of
    the complex symmetric T = sum B B^T at 8 flops each (complex multiply-add)."""
    return nd * (4.0 * k * (k + 1) + 14.0 * k + 12.0)


def extra_hessian(ctx, V, nd: int, k: int, reps: int = 20):
    """The NLL Hessian (error matrix) on the single-V sample: one pass over the
    data rows plus the MC matrix (built once), synchronous calls; the kernels of
    each call timed with HIP events on the context's stream."""
    import numpy as np
    for _ in range(3):
        H = ctx.hessian(V)
    ctx.set_timing(True)
    ctx.hessian_kernel_time()
    w0 = time.perf_counter()
    for _ in range(reps):
        H = ctx.hessian(V)
    ms = (time.perf_counter() - w0) / reps * 1e3
    k_ms, k_count = ctx.hessian_kernel_time()
    ctx.set_timing(False)
    alg_flops = hessian_flops(nd, k)
    achieved = alg_flops / (k_ms * 1e-3) / 1e12
    log(f"hessian: {ms:.3f} ms per call, kernels {k_ms * 1e3:.1f} us ({nd} data rows, K={k})")
    return {"workload": f"NLL Hessian (2K x 2K) at one V, K={k}, {nd} data rows, MC by the Gram matrix",
            "ms_per_call": ms, "kernel_ms": k_ms, "kernel_calls": k_count,
            "symmetric_max_abs_diff": float(np.max(np.abs(H - H.T))),
            "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFS, "traffic": None,
                         "kernel": "hess_mfma_kernel (FP64 MFMA data pass) + partial sums + assembly",
                         "alg_flops_per_call": alg_flops,
                         "note": "events before the first and after the last kernel of one synchronous call "
                                 "(data pass, partial sums, assembly of H); includes the wait for the first "
                                 "launch on the idle stream"}}


def extra_hessian_k48(nd: int = 1_000_000, nm: int = 200_000):
    """The Hessian at K = 48 (the larger wave table), 1e6 FP32 data rows."""
    import synth
    from paper_1108_5882_amd import Context
    import torch
    s = synth.make_sample(2, n_data=nd, n_mc=nm, k=48)
    V = synth.eval_vectors(2, 1, 48)[0]
    with Context(0, "f32", stream=torch.cuda.Stream()) as c:
        c.set_amplitudes("data", s.A_data)
        c.set_amplitudes("mc", s.A_mc)
        return extra_hessian(c, V, nd, 48, reps=10)


# Algorithmic FP64 flops of the kinematic evaluation (FMA = 2): per (event, wave)
# the Breit-Wigner (m_a^2 - m^2, |D|^2, reciprocal with two Newton steps, BW),
# Y_J^0, A and its share of z: 28; the V-gradient term, conj(u) V_a Y_a, BW^2
# and the two resonance-gradient terms: 38.  Per event: Legendre polynomials,
# I, ln I or w I, 1/I and u: 30.
KIN_FLOPS_PER_EVENT_WAVE = 66
KIN_FLOPS_PER_EVENT = 30


def extra_kinematic(reps: int = 50):
    """Amplitudes formed on the GPU from (m, cos theta) with floating masses and
    widths: NLL, V gradient and (m_a, Gamma_a) gradient on the single-V workload's
    kinematics (K = 16, 1e6 data + 5e6 MC events, 8 bytes per event)."""
    import numpy as np
    import torch

    import synth
    from paper_1108_5882_amd import KinContext

    s = synth.make_kin_sample(1)
    V = synth.eval_vectors(1, 1, s.k)[0]
    nd, nm, k = s.mx_data.shape[0], s.mx_mc.shape[0], s.k
    stream = torch.cuda.Stream()
    kc = KinContext(s.waves.J, stream=stream)
    kc.set_events("data", s.mx_data)
    kc.set_events("mc", s.mx_mc)
    for _ in range(5):
        kc.nll_grad(V, s.res)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    for _ in range(reps):
        kc.nll_grad(V, s.res)
    sync_ms = (time.perf_counter() - w0) / reps * 1e3
    v = np.empty(2 * k)
    v[0::2], v[1::2] = V.real, V.imag
    Vd, Rd = torch.from_numpy(v).cuda(), torch.from_numpy(s.res).cuda()
    out = torch.zeros(4 * k + 2, dtype=torch.float64, device="cuda")
    # the launches are bound by vector arithmetic, so the clock matters: time
    # them after the device has run them long enough to reach its steady clock
    for _ in range(4 * reps):
        kc.nll_grad_async(Vd, Rd, out)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(reps):
        kc.nll_grad_async(Vd, Rd, out)
    ev1.record(stream)
    torch.cuda.synchronize()
    k_ms = ev0.elapsed_time(ev1) / reps
    kc.close()
    events = nd + nm
    flops = events * (KIN_FLOPS_PER_EVENT + KIN_FLOPS_PER_EVENT_WAVE * k)
    log(f"kinematic: {sync_ms:.3f} ms per synchronous call, {k_ms:.3f} ms per launch (back to back)")
    return {"workload": f"NLL + V and (mass, width) gradients with amplitudes formed on the GPU from (m, cos theta), "
                        f"K={k}, {nd} data + {nm} MC events, FP64 arithmetic",
            "value": events / (sync_ms * 1e-3), "unit": "event-evals/s", "ms_per_call": sync_ms,
            "kernel_ms": k_ms,
            "roofline": {"bound": "alu", "achieved": flops / (k_ms * 1e-3) / 1e12, "peak": FP64_PEAK_TFS,
                         "unit": "TFLOP/s", "frac": flops / (k_ms * 1e-3) / 1e12 / FP64_PEAK_TFS, "traffic": None,
                         "kernel": "kin_kernel<L=4> (4 waves per lane)", "alg_flops_per_launch": flops,
                         "hbm_bytes_per_launch": events * 8}}


def extra_multifit(steps: int = 50):
    """The 64-fit uneven family: one persistent evaluation + device L-BFGS per iteration."""
    import synth
    from paper_1108_5882_amd import MultiFit

    t0 = time.perf_counter()
    table = synth.multifit_table(64)
    samples, V0 = [], []
    for f, (nd, k, nm) in enumerate(table):
        s = synth.make_sample(3, n_data=nd, n_mc=nm, k=k, fit=f)
        samples.append((s.A_data, s.A_mc, None, None))
        V0.append(synth.eval_vectors(3, 1, k, stream=f)[0])
    rows = sum(a.shape[0] + b.shape[0] for a, b, _, _ in samples)
    bytes_ = sum((a.shape[0] + b.shape[0]) * a.shape[1] * 8 for a, b, _, _ in samples)
    log(f"multifit: 64 fits, {rows} rows, {bytes_ / 1e9:.1f} GB, generated in {time.perf_counter() - t0:.0f}s")
    t0 = time.perf_counter()
    mf = MultiFit(samples, V0)
    del samples
    log(f"multifit: staged on the device in {time.perf_counter() - t0:.1f}s")
    cfgm, tune_ms = mf.autotune(reps=3)
    log(f"multifit: autotuned {cfgm}: {tune_ms:.3f} ms per evaluation of all fits")
    mf.reset(V0)
    mf.step(2)
    mf.reset(V0)
    ms = mf.step(steps)
    log(f"multifit: {ms:.3f} ms per minimiser iteration")
    _, f, st, it = mf.get()
    mf.close()
    return {"workload": "64 fits, N_D log-uniform in [1e4, 1e6], K uniform in 4..48, N_MC = 5 N_D, FP32",
            "rows": rows, "ms_per_iteration": ms, "event_evals_per_s": rows / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": bytes_ / (tune_ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": bytes_ / (tune_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "traffic": None, "kernel": "multi_stream_kernel + combine (persistent item queue)",
                         "autotuned": cfgm},
            "accepted_iterations_min_max": [int(it.min()), int(it.max())]}


if __name__ == "__main__":
    main()
