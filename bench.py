"""Benchmark: forward overlap-and-save of one long complex64 signal with a bank
of filters on one MI355X, through the C ABI.

Workload: 2^23-sample complex64 signal (re/im uniform[-1,1]), 32 complex64
filters of 256 taps (re/im N(0,1)/sqrt(256)), FFT length 2048, output
32 x 2^23 complex64.  Inputs are resident in HBM before timing starts.

One step = one ols_forward call (the whole fused path: segment load, forward
FFT, 32 spectrum products and inverse FFTs, discard and store).  Prints one
JSON line.  The roofline object prices the forward kernel against the HBM
peak using its algorithmic bytes per launch and its average launch duration
(HIP events on the launch stream); the cpu_baseline object times the CPU
oracle (eq. 1, float64) on a bounded prefix of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "valid output samples/sec (all filters) and % HBM roofline; fwd+bwd vs plain OLS"
WORKLOAD = "filter_bank_2p23_k32_m256"
KERNEL_SOURCES = ("ols_kernels.hip", "ols_fft.hpp", "ols_ops.hpp", "ols_twiddle.hpp")
HOST_MARKER = b"// Host side"


def _code_tokens(data: bytes) -> bytes:
    """C++ source without comments and with whitespace runs collapsed (the
    device sources hold no string literals that contain comment markers)."""
    data = re.sub(rb"/\*.*?\*/", b" ", data, flags=re.S)
    data = re.sub(rb"//[^\n]*", b" ", data)
    return re.sub(rb"\s+", b" ", data).strip()


def kernel_hash() -> str:
    """Hash of the device code: the headers and the kernel source up to its
    host-side section, comments and layout ignored (host-only and comment
    edits leave a traffic record valid; the launch shape is checked
    separately)."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1910_01972_amd", "csrc", f), "rb") as fh:
            data = fh.read()
        if f.endswith(".hip"):
            cut = data.find(HOST_MARKER)
            if cut >= 0:
                data = data[:cut]
        h.update(_code_tokens(data))
    return h.hexdigest()[:16]


def measured_traffic(workload: str, launch: dict):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current device code and the same launch shape; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_ols_forward_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash() or rec.get("launch") != launch:
        return None
    return rec.get("hbm_bytes_per_launch")


def launch_spread(ms) -> dict:
    """Per-launch durations of the timed launches (HIP events): mean, min,
    median, max, and the first and last launch."""
    import numpy as np
    ms = np.asarray(ms, dtype=np.float64)
    return {"mean": float(ms.mean()), "min": float(ms.min()), "median": float(np.median(ms)),
            "max": float(ms.max()), "first": float(ms[0]), "last": float(ms[-1]), "n": int(ms.size)}


def settle_clocks(fn, settle_ms: float) -> dict:
    """Runs fn back to back for settle_ms of wall time before any warm-up or
    timed launch, so that the GPU leaves its idle power state first (from
    idle, the first tens of milliseconds of launches run slower).  Reported
    as its own field; none of these launches is timed."""
    import torch
    n = 0
    t0 = time.perf_counter()
    while (time.perf_counter() - t0) * 1e3 < settle_ms:
        for _ in range(10):
            fn()
        n += 10
        torch.cuda.synchronize()
    return {"ms": (time.perf_counter() - t0) * 1e3, "launches": n}


def cpu_baseline(s, h, n_sample: int):
    """The oracle (eq. 1 by definition, float64) on the first n_sample outputs
    of every filter row; returns samples/s and the BLAS thread count."""
    from threadpoolctl import threadpool_info

    from oracle import conv

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    t0 = time.perf_counter()
    conv.direct_conv(s[:n_sample], h)
    dt = time.perf_counter() - t0
    K = h.shape[0]
    return {
        "value": K * n_sample / dt,
        "unit": "samples/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"eq. (1) float64 direct convolution (oracle.conv.direct_conv), first {n_sample} outputs "
                  f"of all {K} filter rows of the same workload; {dt:.1f} s wall",
    }


def fwd_bwd_measurement(steps: int, warmup: int) -> dict:
    """Forward, backward (ds and dh) and forward+backward on the differentiable
    workload (2^22 samples, 16 filters of 512 taps, N = 4096), timed with HIP
    events on the launch stream, beside the plain forward."""
    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSPlan

    wl = workloads.WORKLOADS["grad_2p22_k16_m512"]
    s_np, h_np = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    g_np = workloads.make_grad(wl.K, wl.Ns, seed=wl.seed)
    s = torch.from_numpy(s_np).cuda()
    g = torch.from_numpy(g_np).cuda()
    plan = OLSPlan(torch.from_numpy(h_np).cuda(), N=wl.N)
    plan.reserve_backward()
    y = torch.empty((wl.K, wl.Ns), dtype=torch.complex64, device="cuda")
    ds = torch.empty(wl.Ns, dtype=torch.complex64, device="cuda")
    dh = torch.empty((wl.K, wl.M), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        for a, b in ev:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return float(np.mean([a.elapsed_time(b) for a, b in ev]))

    fwd = timed(lambda: plan.forward(s, y))
    bwd = timed(lambda: plan.backward(s, g, ds=ds, dh=dh))
    both = timed(lambda: (plan.forward(s, y), plan.backward(s, g, ds=ds, dh=dh)))
    plan.close()
    out = wl.K * wl.Ns
    return {
        "workload": wl.name, "Ns": wl.Ns, "K": wl.K, "M": wl.M, "N": wl.N,
        "fwd_ms": fwd, "bwd_ms": bwd, "fwd_bwd_ms": both,
        "fwd_samples_per_s": out / (fwd * 1e-3),
        "fwd_bwd_samples_per_s": out / (both * 1e-3),
        "bwd_over_fwd": bwd / fwd,
    }


def variants_measurement(steps: int, warmup: int) -> dict:
    """The fused post-processing options (power, derivative) on the benchmark
    filter bank, and the real-to-real path on the same shape with real data,
    each timed with HIP events on the launch stream; bytes are the algorithmic
    HBM bytes of each variant (signal + outputs + taps)."""
    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSPlan

    stream = torch.cuda.current_stream()

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    out = {}
    wl = workloads.WORKLOADS["filter_bank_2p23_k32_m256"]
    s_np, h_np = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    s, h = torch.from_numpy(s_np).cuda(), torch.from_numpy(h_np).cuda()
    for name, kw, ybytes in (("power", {"power": True}, 4), ("derivative", {"derivative": True}, 8)):
        plan = OLSPlan(h, N=wl.N, **kw)
        y = torch.empty((wl.K, wl.Ns), dtype=torch.float32 if ybytes == 4 else torch.complex64, device="cuda")
        ms = timed(lambda: plan.forward(s, y))
        alg = ybytes * wl.K * wl.Ns + 8 * wl.Ns + 8 * wl.K * wl.M
        out[name] = {"workload": wl.name, "ms": ms, "samples_per_s": wl.K * wl.Ns / (ms * 1e-3),
                     "alg_GBps": alg / (ms * 1e-3) / 1e9}
        plan.close()
        del y
    del s, h
    wr = workloads.WORKLOADS["filter_bank_real_2p23_k32_m256"]
    s_np, h_np = workloads.make_real_signal_filters(wr.Ns, wr.K, wr.M, seed=wr.seed)
    s, h = torch.from_numpy(s_np).cuda(), torch.from_numpy(h_np).cuda()
    plan = OLSPlan(h, N=wr.N)
    y = torch.empty((wr.K, wr.Ns), dtype=torch.float32, device="cuda")
    ms = timed(lambda: plan.forward(s, y))
    alg = 4 * wr.K * wr.Ns + 4 * wr.Ns + 4 * wr.K * wr.M
    out["r2r"] = {"workload": wr.name, "ms": ms, "samples_per_s": wr.K * wr.Ns / (ms * 1e-3),
                  "alg_GBps": alg / (ms * 1e-3) / 1e9}
    plan.close()
    del y
    torch.cuda.empty_cache()
    return out


def batched_measurement(steps: int, warmup: int, tuned: bool = True) -> dict:
    """The uneven batch (256 signals, N_s log-uniform in [2^14, 2^22], K ~
    U{1..16}, M log-uniform in [16, 1024]) as ONE persistent launch captured in
    a hipGraph and replayed, beside the same items run as one plain launch per
    signal."""
    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSBatch, OLSPlan

    shapes = workloads.batched_items()
    items = []
    outputs = 0
    for Ns, K, M, seed in shapes:
        s, h = workloads.make_signal_filters(Ns, K, M, seed=seed)
        items.append((torch.from_numpy(s).cuda(), torch.from_numpy(h).cuda(), 0))
        outputs += K * Ns
    b = OLSBatch(items)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.run(stream=stream)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b.run(stream=stream)

    def timed(fn):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    graph_ms = timed(graph.replay)
    chosen = [b.item(i)["N"] for i in range(len(items))]
    plans = [OLSPlan(h, N=chosen[i]) for i, (s, h, _) in enumerate(items)]

    def plain():
        for p, (s, h, _), y in zip(plans, items, b.outputs):
            p.forward(s, y)

    plain_ms = timed(plain)
    alg = sum(8.0 * K * Ns + 8.0 * Ns + 8.0 * K * M for Ns, K, M, _ in shapes)
    info = b.info()
    for p in plans:
        p.close()
    del graph  # before the batch it replays is released
    b.close()
    rec = {
        "workload": "uneven_batch_256", "signals": len(shapes), "output_samples": outputs,
        "units": info["units"], "grid": info["grid"], "fft_length": "library cost model",
        "graph_ms": graph_ms, "samples_per_s": outputs / (graph_ms * 1e-3),
        "GBps": alg / (graph_ms * 1e-3) / 1e9,
        "plain_per_signal_ms": plain_ms, "plain_samples_per_s": outputs / (plain_ms * 1e-3),
    }
    if not tuned:
        return rec

    # The same batch with N per (M, K) from the autotuner (single-signal
    # timings on a 2^22-sample proxy, N <= 4096), as its own captured graph.
    from paper_1910_01972_amd import tuner
    t0 = time.perf_counter()
    g = torch.Generator(device="cuda").manual_seed(1)
    proxy = torch.complex(torch.rand(1 << 22, device="cuda", generator=g) * 2 - 1,
                          torch.rand(1 << 22, device="cuda", generator=g) * 2 - 1)
    table = {}
    for Ns, K, M, _ in shapes:
        if (M, K) not in table:
            h = torch.complex(torch.randn(K, M, device="cuda", generator=g),
                              torch.randn(K, M, device="cuda", generator=g)) / M ** 0.5
            table[(M, K)] = tuner.tune(M, K, reps=5, max_n=4096, data=(proxy, h), tile=False)["N"]
    tune_s = time.perf_counter() - t0
    bt = OLSBatch(items, fft_length=lambda M, K: table[(M, K)])
    changed = sum(bt.item(i)["N"] != n for i, n in enumerate(chosen))
    with torch.cuda.stream(stream):
        bt.run(stream=stream)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        bt.run(stream=stream)
    tuned_ms = timed(graph.replay)
    del graph, proxy
    bt.close()
    rec["tuned"] = {"fft_length": "autotuner, 2^22-sample proxy per (M, K)", "pairs": len(table),
                    "tune_s": tune_s, "items_with_other_N": changed, "graph_ms": tuned_ms}
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle timing")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side measurements (adjoint, batched, variants), so that a profile of this "
                         "run holds only the benchmark's launches")
    ap.add_argument("--no-tuned-batch", action="store_true",
                    help="skip the uneven batch with the autotuner's N (keeps a profile to one batch plan)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--settle-ms", type=float, default=1000.0,
                    help="wall time of untimed back-to-back launches before the warm-up (reported as 'settle')")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="instead of the benchmark, run the library's plain copy kernel on MIB MiB "
                         "(known byte count, for scaling HBM traffic counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path is single-GPU", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSPlan

    if args.calibrate_copy:
        from paper_1910_01972_amd.ols import calibration_copy

        n = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(args.warmup + args.steps):
            calibration_copy(dst, src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": n * 8, "launches": args.warmup + args.steps}), flush=True)
        return

    wl = workloads.WORKLOADS[WORKLOAD]
    s_np, h_np = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    s = torch.from_numpy(s_np).to(dev)
    h = torch.from_numpy(h_np).to(dev)
    y = torch.empty((wl.K, wl.Ns), dtype=torch.complex64, device=dev)
    plan = OLSPlan(h, N=wl.N)
    info = plan.info()
    launch = plan.launch()
    nf = plan.tiling()["filters_per_unit"]
    launch_key = {"N": info["N"], "grid": launch["grid"], "block": launch["block"], "filters_per_unit": nf}
    stream = torch.cuda.current_stream()

    settle = settle_clocks(lambda: plan.forward(s, y), args.settle_ms)
    for _ in range(args.warmup):
        plan.forward(s, y)
    torch.cuda.synchronize()

    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        plan.forward(s, y)
        ends[i].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = np.array([a.elapsed_time(b) for a, b in zip(starts, ends)])
    kernel_ms = float(launch_ms.mean())

    ms_per_step = wall * 1e3 / args.steps
    outputs = wl.K * wl.Ns
    value = outputs / (ms_per_step * 1e-3)
    # algorithmic HBM bytes per launch: every output written once (8 B), the
    # signal read once (8 B/sample), the filter taps once
    alg_bytes = 8.0 * wl.K * wl.Ns + 8.0 * wl.Ns + 8.0 * wl.K * wl.M
    achieved = alg_bytes / (kernel_ms * 1e-3) / 1e9
    traffic = measured_traffic(WORKLOAD, launch_key)

    rec = {
        "metric": METRIC,
        "value": value,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": WORKLOAD,
            "Ns": wl.Ns, "K": wl.K, "M": wl.M, "N": info["N"], "hop": info["H"], "delay": info["D"],
            "grid": launch["grid"], "block": launch["block"], "cus": launch["cus"], "filters_per_unit": nf,
        },
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "kernel": f"ols_forward_kernel<{info['N']}, {nf}, false, false>",
            "kernel_ms": kernel_ms,
            "launch_ms": launch_spread(launch_ms),
            "alg_bytes_per_launch": alg_bytes,
        },
        "settle": settle,
    }
    plan.close()
    del y
    torch.cuda.empty_cache()
    if not args.no_side:
        rec["fwd_bwd"] = fwd_bwd_measurement(min(args.steps, 100), min(args.warmup, 50))
        rec["batched"] = batched_measurement(max(3, min(args.steps, 200) // 20), 3, tuned=not args.no_tuned_batch)
        rec["variants"] = variants_measurement(min(args.steps, 100), min(args.warmup, 50))
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(s_np, h_np, args.cpu_sample)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
