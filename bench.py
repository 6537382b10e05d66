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


def profile_record(workload: str, launch: dict):
    """The committed rocprofv3 counter summary of the forward kernel (HBM bytes
    and VALU instructions per launch), if it was taken on the current device
    code and the same launch shape; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_ols_forward_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_hash") != kernel_hash() or rec.get("launch") != launch:
        return None
    return rec


# VALU issue rate of the chip: 256 CUs x 4 SIMDs, one wave64 instruction per
# SIMD every 4 cycles, at the 2.4 GHz peak engine clock (packed FP32 unused).
VALU_WAVE_INSTR_PER_S = 256 * 4 / 4 * 2.4e9


def floors(alg_bytes: float, rec, kernel_ms: float | None = None) -> dict:
    """Lower bounds on the launch time: HBM (algorithmic bytes at the 8 TB/s
    peak) and VALU (the profiled wave64 VALU instructions at the peak issue
    rate); 'binding' names the larger one.  With the measured launch time,
    'valu_frac' is the VALU floor over it (the VALU roofline fraction at the
    peak clock, beside the HBM one that `frac` reports)."""
    hbm_ms = alg_bytes / (HBM_PEAK_GBS * 1e9) * 1e3
    valu = rec.get("valu_instr_per_launch") if rec else None
    valu_ms = valu / VALU_WAVE_INSTR_PER_S * 1e3 if valu else None
    binding = "hbm" if valu_ms is None or hbm_ms >= valu_ms else "valu"
    out = {"hbm_ms": hbm_ms, "valu_ms": valu_ms, "valu_instr_per_launch": valu, "binding": binding}
    if kernel_ms:
        out["valu_frac"] = valu_ms / kernel_ms if valu_ms else None
    return out


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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(s, h, n_sample: int, N: int, reps: int = 3):
    """The oracle timed on the host, best of `reps`, both of its routes: eq. (1)
    by definition (oracle.conv.direct_conv, float64 BLAS) and the hand-written
    radix-2 FFT overlap-and-save (oracle.conv.ols_conv, float64), each on the
    first n_sample outputs of every filter row of the same workload; value is
    the faster route's output samples/s."""
    from threadpoolctl import threadpool_info

    from oracle import conv

    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    K = h.shape[0]
    routes = {}
    for name, fn in (("direct_eq1", lambda: conv.direct_conv(s[:n_sample], h)),
                     ("naive_fft_ols", lambda: conv.ols_conv(s[:n_sample], h, N))):
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            best = min(best, time.perf_counter() - t0)
        routes[name] = {"s": best, "samples_per_s": K * n_sample / best}
    top = max(routes, key=lambda k: routes[k]["samples_per_s"])
    return {
        "value": routes[top]["samples_per_s"],
        "unit": "samples/s",
        "cores": int(threads),
        "kind": "oracle",
        "sample": f"float64 oracle on the first {n_sample} outputs of all {K} filter rows of the same workload, "
                  f"best of {reps}; value = the faster route ({top})",
        "routes": routes,
        "cpu_model": _cpu_model(),
        "logical_cpus": os.cpu_count(),
    }


def single_filter_measurement(graph_launches: int = 128, replays: int = 5) -> dict:
    """The single-filter workload (2^20 samples, one 64-tap filter, N = 1024)
    is a few microseconds of work, so it is timed as graph_launches forward
    launches captured in ONE hipGraph, each on its own replica of the input
    and output (replicas rotated so that the footprint is >= 1 GB, four times
    the 256 MB last-level cache: HBM-cold), replayed `replays` times; also the
    same graph on one replica (cache-hot), labelled as such."""
    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSPlan

    wl = workloads.WORKLOADS["single_filter_2p20"]
    s_np, h_np = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    per_replica = 8 * wl.Ns * (1 + wl.K)
    R = -(-(1 << 30) // per_replica)
    s0 = torch.from_numpy(s_np).cuda()
    ss = [s0.clone() for _ in range(R)]
    ys = [torch.empty((wl.K, wl.Ns), dtype=torch.complex64, device="cuda") for _ in range(R)]
    plan = OLSPlan(torch.from_numpy(h_np).cuda(), N=wl.N)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    out = {"workload": wl.name, "Ns": wl.Ns, "K": wl.K, "M": wl.M, "N": wl.N, "replicas": R,
           "footprint_GB": R * per_replica / 1e9, "launches_per_graph": graph_launches}
    for label, idx in (("hbm_cold", lambda i: i % R), ("cache_hot", lambda i: 0)):
        with torch.cuda.stream(stream):
            for i in range(4):
                plan.forward(ss[idx(i)], ys[idx(i)], stream=stream)
        stream.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=stream):
            for i in range(graph_launches):
                plan.forward(ss[idx(i)], ys[idx(i)], stream=stream)
        graph.replay()
        torch.cuda.synchronize()
        times = []
        for _ in range(replays):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            graph.replay()
            b.record()
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b) * 1e3 / graph_launches)
        us = float(np.median(times))
        out[label] = {"us_per_launch": us, "samples_per_s": wl.K * wl.Ns / (us * 1e-6),
                      "hbm_frac": per_replica / (us * 1e-6) / (HBM_PEAK_GBS * 1e9)}
        del graph
    out["hbm_floor_us"] = per_replica / (HBM_PEAK_GBS * 1e9) * 1e6
    plan.close()
    del ss, ys
    torch.cuda.empty_cache()
    return out


def sweep_measurement(launches: int = 10, rounds: int = 3) -> dict:
    """The FFT-length sweep: 2^25-sample signal, M in {32, 128, 512, 2048} x
    K in {1, 8, 64}.  Per cell every candidate N >= M that keeps at least a
    quarter of each segment is timed at full size, interleaved over `rounds`
    rounds of `launches` launches (median per N), beside the library's
    cost-model choice; GB/s and the HBM fraction use the algorithmic bytes."""
    import numpy as np
    import torch

    from paper_1910_01972_amd import tuner
    from paper_1910_01972_amd.ols import OLSPlan

    cells = []
    for M, K, seed in tuner.SWEEP_CELLS:
        Ns = tuner.SWEEP_NS
        s, h = tuner.synthetic(Ns, K, M, seed)
        y = torch.empty((K, Ns), dtype=torch.complex64, device="cuda")
        plans = {N: OLSPlan(h, N=N) for N in tuner.CANDIDATES if N >= M and 4 * (N - M + 1) >= N}
        auto = OLSPlan(h, N=0)
        chosen, hop = auto.info()["N"], auto.info()["H"]
        tiling, grid = auto.tiling(), auto.launch()["grid"]
        auto.close()
        times = {N: [] for N in plans}
        for p in plans.values():
            for _ in range(3):
                p.forward(s, y)
        for _ in range(rounds):
            for N, p in plans.items():
                ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                      for _ in range(launches)]
                for a, b in ev:
                    a.record()
                    p.forward(s, y)
                    b.record()
                torch.cuda.synchronize()
                times[N] += [a.elapsed_time(b) for a, b in ev]
        med = {N: float(np.median(v)) for N, v in times.items()}
        best = min(med, key=med.get)
        alg = 8.0 * K * Ns + 8.0 * Ns + 8.0 * K * M
        frac = lambda ms: alg / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)
        # the cost model's configuration: hop H, tiling, and segments per
        # persistent workgroup S (average over the grid)
        cells.append({"M": M, "K": K, "cost_model_N": chosen, "hop": hop,
                      "filters_per_unit": tiling["filters_per_unit"],
                      "workgroups_per_cu": tiling["workgroups_per_cu"],
                      "segments_per_workgroup": round(-(-Ns // hop) / grid, 2),
                      "cost_model_ms": med[chosen], "cost_model_frac": frac(med[chosen]),
                      "cost_model_GBps": alg / (med[chosen] * 1e-3) / 1e9, "best_N": best, "best_ms": med[best],
                      "best_frac": frac(med[best]), "samples_per_s": K * Ns / (med[chosen] * 1e-3),
                      "ms_per_N": {str(N): round(v, 4) for N, v in med.items()}})
        for p in plans.values():
            p.close()
        del s, h, y
        torch.cuda.empty_cache()
    return {"Ns": tuner.SWEEP_NS, "launches": launches, "rounds": rounds, "cells": cells}


def roof_measurement(mib: int = 2048, launches: int = 20) -> dict:
    """Practical HBM ceilings on this GPU: the library's plain copy kernel
    (read + write) and a write-only fill of the same bytes."""
    import numpy as np
    import torch

    from paper_1910_01972_amd.ols import calibration_copy

    n = mib * (1 << 20) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)

    def timed(fn):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
        for a, b in ev:
            a.record()
            fn()
            b.record()
        torch.cuda.synchronize()
        return float(np.median([a.elapsed_time(b) for a, b in ev]))

    copy_ms = timed(lambda: calibration_copy(dst, src))
    fill_ms = timed(lambda: dst.fill_(1.0))
    nbytes = n * 8
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": nbytes, "copy_GBps": 2 * nbytes / (copy_ms * 1e-3) / 1e9,
            "fill_GBps": nbytes / (fill_ms * 1e-3) / 1e9}


SIDE_SETTLE_S = 0.2  # back-to-back calls before each side measurement's warm-up


def side_settle(fn, seconds: float = SIDE_SETTLE_S) -> None:
    """Run fn back to back for `seconds` (synchronising every 16 calls), so a
    side measurement starts with its buffers touched and the clocks loaded,
    as the headline's settle phase does for the benchmark."""
    import time

    import torch

    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        for _ in range(16):
            fn()
        torch.cuda.synchronize()


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
        side_settle(fn)
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
        "fwd_ms": fwd, "bwd_ms": bwd, "fwd_bwd_ms": both, "settle_s": SIDE_SETTLE_S,
        "fwd_samples_per_s": out / (fwd * 1e-3),
        "fwd_bwd_samples_per_s": out / (both * 1e-3),
        "bwd_over_fwd": bwd / fwd,
    }


def variants_measurement(steps: int, warmup: int) -> dict:
    """The fused post-processing options (power, derivative, the non-local
    stencil stage) on the benchmark filter bank, and the real-to-real path on
    the same shape with real data,
    each timed with HIP events on the launch stream; bytes are the algorithmic
    HBM bytes of each variant (signal + outputs + taps)."""
    import numpy as np
    import torch

    import workloads
    from paper_1910_01972_amd.ols import OLSPlan

    stream = torch.cuda.current_stream()

    def timed(fn):
        side_settle(fn)
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
    # the non-local stage (sec. 4): the backward difference from neighbouring
    # outputs (J = 1; the same result as the folded derivative above), the
    # cubic midpoint interpolation (J = 2 outputs per sample) and its power
    difference = ([[-1.0, 1.0]], 1)
    cubic = ([[0.0, 1.0, 0.0, 0.0], [-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16]], 1)
    for name, kw, ybytes in (("power", {"power": True}, 4), ("derivative", {"derivative": True}, 8),
                             ("stage_difference", {"stencil": difference}, 8),
                             ("stage_midpoint_cubic", {"stencil": cubic}, 8),
                             ("stage_midpoint_cubic_power", {"stencil": cubic, "power": True}, 4)):
        plan = OLSPlan(h, N=wl.N, **kw)
        J = plan.phases
        y = torch.empty((wl.K, J * wl.Ns), dtype=torch.float32 if ybytes == 4 else torch.complex64, device="cuda")
        ms = timed(lambda: plan.forward(s, y))
        alg = ybytes * J * wl.K * wl.Ns + 8 * wl.Ns + 8 * wl.K * wl.M
        out[name] = {"workload": wl.name, "ms": ms, "samples_per_s": wl.K * wl.Ns / (ms * 1e-3),
                     "outputs_per_sample": J, "alg_GBps": alg / (ms * 1e-3) / 1e9,
                     "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "settle_s": SIDE_SETTLE_S}
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
                  "alg_GBps": alg / (ms * 1e-3) / 1e9, "settle_s": SIDE_SETTLE_S}
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
    ap.add_argument("--no-sweep", action="store_true", help="skip the FFT-length sweep (2^25 samples, 12 cells)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 18)
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
    prof = profile_record(WORKLOAD, launch_key)
    traffic = prof.get("hbm_bytes_per_launch") if prof else None

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
            # the metric is the HBM roofline; "floors" says which floor binds
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
            "floors": floors(alg_bytes, prof, kernel_ms),
        },
        "settle": settle,
    }
    plan.close()
    del y
    torch.cuda.empty_cache()
    if not args.no_side:
        rec["practical_roof"] = roof_measurement()
        rec["single_filter"] = single_filter_measurement()
        rec["fwd_bwd"] = fwd_bwd_measurement(min(args.steps, 100), min(args.warmup, 50))
        rec["batched"] = batched_measurement(max(3, min(args.steps, 200) // 20), 3, tuned=not args.no_tuned_batch)
        rec["variants"] = variants_measurement(min(args.steps, 100), min(args.warmup, 50))
        if not args.no_sweep:
            rec["sweep"] = sweep_measurement()
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(s_np, h_np, args.cpu_sample, wl.N)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
