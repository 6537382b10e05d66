"""Autotuner: the FFT (segment) length and the kernel tiling per (filter
length M, filter count K).

The paper observes that each segment length is best for a band of filter
lengths and that the best choice depends on the implementation (sec. 3.2,
Fig. 9, sec. 5); the library's built-in choice is a cost model (FFT work per
valid output).  This tuner measures instead: for every candidate N >= M it
times the forward kernel on a synthetic signal and keeps the fastest; then,
for that N, it times the tilings of the forward kernel -- filters per work
unit (1 or 2 interleaved inverse transforms) and persistent workgroups per
compute unit, which sets the number of consecutive segments each workgroup
owns -- and keeps the fastest.  Results are cached in a JSON file keyed by the
GPU's architecture name, M and K.

    python -m paper_1910_01972_amd.tuner --M 512 --K 8          # tune one cell
    python -m paper_1910_01972_amd.tuner --sweep                # the 12-cell sweep on 2^25 samples
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

CANDIDATES = (256, 512, 1024, 2048, 4096, 8192)
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ols_mi355x_tune.json")
HBM_PEAK_GBS = 8000.0


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # pragma: no cover
        return "unknown"


def _time_forward(plan, s, y, reps: int, warmup: int = 2) -> float:
    for _ in range(warmup):
        plan.forward(s, y)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        plan.forward(s, y)
        b.record()
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def synthetic(Ns: int, K: int, M: int, seed: int):
    """Timing data drawn on the GPU: signal re/im uniform[-1, 1], filter re/im
    N(0, 1)/sqrt(M) (the values do not change the kernel's time)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    s = torch.complex(torch.rand(Ns, device="cuda", generator=g) * 2 - 1,
                      torch.rand(Ns, device="cuda", generator=g) * 2 - 1)
    h = torch.complex(torch.randn(K, M, device="cuda", generator=g),
                      torch.randn(K, M, device="cuda", generator=g)) / M ** 0.5
    return s, h


# The 12 cells of the FFT-length sweep: M in {32, 128, 512, 2048} x K in {1, 8, 64}
# on a 2^25-sample signal (seeds 3000 + cell index).
SWEEP_NS = 1 << 25
SWEEP_CELLS = tuple((M, K, 3000 + 3 * i + j) for i, M in enumerate((32, 128, 512, 2048))
                    for j, K in enumerate((1, 8, 64)))


def tilings(plan) -> list:
    """Candidate (filters per unit, workgroups per CU) for a plan."""
    from ._lib import OLSError
    out = []
    for nf in (1, 2):
        try:
            plan.set_tiling(nf, 0)
        except OLSError:
            continue
        for wpc in range(1, plan.tiling()["max_workgroups_per_cu"] + 1):
            out.append((nf, wpc))
    plan.set_tiling(0, 0)
    return out


def tune(M: int, K: int, Ns: int = 1 << 22, reps: int = 10, candidates=CANDIDATES, max_n: int = 8192,
         data=None, tile: bool = True) -> dict:
    """Time every candidate N >= M (N <= max_n) with the default tiling, then
    every tiling at the fastest N; returns the best configuration and all
    timings (ms per launch)."""
    from .ols import OLSPlan
    s, h = data if data is not None else synthetic(Ns, K, M, seed=M * 1000 + K)
    Ns = int(s.shape[0])
    y = torch.empty((K, Ns), dtype=torch.complex64, device="cuda")
    times = {}
    usable = [N for N in candidates if M <= N <= max_n]
    # a segment keeps N - (M - 1) outputs; below a quarter of N the overlap
    # dominates and the candidate cannot win (at N = M it keeps one sample)
    good = [N for N in usable if 4 * (N - M + 1) >= N]
    for N in good or usable:
        plan = OLSPlan(h, N=N)
        times[N] = _time_forward(plan, s, y, reps)
        plan.close()
    best = min(times, key=times.get)
    plan = OLSPlan(h, N=best)
    default = plan.tiling()
    cfg = (default["filters_per_unit"], default["workgroups_per_cu"])
    tiling_ms = {f"{cfg[0]}x{cfg[1]}": times[best]}
    if tile:
        for nf, wpc in tilings(plan):
            key = f"{nf}x{wpc}"
            if key in tiling_ms:
                continue
            plan.set_tiling(nf, wpc)
            tiling_ms[key] = _time_forward(plan, s, y, reps)
        key = min(tiling_ms, key=tiling_ms.get)
        cfg = tuple(int(v) for v in key.split("x"))
    H = plan.info()["H"]
    cus = plan.launch()["cus"]
    plan.close()
    nseg = -(-Ns // H)
    return {"M": M, "K": K, "Ns": Ns, "N": best, "filters_per_unit": cfg[0], "workgroups_per_cu": cfg[1],
            "segments_per_workgroup": nseg / (cfg[1] * cus), "ms": times, "tiling_ms": tiling_ms}


class TuneCache:
    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def key(self, M: int, K: int, max_n: int) -> str:
        return f"{_arch()}|M={M}|K={K}|max={max_n}"

    def config(self, M: int, K: int, max_n: int = 8192, **kw) -> dict:
        """Tuned {N, filters_per_unit, workgroups_per_cu} for (M, K), measured
        once and cached."""
        k = self.key(M, K, max_n)
        if not isinstance(self.data.get(k), dict):
            r = tune(M, K, max_n=max_n, **kw)
            self.data[k] = {"N": r["N"], "filters_per_unit": r["filters_per_unit"],
                            "workgroups_per_cu": r["workgroups_per_cu"]}
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            with open(self.path, "w") as f:
                json.dump(self.data, f, indent=1)
        return dict(self.data[k])

    def best(self, M: int, K: int, max_n: int = 8192, **kw) -> int:
        return int(self.config(M, K, max_n=max_n, **kw)["N"])

    def plan(self, h: torch.Tensor, **kw):
        """An OLSPlan for the filter bank h with the tuned N and tiling."""
        from .ols import OLSPlan
        K, M = int(h.shape[0]), int(h.shape[1])
        c = self.config(M, K, **kw)
        p = OLSPlan(h, N=c["N"])
        p.set_tiling(c["filters_per_unit"], c["workgroups_per_cu"])
        return p

    def batched_fft_length(self, M: int, K: int) -> int:
        """Chooser for OLSBatch (batched items use N <= 4096)."""
        return self.best(M, K, max_n=4096)


def sweep(reps: int = 10, tune_ns: int = 1 << 22):
    """The 12 cells (M in {32, 128, 512, 2048} x K in {1, 8, 64}) on a 2^25
    sample signal: N tuned on a 2^22-sample proxy, then measured at full size.
    Prints one JSON line per cell."""
    from types import SimpleNamespace

    from .ols import OLSPlan
    for M, K, seed in SWEEP_CELLS:
        wl = SimpleNamespace(name=f"sweep_2p25_m{M}_k{K}", M=M, K=K, Ns=SWEEP_NS, seed=seed)
        proxy = synthetic(tune_ns, wl.K, wl.M, seed=wl.seed)
        t = tune(wl.M, wl.K, reps=reps, data=proxy)
        del proxy
        s, h = synthetic(wl.Ns, wl.K, wl.M, seed=wl.seed)
        y = torch.empty((wl.K, wl.Ns), dtype=torch.complex64, device="cuda")
        plan = OLSPlan(h, N=t["N"])
        # default and tuned tiling timed alternately (twice each, after a
        # longer warm-up), the lower median of each kept
        ms_default, ms = float("inf"), float("inf")
        for _ in range(2):
            plan.set_tiling(0, 0)
            ms_default = min(ms_default, _time_forward(plan, s, y, max(reps, 20), warmup=20))
            plan.set_tiling(t["filters_per_unit"], t["workgroups_per_cu"])
            ms = min(ms, _time_forward(plan, s, y, max(reps, 20), warmup=20))
        auto = OLSPlan(h, N=0)
        auto_n = auto.info()["N"]
        auto.close()
        alg = 8.0 * wl.K * wl.Ns + 8.0 * wl.Ns + 8.0 * wl.K * wl.M
        rec = {"cell": wl.name, "M": wl.M, "K": wl.K, "Ns": wl.Ns, "tuned_N": t["N"], "cost_model_N": auto_n,
               "filters_per_unit": t["filters_per_unit"], "workgroups_per_cu": t["workgroups_per_cu"],
               "segments_per_workgroup": -(-wl.Ns // plan.info()["H"]) / plan.launch()["grid"],
               "proxy_ms": t["ms"], "proxy_tiling_ms": t["tiling_ms"], "ms_default_tiling": ms_default,
               "ms": ms, "samples_per_s": wl.K * wl.Ns / (ms * 1e-3),
               "GBps": alg / (ms * 1e-3) / 1e9, "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        plan.close()
        del s, h, y
        torch.cuda.empty_cache()
        print(json.dumps(rec), flush=True)


def run_config(M: int, K: int, Ns: int, N: int, nf: int, wpc: int, reps: int = 10) -> dict:
    """The forward for one (M, K) on Ns synthetic samples with a fixed FFT
    length and tiling (0: the library's choice): reps timed launches after
    two warm-ups.  Reports the configuration that ran."""
    from .ols import OLSPlan
    s, h = synthetic(Ns, K, M, seed=M * 1000 + K)
    y = torch.empty((K, Ns), dtype=torch.complex64, device="cuda")
    plan = OLSPlan(h, N=N)
    plan.set_tiling(nf, wpc)
    ms = _time_forward(plan, s, y, reps)
    launch, tiling = plan.launch(), plan.tiling()
    n_used = plan.fft_length()
    plan.close()
    return {"M": M, "K": K, "Ns": Ns, "N": n_used, "filters_per_unit": tiling["filters_per_unit"],
            "workgroups_per_cu": tiling["workgroups_per_cu"], "ms": ms, "grid": launch["grid"]}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--M", type=int)
    ap.add_argument("--K", type=int)
    ap.add_argument("--Ns", type=int, default=1 << 22)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--run", nargs=3, type=int, metavar=("N", "NF", "WPC"),
                    help="only run the forward for --M, --K on --Ns samples with this FFT length and tiling "
                         "(filters per unit, workgroups per CU), e.g. under a profiler")
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    if a.sweep:
        sweep(reps=a.reps)
    elif a.run:
        print(json.dumps(run_config(a.M, a.K, a.Ns, *a.run, reps=a.reps)))
    else:
        print(json.dumps(tune(a.M, a.K, Ns=a.Ns, reps=a.reps)))


if __name__ == "__main__":
    main()
