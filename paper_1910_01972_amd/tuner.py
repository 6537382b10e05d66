"""Autotuner: the FFT (segment) length per (filter length M, filter count K).

The paper observes that each segment length is best for a band of filter
lengths and that the best choice depends on the implementation (sec. 3.2,
Fig. 9, sec. 5); the library's built-in choice is a cost model (FFT work per
valid output).  This tuner measures instead: for every candidate N >= M it
times the forward kernel on a synthetic signal and keeps the fastest per valid
output sample.  Results are cached in a JSON file keyed by the GPU's
architecture name, M and K.

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
    import workloads
    s, h = workloads.make_signal_filters(Ns, K, M, seed=seed)
    return torch.from_numpy(s).cuda(), torch.from_numpy(h).cuda()


def tune(M: int, K: int, Ns: int = 1 << 22, reps: int = 10, candidates=CANDIDATES, max_n: int = 8192,
         data=None) -> dict:
    """Time every candidate N >= M (N <= max_n); returns the fastest and all timings."""
    from .ols import OLSPlan
    s, h = data if data is not None else synthetic(Ns, K, M, seed=M * 1000 + K)
    Ns = int(s.shape[0])
    y = torch.empty((K, Ns), dtype=torch.complex64, device="cuda")
    times = {}
    for N in candidates:
        if N < M or N > max_n:
            continue
        plan = OLSPlan(h, N=N)
        times[N] = _time_forward(plan, s, y, reps)
        plan.close()
    best = min(times, key=times.get)
    return {"M": M, "K": K, "Ns": Ns, "N": best, "ms": times}


class TuneCache:
    def __init__(self, path: str = DEFAULT_CACHE):
        self.path = path
        self.data = {}
        if os.path.exists(path):
            with open(path) as f:
                self.data = json.load(f)

    def key(self, M: int, K: int, max_n: int) -> str:
        return f"{_arch()}|M={M}|K={K}|max={max_n}"

    def best(self, M: int, K: int, max_n: int = 8192, **kw) -> int:
        k = self.key(M, K, max_n)
        if k not in self.data:
            self.data[k] = tune(M, K, max_n=max_n, **kw)["N"]
            os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
            with open(self.path, "w") as f:
                json.dump(self.data, f, indent=1)
        return int(self.data[k])

    def batched_fft_length(self, M: int, K: int) -> int:
        """Chooser for OLSBatch (batched items use N <= 4096)."""
        return self.best(M, K, max_n=4096)


def sweep(reps: int = 10, tune_ns: int = 1 << 22):
    """The 12 cells (M in {32, 128, 512, 2048} x K in {1, 8, 64}) on a 2^25
    sample signal: N tuned on a 2^22-sample proxy, then measured at full size.
    Prints one JSON line per cell."""
    import workloads
    from .ols import OLSPlan
    for wl in workloads.sweep_cells():
        proxy = synthetic(tune_ns, wl.K, wl.M, seed=wl.seed)
        t = tune(wl.M, wl.K, reps=reps, data=proxy)
        del proxy
        s, h = synthetic(wl.Ns, wl.K, wl.M, seed=wl.seed)
        y = torch.empty((wl.K, wl.Ns), dtype=torch.complex64, device="cuda")
        plan = OLSPlan(h, N=t["N"])
        ms = _time_forward(plan, s, y, reps)
        auto = OLSPlan(h, N=0)
        auto_n = auto.info()["N"]
        auto.close()
        alg = 8.0 * wl.K * wl.Ns + 8.0 * wl.Ns + 8.0 * wl.K * wl.M
        rec = {"cell": wl.name, "M": wl.M, "K": wl.K, "Ns": wl.Ns, "tuned_N": t["N"], "cost_model_N": auto_n,
               "proxy_ms": t["ms"], "ms": ms, "samples_per_s": wl.K * wl.Ns / (ms * 1e-3),
               "GBps": alg / (ms * 1e-3) / 1e9, "hbm_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        plan.close()
        del s, h, y
        torch.cuda.empty_cache()
        print(json.dumps(rec), flush=True)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--M", type=int)
    ap.add_argument("--K", type=int)
    ap.add_argument("--Ns", type=int, default=1 << 22)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--sweep", action="store_true")
    a = ap.parse_args(argv)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    if a.sweep:
        sweep(reps=a.reps)
    else:
        print(json.dumps(tune(a.M, a.K, Ns=a.Ns, reps=a.reps)))


if __name__ == "__main__":
    main()
