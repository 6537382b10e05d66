"""Seeded synthetic inputs for overlap-and-save convolution (no method arithmetic).

This module only draws random numbers and describes workload shapes.  It is the
single piece shared by the CPU oracle's tests and the GPU path's tests and
benchmark; it computes nothing the method computes.

Recipe (the paper's workloads are synthetic signal/filter lengths and filter
counts, sec. 4; the paper does not state value distributions, so these are ours):

* generator: ``numpy.random.Generator(numpy.random.PCG64(seed))``;
* draw order: signal real parts, signal imaginary parts, filter real parts
  (shape (K, M)), filter imaginary parts;
* signal: real and imaginary parts i.i.d. uniform[-1, 1];
* filters: real and imaginary parts i.i.d. N(0, 1) / sqrt(M);
* upstream gradient (for the adjoint): real and imaginary parts i.i.d. N(0, 1),
  drawn after the filters;
* everything is cast to complex64 on the host; the float64 oracle sees the very
  same complex64 values promoted to complex128.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

__all__ = ["Workload", "WORKLOADS", "make_signal_filters", "make_grad", "sweep_cells", "batched_items"]


@dataclass(frozen=True)
class Workload:
    name: str
    Ns: int      # signal length
    K: int       # number of filters
    M: int       # filter length
    N: int       # FFT (segment) length; 0 = chosen by the library
    seed: int


# Workloads named for what they are.
WORKLOADS = {
    # one filter: 2^20 samples, M = 64, N = 1024
    "single_filter_2p20": Workload("single_filter_2p20", 1 << 20, 1, 64, 1024, 1),
    # filter bank: 2^23 samples, 32 filters of 256 taps, N = 2048
    "filter_bank_2p23_k32_m256": Workload("filter_bank_2p23_k32_m256", 1 << 23, 32, 256, 2048, 2),
    # differentiable: 2^22 samples, 16 filters of 512 taps, N = 4096
    "grad_2p22_k16_m512": Workload("grad_2p22_k16_m512", 1 << 22, 16, 512, 4096, 5),
    # real data (R2R): 2^23 real samples, 32 real filters of 256 taps, N = 2048
    "filter_bank_real_2p23_k32_m256": Workload("filter_bank_real_2p23_k32_m256", 1 << 23, 32, 256, 2048, 6),
}


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def make_signal_filters(Ns: int, K: int, M: int, seed: int, rng: np.random.Generator | None = None):
    """Return (s complex64 [Ns], h complex64 [K, M]) drawn in the documented order."""
    g = _rng(seed) if rng is None else rng
    sr = g.uniform(-1.0, 1.0, Ns)
    si = g.uniform(-1.0, 1.0, Ns)
    s = (sr + 1j * si).astype(np.complex64)
    scale = 1.0 / np.sqrt(M)
    hr = g.standard_normal((K, M)) * scale
    hi = g.standard_normal((K, M)) * scale
    h = (hr + 1j * hi).astype(np.complex64)
    return s, h


def make_real_signal_filters(Ns: int, K: int, M: int, seed: int):
    """Real-data case (R2R): (s float32 [Ns] ~ U[-1, 1], h float32 [K, M] ~
    N(0, 1/M)), drawn in that order from the seed's stream."""
    g = _rng(seed)
    s = g.uniform(-1.0, 1.0, Ns).astype(np.float32)
    h = (g.standard_normal((K, M)) / np.sqrt(M)).astype(np.float32)
    return s, h


def exact_signal(start: int, stop: int, device="cpu"):
    """Samples start .. stop-1 of a long deterministic complex64 signal,
    s[n] = ((n*40503) mod 2^20)/2^20 - 1/2 + i (((n*65537) mod 2^20)/2^20 - 1/2):
    integer arithmetic and exactly representable float32 values, so any window
    is rebuilt bit for bit from n alone, on any device (for signals too long to
    draw on the host)."""
    import torch
    n = torch.arange(start, stop, dtype=torch.int64, device=device)
    re = ((n * 40503) % (1 << 20)).to(torch.float32) / (1 << 20) - 0.5
    im = ((n * 65537) % (1 << 20)).to(torch.float32) / (1 << 20) - 0.5
    return torch.complex(re, im)


def make_grad(K: int, Ns: int, seed: int):
    """Upstream gradient dL/dy, complex64 [K, Ns], real/imag i.i.d. N(0, 1).

    Drawn from the same stream as the signal and filters of ``seed`` would be
    continued; to keep it independent of (Ns, M) we use a derived seed.
    """
    g = _rng(seed * 1000003 + 17)
    gr = g.standard_normal((K, Ns))
    gi = g.standard_normal((K, Ns))
    return (gr + 1j * gi).astype(np.complex64)


def sweep_cells():
    """(M, K) cells of the FFT-length sweep on a 2^25-sample signal, with seeds."""
    cells = []
    i = 0
    for M in (32, 128, 512, 2048):
        for K in (1, 8, 64):
            cells.append(Workload(f"sweep_2p25_m{M}_k{K}", 1 << 25, K, M, 0, 3000 + i))
            i += 1
    return cells


def batched_items(n_signals: int = 256, seed: int = 4, min_log2: float = 14.0, max_log2: float = 22.0,
                  max_k: int = 16, m_log2_range=(4.0, 10.0)):
    """Shapes of the uneven batch: per signal (Ns, K, M), lengths log-uniform.

    N_s = round(2^U(min_log2, max_log2)), K ~ U{1..max_k}, M = round(2^U(4, 10)).
    Only the shapes are drawn here; values come from ``make_signal_filters``
    with seed ``seed * 100000 + i``.
    """
    g = _rng(seed)
    out = []
    for i in range(n_signals):
        Ns = int(round(2.0 ** g.uniform(min_log2, max_log2)))
        K = int(g.integers(1, max_k + 1))
        M = int(round(2.0 ** g.uniform(*m_log2_range)))
        out.append((Ns, K, M, seed * 100000 + i))
    return out
