"""Oracle: linear convolution by definition (eq. 1), by the convolution theorem
(eq. 2) and by overlap-and-save (sec. 3.2, Alg. 2).  FP64, CPU, test-only.

Readings of the paper taken here (the paper is silent or inconsistent):

* eq. (1) indexes s[n-k] for n-k < 0; we take a zero history (s[m] = 0 for
  m < 0) and produce N_s outputs n = 0 .. N_s-1 (the first N_s samples of the
  full linear convolution).
* The number of aliased samples per segment is M-1 (sec. 3.2), so a segment of
  length N yields L = N-M+1 valid samples; for a causal filter they sit at the
  start of the segment (footnote to eq. 2).
* In Alg. 2 the spectrum product inside the filter loop is written in place;
  we read it as P_r = A * F_r with the segment spectrum A kept unchanged, so
  filter r sees only its own spectrum (sec. 3.4: segment samples are reused for
  every filter).
* Alg. 2 reads segment b at x[b*N_seg + t]; we read segment j as the window
  that starts M-1 samples before the j-th block of H new samples, i.e.
  x[j*H - (M-1) + t], with zeros outside [0, N_s).  The hop H defaults to L and
  may be any 1 <= H <= L (the result does not depend on the segment size,
  sec. 3.2).
* The inverse transform carries the 1/N normalisation.
"""

from __future__ import annotations

import math

import numpy as np

__all__ = [
    "direct_conv",
    "direct_conv_at",
    "direct_conv_loops",
    "direct_conv_real",
    "direct_conv_real_at",
    "dft",
    "fft",
    "ifft",
    "full_fft_conv",
    "ols_conv",
    "ols_segment_count",
]


def _as_filters(h) -> np.ndarray:
    h = np.asarray(h, dtype=np.complex128)
    if h.ndim == 1:
        h = h[None, :]
    if h.ndim != 2 or h.shape[1] < 1:
        raise ValueError("filters must have shape (K, M) with M >= 1")
    return h


def _as_signal(s) -> np.ndarray:
    s = np.asarray(s, dtype=np.complex128)
    if s.ndim != 1:
        raise ValueError("signal must be one-dimensional")
    return s


# ---------------------------------------------------------------------------
# eq. (1): discrete linear convolution, y[n] = sum_{k=0}^{M-1} s[n-k] h[k]
# ---------------------------------------------------------------------------

def direct_conv_loops(s, h) -> np.ndarray:
    """eq. (1) written as explicit loops.  Only for tiny inputs (brute force)."""
    s = _as_signal(s)
    h = _as_filters(h)
    K, M = h.shape
    Ns = s.shape[0]
    y = np.zeros((K, Ns), dtype=np.complex128)
    for r in range(K):
        for n in range(Ns):
            acc = 0j
            for k in range(M):
                if n - k >= 0:
                    acc += s[n - k] * h[r, k]
            y[r, n] = acc
    return y


def direct_conv(s, h, chunk: int = 1 << 16) -> np.ndarray:
    """eq. (1) for all K filters and all n in [0, N_s), zero history.

    Row n of the sliding-window view of ``[0]*(M-1) ++ s`` holds
    s[n-(M-1)] .. s[n]; its j-th entry is s[n-k] with k = M-1-j, so the sum over
    k is one matrix product with the reversed filters (a library matmul used as
    the summation step, done in chunks of output samples to bound memory).
    Returns complex128 of shape (K, N_s).
    """
    s = _as_signal(s)
    h = _as_filters(h)
    K, M = h.shape
    Ns = s.shape[0]
    y = np.empty((K, Ns), dtype=np.complex128)
    if Ns == 0:
        return y
    padded = np.concatenate([np.zeros(M - 1, dtype=np.complex128), s])
    windows = np.lib.stride_tricks.sliding_window_view(padded, M)  # (Ns, M)
    hrev = np.ascontiguousarray(h[:, ::-1].T)  # (M, K): hrev[j, r] = h[r, M-1-j]
    for n0 in range(0, Ns, chunk):
        n1 = min(Ns, n0 + chunk)
        y[:, n0:n1] = (windows[n0:n1] @ hrev).T
    return y


def direct_conv_real(s, h, chunk: int = 1 << 16) -> np.ndarray:
    """eq. (1) for a real signal and real filters (the R2R case of sec. 1 and
    3.4), in float64: the same sum as ``direct_conv`` with real operands.
    Returns float64 of shape (K, N_s)."""
    s = np.asarray(s, dtype=np.float64)
    h = np.asarray(h, dtype=np.float64)
    if h.ndim == 1:
        h = h[None, :]
    if s.ndim != 1 or h.ndim != 2 or h.shape[1] < 1:
        raise ValueError("signal must be 1-D and filters (K, M) with M >= 1")
    K, M = h.shape
    Ns = s.shape[0]
    y = np.empty((K, Ns), dtype=np.float64)
    if Ns == 0:
        return y
    padded = np.concatenate([np.zeros(M - 1), s])
    windows = np.lib.stride_tricks.sliding_window_view(padded, M)  # (Ns, M)
    hrev = np.ascontiguousarray(h[:, ::-1].T)
    for n0 in range(0, Ns, chunk):
        n1 = min(Ns, n0 + chunk)
        y[:, n0:n1] = (windows[n0:n1] @ hrev).T
    return y


def direct_conv_real_at(s, h, idx) -> np.ndarray:
    """``direct_conv_real`` at the output indices idx only (eq. 1 is local)."""
    s = np.asarray(s, dtype=np.float64)
    h = np.atleast_2d(np.asarray(h, dtype=np.float64))
    idx = np.asarray(idx, dtype=np.int64).ravel()
    K, M = h.shape
    Ns = s.shape[0]
    if np.any(idx < 0) or np.any(idx >= Ns):
        raise IndexError("output index out of range")
    src = idx[:, None] - np.arange(M, dtype=np.int64)[None, :]
    vals = np.where(src >= 0, s[np.clip(src, 0, max(Ns - 1, 0))], 0.0)
    return (vals @ h.T).T


def direct_conv_at(s, h, idx) -> np.ndarray:
    """eq. (1) evaluated only at output indices ``idx`` (shape (K, len(idx))).

    eq. (1) is local: y[n] needs only s[n-M+1 .. n], so any output of a huge
    problem can be checked one by one.
    """
    s = _as_signal(s)
    h = _as_filters(h)
    idx = np.asarray(idx, dtype=np.int64).ravel()
    K, M = h.shape
    Ns = s.shape[0]
    if np.any(idx < 0) or np.any(idx >= Ns):
        raise IndexError("output index out of range")
    k = np.arange(M, dtype=np.int64)
    src = idx[:, None] - k[None, :]  # (n, M): s index for tap k
    ok = src >= 0
    vals = np.where(ok, s[np.clip(src, 0, max(Ns - 1, 0))], 0.0)  # (n, M)
    return (vals @ h.T).T  # (K, n)


# ---------------------------------------------------------------------------
# Discrete Fourier transform: definition and radix-2 Cooley-Tukey FFT
# ---------------------------------------------------------------------------

def dft(x, inverse: bool = False) -> np.ndarray:
    """O(N^2) DFT by definition along the last axis.

    forward: X[m] = sum_n x[n] exp(-2 pi i m n / N)
    inverse: x[n] = (1/N) sum_m X[m] exp(+2 pi i m n / N)
    """
    x = np.asarray(x, dtype=np.complex128)
    N = x.shape[-1]
    n = np.arange(N)
    sign = 1.0 if inverse else -1.0
    W = np.exp(sign * 2j * np.pi * np.outer(n, n) / N)
    out = x @ W.T
    return out / N if inverse else out


def _bit_reverse_indices(N: int) -> np.ndarray:
    bits = N.bit_length() - 1
    idx = np.arange(N)
    rev = np.zeros(N, dtype=np.int64)
    for b in range(bits):
        rev |= ((idx >> b) & 1) << (bits - 1 - b)
    return rev


def _fft_core(x: np.ndarray, sign: float) -> np.ndarray:
    """Iterative radix-2 decimation-in-time Cooley-Tukey FFT (last axis).

    Input is permuted into bit-reversed order, then log2(N) butterfly stages of
    span m = 2, 4, ..., N combine pairs (u, t) into (u + w^k t, u - w^k t) with
    w = exp(sign * 2 pi i / m).  Twiddles are evaluated directly per stage
    (no recurrences), in float64.
    """
    N = x.shape[-1]
    if N < 1 or (N & (N - 1)) != 0:
        raise ValueError("FFT length must be a power of two")
    y = x[..., _bit_reverse_indices(N)].astype(np.complex128, copy=True)
    m = 2
    while m <= N:
        half = m // 2
        k = np.arange(half)
        w = np.exp(sign * 2j * np.pi * k / m)  # (half,)
        blocks = y.reshape(y.shape[:-1] + (N // m, m))
        u = blocks[..., :half].copy()
        t = blocks[..., half:] * w
        blocks[..., :half] = u + t
        blocks[..., half:] = u - t
        y = blocks.reshape(y.shape)
        m *= 2
    return y


def fft(x) -> np.ndarray:
    """Forward FFT, X[m] = sum_n x[n] exp(-2 pi i m n / N), along the last axis."""
    return _fft_core(np.asarray(x, dtype=np.complex128), -1.0)


def ifft(X) -> np.ndarray:
    """Inverse FFT with the 1/N normalisation, along the last axis."""
    X = np.asarray(X, dtype=np.complex128)
    return _fft_core(X, +1.0) / X.shape[-1]


# ---------------------------------------------------------------------------
# eq. (2): convolution theorem on the whole signal, zero padded
# ---------------------------------------------------------------------------

def full_fft_conv(s, h) -> np.ndarray:
    """eq. (2): y = IFFT(FFT(pad(h)) * FFT(pad(s))) with padding to a power of
    two >= N_s + M - 1 (the footnote's condition, so no circular aliasing),
    truncated to the first N_s outputs (zero history, as eq. (1))."""
    s = _as_signal(s)
    h = _as_filters(h)
    K, M = h.shape
    Ns = s.shape[0]
    if Ns == 0:
        return np.zeros((K, 0), dtype=np.complex128)
    P = 1 << max(0, math.ceil(math.log2(Ns + M - 1)))
    S = fft(np.concatenate([s, np.zeros(P - Ns)]))
    Hf = fft(np.concatenate([h, np.zeros((K, P - M))], axis=1))
    return ifft(Hf * S[None, :])[:, :Ns]


# ---------------------------------------------------------------------------
# sec. 3.2 / Alg. 2: overlap-and-save
# ---------------------------------------------------------------------------

def ols_segment_count(Ns: int, hop: int) -> int:
    """Number of segments needed to cover N_s outputs with hop H."""
    return -(-Ns // hop) if Ns > 0 else 0


def ols_conv(s, h, N: int, hop: int | None = None) -> np.ndarray:
    """Overlap-and-save convolution of one signal with K filters (sec. 3.2).

    Steps, in the paper's order (Fig. 1 and Alg. 2):
      1. F_r = FFT(h_r zero padded to N)                   (filters first)
      2. split s into overlapping segments of length N; segment j covers
         s[j*H - (M-1) .. j*H - (M-1) + N - 1] (zeros outside [0, N_s))
      3. A_j = FFT(segment j)
      4. for every filter r: P = A_j * F_r  (A_j kept), a = IFFT(P)
      5. discard the M-1 aliased samples a[0 .. M-2]; keep a[M-1 .. M-1+H-1]
         as outputs j*H .. j*H+H-1 (clipped to N_s).
    Returns complex128 of shape (K, N_s).
    """
    s = _as_signal(s)
    h = _as_filters(h)
    K, M = h.shape
    Ns = s.shape[0]
    if N < 1 or (N & (N - 1)) != 0:
        raise ValueError("segment length N must be a power of two")
    if M > N:
        raise ValueError("filter longer than the segment")
    L = N - M + 1
    H = L if hop is None else int(hop)
    if not (1 <= H <= L):
        raise ValueError("hop must satisfy 1 <= H <= N-M+1")
    y = np.zeros((K, Ns), dtype=np.complex128)
    nseg = ols_segment_count(Ns, H)
    if nseg == 0:
        return y
    # step 1
    F = fft(np.concatenate([h, np.zeros((K, N - M))], axis=1))  # (K, N)
    # step 2: xp[i] = s[i - (M-1)], zero outside
    total = (nseg - 1) * H + N
    xp = np.zeros(total, dtype=np.complex128)
    xp[M - 1:M - 1 + Ns] = s[: max(0, min(Ns, total - (M - 1)))]
    starts = np.arange(nseg) * H
    segs = xp[starts[:, None] + np.arange(N)[None, :]]  # (nseg, N)
    # step 3
    A = fft(segs)
    out = np.zeros((K, nseg * H), dtype=np.complex128)
    for r in range(K):
        # step 4
        a = ifft(A * F[r][None, :])
        # step 5
        out[r] = a[:, M - 1:M - 1 + H].reshape(-1)
    y[:, :] = out[:, :Ns]
    return y
