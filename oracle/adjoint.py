"""Oracle: adjoint of eq. (1) (gradients of a real loss), FP64, test-only.

eq. (1) with zero history is linear in the signal and in each filter:
    y_r[n] = sum_{k=0}^{M-1} h_r[k] s[n-k],   n = 0 .. N_s-1, s[m<0] = 0.
For a real loss with upstream gradient g_r[n] (complex convention: the gradient
of a real function with respect to z is dL/d(conj z), the one PyTorch uses),
the gradients are the adjoint maps applied to g:
    ds[m]    = sum_r sum_k conj(h_r[k]) g_r[m+k]        (g_r[n] = 0 for n >= N_s)
    dh_r[k]  = sum_n conj(s[n-k]) g_r[n]               (s[m] = 0 for m < 0)
ds is a correlation with the conjugated filters that uses only future samples
of g, so in overlap-and-save form it aliases the END of each segment (the
footnote to eq. 2).  Both are written here by their plain definitions.
"""

from __future__ import annotations

import numpy as np

__all__ = ["grad_signal", "grad_filters", "grad_signal_at", "grad_signal_loops", "grad_filters_loops"]


def grad_signal_loops(g, h) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128)
    K, Ns = g.shape
    M = h.shape[1]
    ds = np.zeros(Ns, dtype=np.complex128)
    for m in range(Ns):
        acc = 0j
        for r in range(K):
            for k in range(M):
                if m + k < Ns:
                    acc += np.conj(h[r, k]) * g[r, m + k]
        ds[m] = acc
    return ds


def grad_filters_loops(g, s, M: int) -> np.ndarray:
    g = np.asarray(g, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    K, Ns = g.shape
    dh = np.zeros((K, M), dtype=np.complex128)
    for r in range(K):
        for k in range(M):
            acc = 0j
            for n in range(Ns):
                if n - k >= 0:
                    acc += np.conj(s[n - k]) * g[r, n]
            dh[r, k] = acc
    return dh


def grad_signal(g, h, chunk: int = 1 << 16) -> np.ndarray:
    """ds[m] = sum_r sum_k conj(h_r[k]) g_r[m+k], m in [0, N_s)."""
    g = np.asarray(g, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128)
    K, Ns = g.shape
    M = h.shape[1]
    ds = np.zeros(Ns, dtype=np.complex128)
    if Ns == 0:
        return ds
    hc = np.conj(h)  # (K, M)
    for r in range(K):
        gp = np.concatenate([g[r], np.zeros(M - 1, dtype=np.complex128)])
        win = np.lib.stride_tricks.sliding_window_view(gp, M)  # win[m, k] = g[m+k]
        for m0 in range(0, Ns, chunk):
            m1 = min(Ns, m0 + chunk)
            ds[m0:m1] += win[m0:m1] @ hc[r]
    return ds


def grad_filters(g, s, M: int, chunk: int = 1 << 16) -> np.ndarray:
    """dh_r[k] = sum_n conj(s[n-k]) g_r[n], k in [0, M)."""
    g = np.asarray(g, dtype=np.complex128)
    s = np.asarray(s, dtype=np.complex128)
    K, Ns = g.shape
    dh = np.zeros((K, M), dtype=np.complex128)
    if Ns == 0:
        return dh
    sp = np.concatenate([np.zeros(M - 1, dtype=np.complex128), np.conj(s)])
    # win[n, j] = conj(s[n + j - (M-1)]); tap k = M-1-j
    win = np.lib.stride_tricks.sliding_window_view(sp, M)
    for n0 in range(0, Ns, chunk):
        n1 = min(Ns, n0 + chunk)
        dh += (g[:, n0:n1] @ win[n0:n1])[:, ::-1]
    return dh


def grad_signal_at(g, h, idx) -> np.ndarray:
    """ds[m] = sum_r sum_k conj(h_r[k]) g_r[m+k] at the indices idx only
    (local: ds[m] needs g_r[m .. m+M-1]), for sampled checks of huge problems."""
    g = np.asarray(g, dtype=np.complex128)
    h = np.asarray(h, dtype=np.complex128)
    idx = np.asarray(idx, dtype=np.int64).ravel()
    K, Ns = g.shape
    M = h.shape[1]
    if np.any(idx < 0) or np.any(idx >= Ns):
        raise IndexError("index out of range")
    src = idx[:, None] + np.arange(M)[None, :]  # (n, M): g index for tap k
    ok = src < Ns
    src = np.minimum(src, Ns - 1)
    out = np.zeros(idx.shape[0], dtype=np.complex128)
    hc = np.conj(h)
    for r in range(K):
        vals = np.where(ok, g[r][src], 0.0)
        out += vals @ hc[r]
    return out
