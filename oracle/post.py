"""Oracle: post-processing of the convolved signal (sec. 4), FP64, test-only.

The paper applies post-processing to the OLS output inside the convolution
kernel, per element (its example: the power) or over a neighbourhood of
elements (its example: the numerical derivative).  Readings taken here, where
the paper names the operation but not its formula:

* power: P_r[n] = |y_r[n]|^2 = Re(y_r[n])^2 + Im(y_r[n])^2, real valued (the
  complex-to-real case of the footnote in sec. 1);
* derivative: the backward first difference with unit sample spacing and the
  zero history of eq. (1), d_r[n] = y_r[n] - y_r[n-1], y_r[-1] = 0.  It is
  causal, so it needs only samples the segment already holds.
* stencil: the general neighbourhood operation of sec. 4 (its examples: the
  derivative and interpolation) read as a stencil with real weights and J
  outputs (phases) per sample: each output sample n yields J values
      z_r[J n + j] = sum_{d=-L}^{R} w[j][d + L] * y_r[n + d],   n = 0 .. N_s - 1,
  so a row of z has J * N_s samples.  y_r[m] = 0 for m < 0 (zero history of
  eq. (1)); for m >= N_s, y_r[m] is eq. (1) of the signal continued by zeros
  (the convolution's tail), the reading under which the last outputs of a
  stencil that looks ahead are defined.  The power may follow the stencil,
  which makes the whole operation non-linear in y.
* interpolation: the Lagrange polynomial through the samples at offsets
  nodes[0..T-1], evaluated at offset x (weights by the product formula).  The
  cubic midpoint (nodes -1, 0, 1, 2, x = 1/2) is the J = 2 stencil with
  phase 0 = y[n] and phase 1 = the value half a sample later.

All are written by their definitions on top of ``conv.direct_conv``.
"""

from __future__ import annotations

import numpy as np

from . import conv

__all__ = ["power", "derivative", "conv_power", "conv_derivative", "derivative_at", "stencil", "conv_stencil",
           "conv_stencil_real", "stencil_at", "lagrange_weights", "midpoint_interpolation_stencil"]


def power(y) -> np.ndarray:
    """|y|^2 element by element, float64."""
    y = np.asarray(y, dtype=np.complex128)
    return y.real * y.real + y.imag * y.imag


def derivative(y) -> np.ndarray:
    """Backward first difference along the last axis, y[-1] = 0."""
    y = np.asarray(y, dtype=np.complex128)
    d = y.copy()
    d[..., 1:] -= y[..., :-1]
    return d


def conv_power(s, h) -> np.ndarray:
    """Power of eq. (1)'s output, shape (K, N_s)."""
    return power(conv.direct_conv(s, h))


def conv_derivative(s, h) -> np.ndarray:
    """Derivative of eq. (1)'s output, shape (K, N_s)."""
    return derivative(conv.direct_conv(s, h))


def derivative_at(s, h, idx) -> np.ndarray:
    """d_r[n] at the output indices idx only: eq. (1) at n and n-1, differenced
    (zero for n-1 < 0), for sampled checks of large problems."""
    idx = np.asarray(idx, dtype=np.int64).ravel()
    cur = conv.direct_conv_at(s, h, idx)
    prev_idx = np.maximum(idx - 1, 0)
    prev = conv.direct_conv_at(s, h, prev_idx)
    prev[:, idx == 0] = 0
    return cur - prev


def stencil(y, w, left: int, Ns: int) -> np.ndarray:
    """z[..., J n + j] = sum_d w[j][d + left] * y[..., n + d] for n in [0, Ns),
    d in [-left, right], with y[m] = 0 for m < 0.

    y holds samples 0 .. Ns + right - 1 along its last axis (right = T - 1 -
    left, T = w.shape[1]); w has shape (J, T).  Returns shape (..., J * Ns),
    complex128.  Written as the double sum, one shifted slice of y per (j, d).
    """
    y = np.asarray(y, dtype=np.complex128)
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    J, T = w.shape
    right = T - 1 - left
    if left < 0 or right < 0:
        raise ValueError("the stencil must cover offset 0")
    if y.shape[-1] != Ns + right:
        raise ValueError(f"y needs {Ns + right} samples, has {y.shape[-1]}")
    z = np.zeros(y.shape[:-1] + (Ns, J), dtype=np.complex128)
    for j in range(J):
        for d in range(-left, right + 1):
            lo = max(0, -d)  # first n with n + d >= 0; earlier terms are zero
            if lo < Ns:
                z[..., lo:, j] += w[j, d + left] * y[..., lo + d:Ns + d]
    return z.reshape(y.shape[:-1] + (J * Ns,))


def _right_reach(w, left: int) -> int:
    return np.atleast_2d(np.asarray(w)).shape[1] - 1 - left


def conv_stencil(s, h, w, left: int) -> np.ndarray:
    """The stencil applied to eq. (1)'s output, shape (K, J * N_s): eq. (1) is
    evaluated on the signal continued by `right` zeros, which gives the tail
    samples y[N_s .. N_s + right - 1] the stencil reads."""
    s = np.asarray(s, dtype=np.complex128).ravel()
    R = _right_reach(w, left)
    y = conv.direct_conv(np.concatenate([s, np.zeros(R, dtype=np.complex128)]), h)
    return stencil(y, w, left, s.shape[0])


def conv_stencil_real(s, h, w, left: int) -> np.ndarray:
    """conv_stencil for a real signal and real filters (R2R); float64."""
    s = np.asarray(s, dtype=np.float64).ravel()
    R = _right_reach(w, left)
    y = conv.direct_conv_real(np.concatenate([s, np.zeros(R)]), h)
    return stencil(y, w, left, s.shape[0]).real


def stencil_at(s, h, w, left: int, idx, real: bool = False) -> np.ndarray:
    """Entries idx of conv_stencil's rows only (eq. (1) evaluated at the few
    samples each needs), for sampled checks of large problems."""
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    J, T = w.shape
    R = T - 1 - left
    idx = np.asarray(idx, dtype=np.int64).ravel()
    n, j = idx // J, idx % J
    dt = np.float64 if real else np.complex128
    s = np.asarray(s, dtype=dt).ravel()
    if np.any(idx < 0) or np.any(n >= s.shape[0]):
        raise IndexError("output index out of range")
    s_ext = np.concatenate([s, np.zeros(R, dtype=dt)])
    at = conv.direct_conv_real_at if real else conv.direct_conv_at
    z = None
    for d in range(-left, R + 1):
        m = n + d
        vals = at(s_ext, h, np.maximum(m, 0))
        vals = np.where((m >= 0)[None, :], vals, 0)
        term = w[j, d + left][None, :] * vals
        z = term if z is None else z + term
    return z


def lagrange_weights(nodes, x: float) -> np.ndarray:
    """Weights l_k(x) = prod_{i != k} (x - t_i) / (t_k - t_i) of the Lagrange
    polynomial through the sample offsets t = nodes: sum_k l_k(x) y[t_k] is the
    value at offset x of the polynomial of degree T-1 through the samples."""
    t = np.asarray(nodes, dtype=np.float64)
    out = np.ones(t.shape[0])
    for k in range(t.shape[0]):
        for i in range(t.shape[0]):
            if i != k:
                out[k] *= (x - t[i]) / (t[k] - t[i])
    return out


def midpoint_interpolation_stencil(left: int = 1, right: int = 2):
    """(w, left) of the J = 2 stencil that keeps y[n] (phase 0) and adds the
    Lagrange value at n + 1/2 through offsets -left .. right (phase 1)."""
    nodes = np.arange(-left, right + 1)
    w = np.zeros((2, nodes.shape[0]))
    w[0, left] = 1.0
    w[1] = lagrange_weights(nodes, 0.5)
    return w, left
