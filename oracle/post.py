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

Both are written by their definitions on top of ``conv.direct_conv``.
"""

from __future__ import annotations

import numpy as np

from . import conv

__all__ = ["power", "derivative", "conv_power", "conv_derivative", "derivative_at"]


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
