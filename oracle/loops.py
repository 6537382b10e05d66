"""Oracle (test infrastructure only): ctypes access to ``adjoint_loops.c``, the
adjoint of eq. (1) -- and eq. (1) itself -- as plain float64 loops in C.

Same definitions as ``adjoint.grad_signal`` / ``adjoint.grad_filters`` and
``conv.direct_conv``; compiled code only so that full-size problems (about
3e10 complex multiply-adds) finish in seconds.  ``build()`` compiles the
library in place with gcc; the functions raise if it is missing.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

__all__ = ["build", "available", "grad_signal", "grad_filters", "direct_conv"]

_DIR = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_DIR, "adjoint_loops.c")
_LIB = os.path.join(_DIR, "liboracle_loops.so")
_lib = None


def build() -> str:
    """Compile adjoint_loops.c with gcc (OpenMP, -O2, no fast-math)."""
    tmp = _LIB + ".tmp"
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC], check=True)
    os.replace(tmp, _LIB)
    return _LIB


def available() -> bool:
    return os.path.exists(_LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise ImportError(f"{_LIB} is missing: run oracle.loops.build()")
        L = ctypes.CDLL(_LIB)
        P, I = ctypes.c_void_p, ctypes.c_int64
        L.oracle_grad_signal.argtypes = [P, I, I, P, I, P]
        L.oracle_grad_filters.argtypes = [P, I, I, P, I, P]
        L.oracle_direct_conv.argtypes = [P, I, P, I, I, P]
        for f in (L.oracle_grad_signal, L.oracle_grad_filters, L.oracle_direct_conv):
            f.restype = None
        _lib = L
    return _lib


def _c128(a, ndim):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128))
    if a.ndim != ndim:
        raise ValueError(f"expected {ndim} dimension(s), got {a.ndim}")
    return a


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


def grad_signal(g, h) -> np.ndarray:
    """ds[m] = sum_r sum_k conj(h_r[k]) g_r[m+k] (g_r[n] = 0 for n >= N_s)."""
    g, h = _c128(g, 2), _c128(h, 2)
    K, Ns = g.shape
    if h.shape[0] != K:
        raise ValueError("g and h disagree on K")
    ds = np.empty(Ns, dtype=np.complex128)
    if Ns:
        _load().oracle_grad_signal(_p(g), K, Ns, _p(h), h.shape[1], _p(ds))
    return ds


def grad_filters(g, s, M: int) -> np.ndarray:
    """dh_r[k] = sum_n conj(s[n-k]) g_r[n] (s[m] = 0 for m < 0), k < M."""
    g, s = _c128(g, 2), _c128(s, 1)
    K, Ns = g.shape
    if s.shape[0] != Ns:
        raise ValueError("g and s disagree on N_s")
    dh = np.zeros((K, M), dtype=np.complex128)
    if Ns:
        _load().oracle_grad_filters(_p(g), K, Ns, _p(s), M, _p(dh))
    return dh


def direct_conv(s, h) -> np.ndarray:
    """eq. (1): y_r[n] = sum_k h_r[k] s[n-k], zero history, n < N_s."""
    s, h = _c128(s, 1), _c128(h, 2)
    K, M = h.shape
    Ns = s.shape[0]
    y = np.zeros((K, Ns), dtype=np.complex128)
    if Ns:
        _load().oracle_direct_conv(_p(s), Ns, _p(h), K, M, _p(y))
    return y
