"""Host emulator of the HIP kernels (libols_emu.so): the same per-lane code run
on the CPU, for tests of the kernel dataflow, indexing, LDS exchanges and
bounds without a GPU.  Not a fallback: the product path never calls it."""

from __future__ import annotations

import ctypes
import os

import numpy as np

from ._lib import EMU_PATH

_emu = None


def emu() -> ctypes.CDLL:
    global _emu
    if _emu is None:
        if not os.path.exists(EMU_PATH):
            raise ImportError(f"{EMU_PATH} is missing: build it with `python -m paper_1910_01972_amd.build`")
        L = ctypes.CDLL(EMU_PATH)
        P, I32, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
        L.ols_emu_forward.argtypes = [I32, P, I64, P, I32, I32, I32, I32, I32, P]
        L.ols_emu_forward_post.argtypes = [I32, P, I64, P, I32, I32, I32, I32, I32, I32, P]
        L.ols_emu_forward_post.restype = I32
        L.ols_emu_spectra.argtypes = [I32, P, I32, I32, P]
        L.ols_emu_lds_report.argtypes = [I32, P]
        L.ols_emu_geometry.argtypes = [I32, P]
        L.ols_emu_wave_local.argtypes = [I32, P]
        L.ols_emu_wave_local.restype = I32
        L.ols_emu_backward.argtypes = [I32, P, I64, P, P, I32, I32, I32, I32, I32, P, P]
        L.ols_emu_backward.restype = I32
        L.ols_emu_forward_stencil.argtypes = [I32, P, I64, P, I32, I32, I32, I32, I32, I32, I32, I32, I32, P, I32, P]
        L.ols_emu_forward_stencil.restype = I32
        L.ols_emu_stencil_delay.argtypes = [I32, I32, I32, I32]
        L.ols_emu_stencil_delay.restype = I32
        L.ols_emu_stencil_hop.argtypes = [I32, I32, I32]
        L.ols_emu_stencil_hop.restype = I32
        L.ols_emu_batch_geometry.argtypes = [I32, I32, P, I64, P]
        L.ols_emu_batch_geometry.restype = None
        L.ols_emu_row_shift.argtypes = [P, I64, I32, I32, I32]
        L.ols_emu_row_shift_geometry.argtypes = [P, I64, I32, I32, I32, I32, P]
        L.ols_emu_row_shift_geometry.restype = None
        L.ols_emu_row_shift.restype = I32
        L.ols_emu_cost_model.argtypes = [I32, I32, I32]
        L.ols_emu_cost_model.restype = I32
        for f in (L.ols_emu_forward, L.ols_emu_spectra, L.ols_emu_lds_report, L.ols_emu_geometry):
            f.restype = I32
        _emu = L
    return _emu


def _ptr(a: np.ndarray) -> ctypes.c_void_p:
    return ctypes.c_void_p(a.ctypes.data)


def geometry(N: int) -> dict:
    out = np.zeros(7, dtype=np.int32)
    if emu().ols_emu_geometry(N, _ptr(out)) != 0:
        raise ValueError(N)
    return dict(zip(("G", "P", "R0", "WG", "SEGS", "LDS", "TWR"), out.tolist()))


def wave_local(N: int) -> list:
    """Per exchange E = 0 .. P-2: True if every value stays in the wave that
    wrote it."""
    out = np.zeros(8, dtype=np.int32)
    if emu().ols_emu_wave_local(N, _ptr(out)) != 0:
        raise ValueError(N)
    return [bool(v) for v in out[:geometry(N)["P"] - 1]]


def lds_report(N: int) -> dict:
    out = np.zeros(8, dtype=np.int64)
    if emu().ols_emu_lds_report(N, _ptr(out)) != 0:
        raise ValueError(N)
    keys = ("worst16", "worst32", "out_of_range", "max_addr", "double_writes", "unwritten_reads", "lds_size",
            "twiddles")
    return dict(zip(keys, out.tolist()))


def spectra(h: np.ndarray, N: int) -> np.ndarray:
    h = np.ascontiguousarray(h, dtype=np.complex64)
    K, M = h.shape
    out = np.zeros((K, N), dtype=np.complex64)
    rc = emu().ols_emu_spectra(N, _ptr(h), K, M, _ptr(out))
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    return out


def forward(s: np.ndarray, h: np.ndarray, N: int, D: int, H: int, grid: int, guard: int = 4096):
    """Forward OLS through the kernel dataflow.  Signal and output are placed
    inside NaN guard bands; returns (y, s_guard_ok, y_guard_ok)."""
    h = np.ascontiguousarray(h, dtype=np.complex64)
    K, M = h.shape
    Ns = int(s.shape[0])
    nan = np.complex64(complex(np.nan, np.nan))
    sbuf = np.full(Ns + 2 * guard, nan, dtype=np.complex64)
    sbuf[guard:guard + Ns] = s
    ybuf = np.full(K * Ns + 2 * guard, nan, dtype=np.complex64)
    sp = ctypes.c_void_p(sbuf.ctypes.data + guard * 8)
    yp = ctypes.c_void_p(ybuf.ctypes.data + guard * 8)
    rc = emu().ols_emu_forward(N, sp, Ns, _ptr(h), K, M, D, H, grid, yp)
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    y = ybuf[guard:guard + K * Ns].reshape(K, Ns).copy()
    y_guard_ok = bool(np.all(np.isnan(ybuf[:guard])) and np.all(np.isnan(ybuf[guard + K * Ns:])))
    s_guard_ok = bool(np.all(np.isnan(sbuf[:guard])) and np.all(np.isnan(sbuf[guard + Ns:])))
    return y, s_guard_ok, y_guard_ok


def forward_post(s: np.ndarray, h: np.ndarray, N: int, D: int, H: int, grid: int, post: int, guard: int = 4096,
                 y_offset: int = 0):
    """Forward OLS with flags (1 derivative, 2 power, 4 R2R with float32 s, h
    and y, 8 the library's row shift for outputs off the 128-byte line grid); the
    output is complex64 [K][N_s], or float32 for power and R2R, inside NaN
    guard bands, starting y_offset elements past a 64-byte aligned address.
    Returns (y, y_guard_ok)."""
    real = bool(post & 4)
    cdt = np.float32 if real else np.complex64
    h = np.ascontiguousarray(h, dtype=cdt)
    s = np.ascontiguousarray(s, dtype=cdt)
    K, M = h.shape
    Ns = int(s.shape[0])
    dt, esz = (np.float32, 4) if post & 6 else (np.complex64, 8)
    # the signal sits between NaN bands: a read outside [0, N_s) poisons the output
    sbuf = np.full(Ns + 2 * guard, np.nan, dtype=cdt)
    sbuf[guard:guard + Ns] = s
    raw = np.full(K * Ns + 2 * guard + 64, np.nan, dtype=dt)
    lo = (-(raw.ctypes.data // esz)) % (64 // esz) + guard + y_offset  # aligned to 64 bytes, then y_offset
    ybuf = raw[lo - guard:lo + K * Ns + guard]
    rc = emu().ols_emu_forward_post(N, ctypes.c_void_p(sbuf.ctypes.data + guard * sbuf.itemsize), Ns, _ptr(h), K, M,
                                    D, H, grid, int(post), ctypes.c_void_p(ybuf.ctypes.data + guard * esz))
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    ok = bool(np.all(np.isnan(ybuf[:guard])) and np.all(np.isnan(ybuf[guard + K * Ns:])))
    return ybuf[guard:guard + K * Ns].reshape(K, Ns).copy(), ok


def row_shift_geometry(y_addr: int, Ns: int, N: int, D: int, H: int, el: int) -> dict:
    """The single-signal forward's hop and row-shift mask for a call."""
    out = (ctypes.c_int32 * 2)()
    emu().ols_emu_row_shift_geometry(ctypes.c_void_p(y_addr), Ns, N, D, H, el, out)
    return {"H": out[0], "mask": out[1]}


def stencil_delay(N: int, Meff: int, left: int, right: int) -> int:
    """First kept position of a plan with a stencil (hop at most N - D - right)."""
    return int(emu().ols_emu_stencil_delay(N, Meff, left, right))


def stencil_hop(N: int, D: int, right: int) -> int:
    """Default hop of a plan with a stencil."""
    return int(emu().ols_emu_stencil_hop(N, D, right))


def forward_stencil(s: np.ndarray, h: np.ndarray, N: int, D: int, H: int, grid: int, post: int, weights, left: int,
                    guard: int = 4096, packed: bool = True):
    """forward_post followed by the non-local stencil stage: rows of J * N_s
    outputs inside NaN guard bands (packed=False: the per-phase store form
    for every J).  Returns (y, y_guard_ok)."""
    w = np.ascontiguousarray(np.atleast_2d(np.asarray(weights, dtype=np.float32)))
    J, T = w.shape
    real = bool(post & 4)
    cdt = np.float32 if real else np.complex64
    h = np.ascontiguousarray(h, dtype=cdt)
    s = np.ascontiguousarray(s, dtype=cdt)
    K, M = h.shape
    Ns = int(s.shape[0])
    dt, esz = (np.float32, 4) if post & 6 else (np.complex64, 8)
    sbuf = np.full(Ns + 2 * guard, np.nan, dtype=cdt)
    sbuf[guard:guard + Ns] = s
    n_out = K * J * Ns
    ybuf = np.full(n_out + 2 * guard, np.nan, dtype=dt)
    rc = emu().ols_emu_forward_stencil(N, ctypes.c_void_p(sbuf.ctypes.data + guard * sbuf.itemsize), Ns, _ptr(h), K,
                                       M, D, H, grid, int(post), J, int(left), T - 1 - int(left), _ptr(w),
                                       int(bool(packed)), ctypes.c_void_p(ybuf.ctypes.data + guard * esz))
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    ok = bool(np.all(np.isnan(ybuf[:guard])) and np.all(np.isnan(ybuf[guard + n_out:])))
    return ybuf[guard:guard + n_out].reshape(K, J * Ns).copy(), ok


def backward(s: np.ndarray, gy: np.ndarray, h: np.ndarray, N: int, D: int, H: int, grid: int, guard: int = 4096):
    """Adjoint through the kernel dataflow; ds is NaN-prefilled inside NaN
    guard bands.  Returns (ds, dh, ds_guard_ok)."""
    h = np.ascontiguousarray(h, dtype=np.complex64)
    gy = np.ascontiguousarray(gy, dtype=np.complex64)
    s = np.ascontiguousarray(s, dtype=np.complex64)
    K, M = h.shape
    Ns = int(s.shape[0])
    nan = np.complex64(complex(np.nan, np.nan))
    dsbuf = np.full(Ns + 2 * guard, nan, dtype=np.complex64)
    dh = np.full((K, M), nan, dtype=np.complex64)
    rc = emu().ols_emu_backward(N, _ptr(s), Ns, _ptr(gy), _ptr(h), K, M, D, H, grid,
                                ctypes.c_void_p(dsbuf.ctypes.data + guard * 8), _ptr(dh))
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    ok = bool(np.all(np.isnan(dsbuf[:guard])) and np.all(np.isnan(dsbuf[guard + Ns:])))
    return dsbuf[guard:guard + Ns].copy(), dh, ok


def batch_geometry(N: int, M: int, y_addr: int, Ns: int) -> dict:
    """The batched plan's D, H and row-shift choice for an item (the setup
    kernel's rule)."""
    out = (ctypes.c_int32 * 3)()
    emu().ols_emu_batch_geometry(N, M, ctypes.c_void_p(y_addr), Ns, out)
    return {"D": out[0], "H": out[1], "mask": out[2]}


def row_shift(y_addr: int, Ns: int, D: int, r: int, mask: int) -> int:
    return int(emu().ols_emu_row_shift(ctypes.c_void_p(y_addr), Ns, D, r, mask))


def batched(items, grid: int):
    """items: list of dicts with s (complex64 [N_s]), h (complex64 [K][M]), N,
    D, H (H = 0: the library's geometry, including the row shift of outputs
    off the 128-byte line grid) and optionally y_offset (complex elements past a
    64-byte aligned address).  Returns the list of outputs y_i [K_i][N_i_s]
    (NaN-prefilled, so an unwritten output stays NaN)."""
    L = emu()
    L.ols_emu_batched.restype = ctypes.c_int
    n = len(items)
    keep = []
    S = (ctypes.c_void_p * n)()
    Y = (ctypes.c_void_p * n)()
    Hp = (ctypes.c_void_p * n)()
    Ns = (ctypes.c_int64 * n)()
    K = (ctypes.c_int * n)()
    M = (ctypes.c_int * n)()
    Nn = (ctypes.c_int * n)()
    D = (ctypes.c_int * n)()
    Hh = (ctypes.c_int * n)()
    outs = []
    for i, it in enumerate(items):
        s = np.ascontiguousarray(it["s"], dtype=np.complex64)
        h = np.ascontiguousarray(it["h"], dtype=np.complex64)
        n_y = h.shape[0] * s.shape[0]
        off = int(it.get("y_offset", 0))
        raw = np.full(n_y + off + 8, np.complex64(complex(np.nan, np.nan)), dtype=np.complex64)
        base = (-(raw.ctypes.data // 8)) % 8  # elements to the next 64-byte boundary
        y = raw[base + off:base + off + n_y].reshape(h.shape[0], s.shape[0])
        keep += [s, h, raw]
        outs.append(y)
        S[i], Y[i], Hp[i] = s.ctypes.data, y.ctypes.data, h.ctypes.data
        Ns[i], K[i], M[i] = s.shape[0], h.shape[0], h.shape[1]
        Nn[i], D[i], Hh[i] = it["N"], it["D"], it["H"]
    rc = L.ols_emu_batched(n, S, Y, Ns, Hp, K, M, Nn, D, Hh, grid)
    if rc != 0:
        raise RuntimeError(f"emulator returned {rc}")
    return outs


def cost_model(K: int, M: int, max_n: int = 8192) -> int:
    """The library's FFT-length choice for N = 0 (host code of the C library)."""
    return int(emu().ols_emu_cost_model(int(K), int(M), int(max_n)))
