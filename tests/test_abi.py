"""C-ABI library: loads, exports every symbol include/ols.h declares, and
validates arguments on the host before touching the GPU (no compute here)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ols.h")

_lib = pytest.importorskip("paper_1910_01972_amd._lib")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ols_[a-z_]+)\s*\(", text)))


def test_header_parses():
    names = declared_symbols()
    for want in ("ols_plan", "ols_forward", "ols_plan_destroy", "ols_status_string"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_symbols() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_header():
    assert set(declared_symbols()) <= set(_lib.SIGNATURES), set(declared_symbols()) - set(_lib.SIGNATURES)


def test_status_strings():
    L = _lib.lib()
    assert L.ols_status_string(0) == b"success"
    assert L.ols_status_string(2) == b"unsupported"
    assert L.ols_status_string(99) == b"unknown status"


def _plan(h, K, M, N):
    p = ctypes.c_void_p()
    st = _lib.lib().ols_plan(ctypes.byref(p), h, K, M, N, None)
    return st, p


@pytest.mark.parametrize("K,M,N,want", [
    (0, 4, 256, 1),      # K < 1
    (2, 0, 256, 1),      # M < 1
    (2, 300, 256, 1),    # M > N
    (2, 4, 300, 2),      # N not a power of two
    (2, 4, 128, 2),      # N below range
    (2, 4, 16384, 2),    # N above range
    (2, 9000, 0, 1),     # auto N impossible
])
def test_plan_validation_before_any_gpu_call(K, M, N, want):
    buf = ctypes.create_string_buffer(64)
    st, p = _plan(ctypes.cast(buf, ctypes.c_void_p), K, M, N)
    assert st == want
    assert not p.value
    assert _lib.lib().ols_last_error() != b""


def test_null_arguments():
    L = _lib.lib()
    assert L.ols_plan(None, None, 1, 1, 256, None) == 1
    p = ctypes.c_void_p()
    assert L.ols_plan(ctypes.byref(p), None, 1, 1, 256, None) == 1
    assert L.ols_forward(None, None, 10, None, None) == 1
    assert L.ols_plan_set_hop(None, 5) == 1
    assert L.ols_plan_get_info(None, None, None, None, None, None) == 1
    assert L.ols_plan_destroy(None) == 0
    assert L.ols_calibration_copy(None, None, 16, None) == 1


def test_misaligned_filter_pointer_rejected():
    buf = ctypes.create_string_buffer(64)
    st, _ = _plan(ctypes.c_void_p(ctypes.addressof(buf) + 4), 1, 4, 256)
    assert st == 1


def test_batched_workspace_size_host_only():
    """ols_batched_workspace_size validates items and sizes the batch on the
    host alone (fake, never dereferenced pointers; no GPU call)."""
    L = _lib.lib()
    BI = _lib.BatchItem

    def size(items):
        arr = (BI * len(items))(*items)
        out = ctypes.c_size_t()
        rc = L.ols_batched_workspace_size(arr, len(items), ctypes.byref(out))
        return rc, out.value

    base = 1 << 40
    a = BI(base, 1000, base + (1 << 30), 3, 100, 512, base + (2 << 30))
    b = BI(base + (3 << 30), 5000, base + (4 << 30), 2, 30, 256, base + (5 << 30))
    rc, n512 = size([a, b])
    assert rc == 0 and n512 > 0
    a256 = BI(base, 1000, base + (1 << 30), 3, 100, 256, base + (2 << 30))
    rc, n256 = size([a256, b])
    assert rc == 0 and n512 - n256 == 3 * (512 - 256) * 8  # spectra K x N complex64
    bad = BI(base, 1000, base + (1 << 30), 3, 100, 8192, base + (2 << 30))   # batched N <= 4096
    assert size([bad])[0] == 2
    overlap = BI(base, 1000, base + (1 << 30), 3, 100, 512, base + 8)          # y overlaps s
    assert size([overlap])[0] == 1
    assert L.ols_batched_workspace_size(None, 1, None) == 1


def test_batched_device_call_host_checks():
    """ols_batched rejects NULL or misaligned pointers, n < 1 and a workspace
    too small for n items on the host, before anything is enqueued (the fake
    pointers are never dereferenced)."""
    L = _lib.lib()
    items = ctypes.c_void_p(1 << 40)
    ws = ctypes.c_void_p(1 << 41)
    big = 1 << 30
    assert L.ols_batched(None, 1, ws, big, None) == 1
    assert L.ols_batched(items, 0, ws, big, None) == 1
    assert L.ols_batched(ctypes.c_void_p((1 << 40) + 4), 1, ws, big, None) == 1
    assert L.ols_batched(items, 1, None, big, None) == 1
    assert L.ols_batched(items, 1, ctypes.c_void_p((1 << 41) + 128), big, None) == 1
    assert L.ols_batched(items, 1000, ws, 4096, None) == 1
    assert b"workspace" in L.ols_last_error()
    assert L.ols_batched_status(None, None, None, None) == 1


def test_batched_workspace_grows_with_items():
    """Workspace bytes: fixed parts grow with the item count, spectra with K x N."""
    L = _lib.lib()
    BI = _lib.BatchItem
    base = 1 << 40

    def size(n):
        arr = (BI * n)(*[BI(base + (2 * i) * (1 << 30), 1000, base + (2 * i + 1) * (1 << 30), 1, 16, 256,
                            base + (1 << 38) + i * (1 << 30)) for i in range(n)])
        out = ctypes.c_size_t()
        assert L.ols_batched_workspace_size(arr, n, ctypes.byref(out)) == 0
        return out.value

    s1, s2 = size(1), size(2)
    assert s2 - s1 >= 256 * 8 and s1 % 256 == 0


def test_binding_imports_and_named_stencils():
    """The Python binding imports without a GPU, and its named stencils are the
    backward difference and the four-point Lagrange midpoint interpolation."""
    import numpy as np
    from oracle import post
    from paper_1910_01972_amd import ols

    w, left = ols.DIFFERENCE_STENCIL
    assert left == 1 and np.allclose(w, [[-1.0, 1.0]])
    w, left = ols.MIDPOINT_CUBIC_STENCIL
    ow, oleft = post.midpoint_interpolation_stencil(1, 2)
    assert left == oleft and np.allclose(w, ow, rtol=0, atol=1e-15)
