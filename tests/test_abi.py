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
