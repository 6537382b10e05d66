"""Host-side checks of the benchmark's traffic record keying (no GPU): the
device-code hash ignores comments and layout but not code, and a record taken
on other code or another launch shape is not reported."""

import json
import os

import pytest

import bench


def test_code_tokens_ignore_comments_and_layout():
    a = b"int f(int x) {  // the input\n  return x + 1; /* one\n more */ }\n"
    b = b"int f(int x)\n{\n\treturn x + 1;\n}"
    assert bench._code_tokens(a) == bench._code_tokens(b)
    assert bench._code_tokens(a) != bench._code_tokens(b.replace(b"+ 1", b"+ 2"))


def test_kernel_hash_is_stable_and_short():
    h = bench.kernel_hash()
    assert h == bench.kernel_hash() and len(h) == 16


def test_traffic_record_needs_matching_code_and_launch(tmp_path, monkeypatch):
    launch = {"N": 2048, "grid": 512, "block": 256, "filters_per_unit": 2}
    rec = {"kernel_hash": bench.kernel_hash(), "launch": launch, "hbm_bytes_per_launch": 123.0}
    prof = tmp_path / "profiles"
    prof.mkdir()
    path = prof / "traffic_ols_forward_test_workload.json"
    path.write_text(json.dumps(rec))
    h = bench.kernel_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: h)
    assert bench.measured_traffic("test_workload", launch) == pytest.approx(123.0)
    assert bench.measured_traffic("test_workload", dict(launch, grid=256)) is None
    rec["kernel_hash"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.measured_traffic("test_workload", launch) is None
    assert bench.measured_traffic("other_workload", launch) is None
