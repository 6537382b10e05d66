"""Host-side checks of the benchmark's profile record keying (no GPU): the
device-code hash ignores comments and layout but not code, a record taken on
other code or another launch shape is not reported, and the floors name the
binding one."""

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
    assert bench.profile_record("test_workload", launch)["hbm_bytes_per_launch"] == pytest.approx(123.0)
    assert bench.profile_record("test_workload", dict(launch, grid=256)) is None
    rec["kernel_hash"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.profile_record("test_workload", launch) is None
    assert bench.profile_record("other_workload", launch) is None


def test_floors_name_the_binding_one():
    alg = 8e9  # 1 ms at 8 TB/s
    assert bench.floors(alg, None) == {"hbm_ms": pytest.approx(1.0), "valu_ms": None,
                                       "valu_instr_per_launch": None, "binding": "hbm"}
    # 614.4e9 wave instructions per second: 1.2288e9 of them take 2 ms
    f = bench.floors(alg, {"valu_instr_per_launch": 1.2288e9})
    assert f["valu_ms"] == pytest.approx(2.0) and f["binding"] == "valu"
    assert bench.floors(alg, {"valu_instr_per_launch": 1e8})["binding"] == "hbm"
    # with the measured launch time: the VALU floor over it
    g = bench.floors(alg, {"valu_instr_per_launch": 1.2288e9}, kernel_ms=4.0)
    assert g["valu_frac"] == pytest.approx(g["valu_ms"] / 4.0)
    assert bench.floors(alg, None, kernel_ms=4.0)["valu_frac"] is None
