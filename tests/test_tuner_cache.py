"""Tuner cache logic on the CPU: tune() is replaced by a stub, so only the
caching, key layout and the batched chooser are exercised (no GPU)."""

import json

import pytest

pytest.importorskip("torch")
tuner = pytest.importorskip("paper_1910_01972_amd.tuner")


def test_cache_tunes_once_per_key(tmp_path, monkeypatch):
    calls = []

    def fake_tune(M, K, max_n=8192, **kw):
        calls.append((M, K, max_n))
        return {"N": 512 if max_n == 8192 else 256, "filters_per_unit": 1, "workgroups_per_cu": 2}

    monkeypatch.setattr(tuner, "tune", fake_tune)
    monkeypatch.setattr(tuner, "_arch", lambda: "gfx950")
    path = tmp_path / "c.json"
    c = tuner.TuneCache(str(path))
    assert c.best(100, 4) == 512
    assert c.best(100, 4) == 512
    assert c.batched_fft_length(100, 4) == 256           # its own key (N <= 4096)
    assert c.config(100, 4) == {"N": 512, "filters_per_unit": 1, "workgroups_per_cu": 2}
    assert calls == [(100, 4, 8192), (100, 4, 4096)]
    data = json.load(open(path))
    assert set(data) == {"gfx950|M=100|K=4|max=8192", "gfx950|M=100|K=4|max=4096"}
    # a new cache object reads the file and does not tune again
    assert tuner.TuneCache(str(path)).best(100, 4) == 512 and len(calls) == 2


def test_cache_upgrades_old_integer_entries(tmp_path, monkeypatch):
    monkeypatch.setattr(tuner, "_arch", lambda: "gfx950")
    monkeypatch.setattr(tuner, "tune", lambda M, K, max_n=8192, **kw: {"N": 1024, "filters_per_unit": 2,
                                                                      "workgroups_per_cu": 2})
    path = tmp_path / "c.json"
    path.write_text(json.dumps({"gfx950|M=64|K=8|max=8192": 2048}))
    c = tuner.TuneCache(str(path))
    assert c.config(64, 8)["N"] == 1024  # an entry without the tiling is measured again
