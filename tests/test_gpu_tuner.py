"""GPU tests of the forward-kernel tiling control and the autotuner: the
workgroup count leaves the output bit-identical (same kernel, same
per-transform arithmetic), the filters-per-unit choice (a different kernel
instance) changes it only at rounding level, invalid tilings are refused, and
the tuner's choice is cached and applied."""

import json
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conv  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ols():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01972_amd import ols as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.mark.parametrize("Ns,K,M,N,real", [(70000, 6, 100, 512, False), (90001, 5, 300, 2048, False),
                                           (50000, 4, 700, 4096, False), (60000, 3, 200, 1024, True)])
def test_tilings_agree(ols, Ns, K, M, N, real):
    print(f"tilings Ns={Ns} K={K} M={M} N={N} real={real}", flush=True)
    if real:
        s, h = workloads.make_real_signal_filters(Ns, K, M, seed=K + M)
    else:
        s, h = workloads.make_signal_filters(Ns, K, M, seed=K + M)
    plan = ols.OLSPlan(dev(h), N=N)
    ref = plan.forward(dev(s)).cpu().numpy()
    want = conv.direct_conv_real(s, h) if real else conv.direct_conv(s, h)
    assert np.all(np.linalg.norm(ref - want, axis=1) <= 1e-5 * np.linalg.norm(want, axis=1))
    from paper_1910_01972_amd.tuner import tilings
    cands = tilings(plan)
    assert (1, 1) in cands and len(cands) >= 2
    first = {}
    for nf, wpc in cands:
        plan.set_tiling(nf, wpc)
        t = plan.tiling()
        assert (t["filters_per_unit"], t["workgroups_per_cu"]) == (nf, wpc)
        assert plan.launch()["grid"] == wpc * plan.launch()["cus"]
        got = plan.forward(dev(s)).cpu().numpy()
        if nf in first:
            assert np.array_equal(got, first[nf]), (nf, wpc)   # same kernel, other grid: bit-identical
        else:
            first[nf] = got
        rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
        assert np.all(rel <= 1e-6), (nf, wpc, rel)               # other kernel instance: rounding only
    plan.close()


def test_tiling_validation(ols):
    _, h = workloads.make_signal_filters(1, 2, 50, seed=1)
    plan = ols.OLSPlan(dev(h), N=8192)
    with pytest.raises(ols.OLSError):
        plan.set_tiling(2, 0)          # two filters per unit only up to N = 4096
    with pytest.raises(ols.OLSError):
        plan.set_tiling(3, 0)
    with pytest.raises(ols.OLSError):
        plan.set_tiling(1, plan.tiling()["max_workgroups_per_cu"] + 1)
    with pytest.raises(ols.OLSError):
        plan.set_tiling(1, -1)
    plan.set_tiling(0, 0)
    plan.close()
    _, hr = workloads.make_real_signal_filters(1, 2, 50, seed=1)
    plan = ols.OLSPlan(dev(hr), N=4096)
    with pytest.raises(ols.OLSError):
        plan.set_tiling(2, 0)          # R2R: two filters per unit only up to N = 2048
    plan.close()


def test_tuner_choice_cached_and_applied(ols, tmp_path):
    from paper_1910_01972_amd import tuner
    r = tuner.tune(100, 4, Ns=1 << 18, reps=2, candidates=(256, 512, 1024))
    assert r["N"] in (256, 512, 1024) and set(r["ms"]) == {256, 512, 1024}
    assert r["filters_per_unit"] in (1, 2) and r["workgroups_per_cu"] >= 1
    assert f"{r['filters_per_unit']}x{r['workgroups_per_cu']}" in r["tiling_ms"]
    assert r["segments_per_workgroup"] > 0
    json.dumps(r)
    path = str(tmp_path / "tune.json")
    cache = tuner.TuneCache(path)
    s, h = workloads.make_signal_filters(30000, 4, 100, seed=5)
    cfg = cache.config(100, 4, Ns=1 << 18, reps=2, candidates=(256, 512))
    assert json.load(open(path))[cache.key(100, 4, 8192)] == cfg
    plan = tuner.TuneCache(path).plan(dev(h))
    assert plan.info()["N"] == cfg["N"]
    t = plan.tiling()
    assert (t["filters_per_unit"], t["workgroups_per_cu"]) == (cfg["filters_per_unit"], cfg["workgroups_per_cu"])
    got = plan.forward(dev(s)).cpu().numpy()
    want = conv.direct_conv(s, h)
    assert np.all(np.linalg.norm(got - want, axis=1) <= 1e-5 * np.linalg.norm(want, axis=1))
    plan.close()
    sys.stdout.flush()


def test_batched_with_tuned_fft_lengths(ols, tmp_path):
    """OLSBatch with the tuner choosing each item's N (cached per (M, K)):
    every item uses the cached choice and matches the oracle."""
    from paper_1910_01972_amd import tuner
    cache = tuner.TuneCache(str(tmp_path / "tune.json"))
    shapes = [(20000, 3, 40), (9000, 2, 300), (20000, 3, 40)]
    items, host = [], []
    for i, (Ns, K, M) in enumerate(shapes):
        s, h = workloads.make_signal_filters(Ns, K, M, seed=90 + i)
        items.append((dev(s), dev(h)))
        host.append((s, h))
    b = ols.OLSBatch(items, fft_length=cache.batched_fft_length)
    outs = b.run()
    torch.cuda.synchronize()
    for i, ((s, h), y) in enumerate(zip(host, outs)):
        K, M = h.shape
        assert b.item(i)["N"] == cache.best(M, K, max_n=4096) <= 4096
        want = conv.direct_conv(s, h)
        assert np.all(np.linalg.norm(y.cpu().numpy() - want, axis=1) <= 1e-5 * np.linalg.norm(want, axis=1))
    assert len(json.load(open(str(tmp_path / "tune.json")))) == 2  # one entry per distinct (M, K)
    b.close()


def test_run_config_fixed_configuration(ols):
    """tuner --run: the forward with a given N and tiling, timed; the launch
    follows the tiling (workgroups per CU x CUs)."""
    from paper_1910_01972_amd import tuner
    r = tuner.run_config(100, 6, 1 << 18, 1024, 2, 1, reps=3)
    assert r["N"] == 1024 and r["filters_per_unit"] == 2 and r["ms"] > 0
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    assert r["grid"] == cus
    # zeros: the library's configuration, reported as it ran (many short
    # filters: the cost model's N = 2048, two filters per unit)
    r = tuner.run_config(32, 24, 1 << 16, 0, 0, 0, reps=2)
    assert r["N"] == 2048 and r["filters_per_unit"] == 2 and r["workgroups_per_cu"] >= 1
