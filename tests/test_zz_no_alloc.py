"""ols_backward_static -- the adjoint with its scratch in a library-static
device array, for callers that cannot allocate -- against ols_backward (the
plan-workspace entry point, itself checked against the FP64 oracle adjoint in
the adjoint tests) on the same plans and inputs.

Bar: per-row relative L2 <= 1e-5 (ds as one row, dh per filter), and
bit-identical outputs whenever the full persistent grid's scratch fits."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
GUARD = 4096


@pytest.fixture(scope="module")
def ols():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01972_amd import ols as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_rows(a, b):
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def nan_c64(shape):
    return torch.full(shape, complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")


def static_guarded(plan, sd, gd):
    """ols_backward_static into NaN-filled outputs; ds has guard bands."""
    Ns = int(sd.shape[0])
    buf = nan_c64((Ns + 2 * GUARD,))
    ds = buf[GUARD:GUARD + Ns]
    dh = nan_c64((plan.K, plan.M))
    plan.backward(sd, gd, ds=ds, dh=dh, static_scratch=True)
    torch.cuda.synchronize()
    assert bool(torch.isnan(buf[:GUARD].real).all()) and bool(torch.isnan(buf[GUARD + Ns:].real).all()), \
        "guard band written"
    assert not bool(torch.isnan(ds.real).any()) and not bool(torch.isnan(dh.real).any()), "output not written"
    return ds, dh


def compare(plan, sd, gd, exact):
    ds_r, dh_r = plan.backward(sd, gd)
    torch.cuda.synchronize()
    ds_s, dh_s = static_guarded(plan, sd, gd)
    assert np.all(rel_rows(ds_s.cpu().numpy(), ds_r.cpu().numpy()) <= TOL)
    assert np.all(rel_rows(dh_s.cpu().numpy(), dh_r.cpu().numpy()) <= TOL)
    if exact:
        assert torch.equal(ds_s, ds_r) and torch.equal(dh_s, dh_r)


def test_two_calls_second_smaller(ols):
    Ns, K, M, N = 300000, 8, 256, 2048
    say(f"static backward Ns={Ns} K={K} M={M} N={N}, then Ns=40001")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=81)
    g = workloads.make_grad(K, Ns, seed=81)
    plan = ols.OLSPlan(dev(h), N=N)
    compare(plan, dev(s), dev(g), exact=True)
    n2 = 40001
    compare(plan, dev(s[:n2]), dev(g[:, :n2]), exact=True)
    plan.close()


def test_second_plan_smaller_shapes(ols):
    say("static backward: plan (4, 700, 4096) then plan (3, 50, 512)")
    for Ns, K, M, N, seed in ((50000, 4, 700, 4096, 82), (7000, 3, 50, 512, 83)):
        s, h = workloads.make_signal_filters(Ns, K, M, seed=seed)
        g = workloads.make_grad(K, Ns, seed=seed)
        plan = ols.OLSPlan(dev(h), N=N)
        compare(plan, dev(s), dev(g), exact=True)
        plan.close()


def test_full_size_clamped_grid(ols):
    """2^22 samples, 16 filters of 512 taps, N = 4096: the full grid's scratch
    exceeds the static array, so fewer workgroups run; results agree with
    ols_backward to float rounding."""
    wl = workloads.WORKLOADS["grad_2p22_k16_m512"]
    say(f"static backward full size {wl.Ns} x {wl.K} x {wl.M}, N = {wl.N}")
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    g = workloads.make_grad(wl.K, wl.Ns, seed=wl.seed)
    plan = ols.OLSPlan(dev(h), N=wl.N)
    sd, gd = dev(s), dev(g)
    compare(plan, sd, gd, exact=False)
    # second call, smaller input, same plan
    n2 = wl.Ns // 3 + 17
    compare(plan, sd[:n2].contiguous(), gd[:, :n2].contiguous(), exact=False)
    plan.close()


def test_graph_capture_replays(ols):
    """Captured once (no allocation, no memset inside) and replayed with new
    gradients; every replay equals an eager ols_backward."""
    Ns, K, M, N = 30000, 3, 128, 1024
    say("static backward under graph capture")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=84)
    plan = ols.OLSPlan(dev(h), N=N)
    sd = dev(s)
    gd = dev(workloads.make_grad(K, Ns, seed=84))
    ds = torch.empty(Ns, dtype=torch.complex64, device="cuda")
    dh = torch.empty((K, M), dtype=torch.complex64, device="cuda")
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        plan.backward(sd, gd, ds=ds, dh=dh, stream=stream, static_scratch=True)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        plan.backward(sd, gd, ds=ds, dh=dh, stream=stream, static_scratch=True)
    for rep in range(3):
        gd.copy_(dev(workloads.make_grad(K, Ns, seed=900 + rep)))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ds_r, dh_r = plan.backward(sd, gd)
        torch.cuda.synchronize()
        assert torch.equal(ds, ds_r) and torch.equal(dh, dh_r), rep
    del graph
    plan.close()


def test_oversize_rejected_before_launch(ols):
    """One workgroup's dh partials alone (K x M complex64) exceed the static
    array: the call fails on the host with INVALID_VALUE and writes nothing."""
    from paper_1910_01972_amd._lib import OLSError
    K, M, N = 1100, 8192, 8192
    say(f"static backward oversize K={K} M={M}")
    h = torch.zeros((K, M), dtype=torch.complex64, device="cuda")
    plan = ols.OLSPlan(h, N=N)
    sd = torch.zeros(1000, dtype=torch.complex64, device="cuda")
    gd = torch.zeros((K, 1000), dtype=torch.complex64, device="cuda")
    ds = nan_c64((1000,))
    dh = nan_c64((K, M))
    with pytest.raises(OLSError) as ei:
        plan.backward(sd, gd, ds=ds, dh=dh, static_scratch=True)
    assert "OLS_ERROR_INVALID_VALUE" in str(ei.value) and "bytes" in str(ei.value)
    torch.cuda.synchronize()
    assert bool(torch.isnan(ds.real).all()) and bool(torch.isnan(dh.real).all())
    plan.close()
