"""hipGraph capture of the single-signal forward (plain, power, R2R, with the
non-local stage) and of the adjoint: the launches allocate nothing (backward
after reserve_backward) and record no memset, so they can be captured once
and replayed; every replay reads the inputs' current contents and matches the
oracle and an eager call."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint, conv, post  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def ols():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_01972_amd import ols as m
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_rows(a, b):
    a = np.atleast_2d(a)
    b = np.atleast_2d(b)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def capture(fn):
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        fn(stream)  # warm-up on the capture stream
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        fn(stream)
    return graph


@pytest.mark.parametrize("kind", ["plain", "power", "real"])
def test_forward_graph_replays(ols, kind):
    print(f"graph forward {kind}", flush=True)
    Ns, K, M, N = 40000, 4, 200, 1024
    real = kind == "real"
    gen = workloads.make_real_signal_filters if real else workloads.make_signal_filters
    s, h = gen(Ns, K, M, seed=71)
    plan = ols.OLSPlan(dev(h), N=N, power=kind == "power")
    sd = dev(s)
    y = torch.empty((K, Ns), dtype=torch.float32 if kind != "plain" else torch.complex64, device="cuda")
    graph = capture(lambda st: plan.forward(sd, y=y, stream=st))
    for rep in range(3):
        s2, _ = gen(Ns, 1, 1, seed=600 + rep)
        sd.copy_(dev(s2))  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        if real:
            ref = conv.direct_conv_real(s2, h)
        else:
            ref = conv.direct_conv(s2, h)
            if kind == "power":
                ref = post.power(ref)
        assert np.all(rel_rows(y.cpu().numpy(), ref) <= TOL), rep
        got = y.clone()
        plan.forward(sd, y=y)
        torch.cuda.synchronize()
        assert torch.equal(got, y)
    plan.close()


def test_backward_graph_replays(ols):
    print("graph backward", flush=True)
    Ns, K, M, N = 30000, 3, 128, 1024
    s, h = workloads.make_signal_filters(Ns, K, M, seed=72)
    plan = ols.OLSPlan(dev(h), N=N)
    plan.reserve_backward()
    sd = dev(s)
    gd = dev(workloads.make_grad(K, Ns, seed=72))
    ds = torch.empty(Ns, dtype=torch.complex64, device="cuda")
    dh = torch.empty((K, M), dtype=torch.complex64, device="cuda")
    graph = capture(lambda st: plan.backward(sd, gd, ds=ds, dh=dh, stream=st))
    for rep in range(3):
        g2 = workloads.make_grad(K, Ns, seed=700 + rep)
        gd.copy_(dev(g2))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert rel_rows(ds.cpu().numpy(), adjoint.grad_signal(g2, h))[0] <= TOL, rep
        rh = adjoint.grad_filters(g2, s, M)
        assert np.all(rel_rows(dh.cpu().numpy(), rh) <= TOL), rep
        a, b = ds.clone(), dh.clone()
        plan.backward(sd, gd, ds=ds, dh=dh)
        torch.cuda.synchronize()
        assert torch.equal(a, ds) and torch.equal(b, dh)
    plan.close()
    sys.stdout.flush()


@pytest.mark.parametrize("kind", ["plain", "power", "real"])
def test_forward_graph_replays_rows_off_grid(ols, kind):
    """Rows off the 128-byte grid (re-aligned, >= 2^22 outputs): replays read
    the plan's delayed spectra, which an eager filter update rewrites, and
    stay right when an eager call with other row phases runs in between."""
    print(f"graph forward off-grid {kind}", flush=True)
    Ns, K, M, N = (1 << 20) + 1, 4, 64, 1024  # >= 2^22 outputs: the call re-aligns its rows
    real = kind == "real"
    gen = workloads.make_real_signal_filters if real else workloads.make_signal_filters
    s, h = gen(Ns, K, M, seed=72)
    plan = ols.OLSPlan(dev(h), N=N, power=kind == "power")
    sd = dev(s)
    dt = torch.float32 if kind != "plain" else torch.complex64
    y = torch.empty((K, Ns), dtype=dt, device="cuda")
    other = torch.empty((K * (Ns - 2) + 3,), dtype=dt, device="cuda")
    y_other = other[3:].view(K, Ns - 2)  # another length and row phase
    graph = capture(lambda st: plan.forward(sd, y=y, stream=st))
    for rep in range(3):
        _, h2 = gen(1, K, M, seed=700 + rep)
        hd = dev(h2)
        plan.update_filters(hd)
        plan.forward(sd[:Ns - 2], y=y_other)  # eager, other phases
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        if real:
            ref = conv.direct_conv_real(s, h2)
        else:
            ref = conv.direct_conv(s, h2)
            if kind == "power":
                ref = post.power(ref)
        assert np.all(rel_rows(y.cpu().numpy(), ref) <= TOL), rep
    plan.close()


def test_stencil_graph_replays(ols):
    """A plan with the non-local stage (cubic midpoint interpolation, two
    outputs per sample) captured once: every replay reads the current input
    and matches the oracle's stencil of eq. (1)."""
    print("graph forward stencil", flush=True)
    Ns, K, M, N = 30001, 3, 200, 1024
    s, h = workloads.make_signal_filters(Ns, K, M, seed=73)
    w, left = post.midpoint_interpolation_stencil(1, 2)
    plan = ols.OLSPlan(dev(h), N=N, stencil=(w, left))
    sd = dev(s)
    y = torch.empty((K, 2 * Ns), dtype=torch.complex64, device="cuda")
    graph = capture(lambda st: plan.forward(sd, y=y, stream=st))
    for rep in range(3):
        s2, _ = workloads.make_signal_filters(Ns, 1, 1, seed=800 + rep)
        sd.copy_(dev(s2))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        ref = post.conv_stencil(s2, h, w, left)
        assert np.all(rel_rows(y.cpu().numpy(), ref) <= TOL), rep
        got = y.clone()
        plan.forward(sd, y=y)
        torch.cuda.synchronize()
        assert torch.equal(got, y)
    plan.close()
