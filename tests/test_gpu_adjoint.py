"""GPU parity of the adjoint (ols_backward) and the autograd binding against
the FP64 oracle adjoint, exact finite differences and dot-product identities.

Bar: relative L2 error <= 1e-5 (per filter row for dh) against the oracle."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint, conv  # noqa: E402
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


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def rel_rows(a, b):
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


@pytest.fixture(scope="module")
def loops():
    from oracle import loops as L
    if not L.available():
        L.build()
    return L


def backward_guarded(plan, s, g, Ns):
    """ds written into a NaN-filled buffer with guard bands on both sides."""
    buf = torch.full((Ns + 2 * GUARD,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    ds = buf[GUARD:GUARD + Ns]
    _, dh = plan.backward(s, g, ds=ds)
    torch.cuda.synchronize()
    assert bool(torch.isnan(buf[:GUARD].real).all()) and bool(torch.isnan(buf[GUARD + Ns:].real).all()), \
        "guard band written"
    assert not bool(torch.isnan(ds).any()), "ds not written everywhere"
    return ds, dh


CASES = [
    # (Ns, K, M, N, hop)
    (1, 1, 1, 256, None),
    (5000, 3, 40, 256, None),
    (20000, 4, 100, 1024, None),
    (9000, 5, 513, 2048, None),
    (30000, 2, 300, 4096, 1000),
    (40000, 3, 1000, 8192, None),
    (3000, 7, 16, 512, None),
    (100001, 16, 64, 256, None),
    (65536, 32, 256, 2048, None),
]


@pytest.mark.parametrize("Ns,K,M,N,hop", CASES)
def test_backward_full(ols, Ns, K, M, N, hop):
    say(f"backward Ns={Ns} K={K} M={M} N={N}")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=Ns + 7)
    g = workloads.make_grad(K, Ns, seed=Ns + 7)
    plan = ols.OLSPlan(dev(h), N=N)
    if hop is not None:
        plan.set_hop(hop)
    buf = torch.full((Ns + 2 * GUARD,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    ds = buf[GUARD:GUARD + Ns]
    _, dh = plan.backward(dev(s), dev(g), ds=ds)
    torch.cuda.synchronize()
    assert bool(torch.isnan(buf[:GUARD].real).all()) and bool(torch.isnan(buf[GUARD + Ns:].real).all())
    ds_h = ds.cpu().numpy()
    assert not np.isnan(ds_h).any()
    assert rel(ds_h, adjoint.grad_signal(g, h)) <= TOL
    dh_h = dh.cpu().numpy()
    rh = adjoint.grad_filters(g, s, M)
    assert np.all(np.linalg.norm(dh_h - rh, axis=1) <= TOL * np.linalg.norm(rh, axis=1))
    plan.close()


def test_backward_partial_outputs_and_empty(ols):
    s, h = workloads.make_signal_filters(7000, 3, 50, seed=3)
    g = workloads.make_grad(3, 7000, seed=3)
    plan = ols.OLSPlan(dev(h), N=512)
    ds, dh = plan.backward(dev(s), dev(g), need_dh=False)
    assert dh is None and rel(ds.cpu().numpy(), adjoint.grad_signal(g, h)) <= TOL
    ds, dh = plan.backward(dev(s), dev(g), need_ds=False)
    assert ds is None and np.all(rel_rows(dh.cpu().numpy(), adjoint.grad_filters(g, s, 50)) <= TOL)
    e = torch.empty(0, dtype=torch.complex64, device="cuda")
    _, dh0 = plan.backward(e, torch.empty((3, 0), dtype=torch.complex64, device="cuda"), need_ds=False)
    torch.cuda.synchronize()
    assert torch.count_nonzero(dh0).item() == 0
    plan.close()


def test_backward_deterministic(ols):
    s, h = workloads.make_signal_filters(300000, 8, 256, seed=4)
    g = workloads.make_grad(8, 300000, seed=4)
    plan = ols.OLSPlan(dev(h), N=2048)
    plan.reserve_backward()
    sd, gd = dev(s), dev(g)
    a = plan.backward(sd, gd)
    b = plan.backward(sd, gd)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    plan.close()


def test_grad_workload_sampled_and_dot_products(ols):
    """Full-size differentiable workload (2^22 samples, 16 filters of 512
    taps, N = 4096): ds on sampled indices against eq. (1)'s adjoint, and both
    gradients through the identities <A s', g> = <s', ds>, <B h', g> = <h', dh>
    with the forward operator itself (independently checked against the
    oracle), which hold at any size."""
    wl = workloads.WORKLOADS["grad_2p22_k16_m512"]
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    g = workloads.make_grad(wl.K, wl.Ns, seed=wl.seed)
    plan = ols.OLSPlan(dev(h), N=wl.N)
    sd, gd = dev(s), dev(g)
    ds, dh = plan.backward(sd, gd)
    torch.cuda.synchronize()
    rng = np.random.default_rng(wl.seed)
    H = plan.info()["H"]
    idx = np.unique(np.concatenate([np.arange(0, 600), np.arange(wl.Ns - 2 * wl.M, wl.Ns)] +
                                   [np.arange(j * H - 3, j * H + 3) for j in rng.integers(1, wl.Ns // H, 32)] +
                                   [np.arange(st, st + 512) for st in rng.integers(0, wl.Ns - 512, 8)]))
    got = ds[torch.from_numpy(idx).cuda()].cpu().numpy()
    assert rel(got, adjoint.grad_signal_at(g, h, idx)) <= TOL
    # <B h', g> = <h', dh>
    _, h2 = workloads.make_signal_filters(1, wl.K, wl.M, seed=99)
    plan2 = ols.OLSPlan(dev(h2), N=wl.N)
    y2 = plan2.forward(sd).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y2.ravel(), g.astype(np.complex128).ravel())
    rhs = np.vdot(h2.astype(np.complex128).ravel(), dh.cpu().numpy().astype(np.complex128).ravel())
    say(f"  <B h', g> = {lhs:.6e}  <h', dh> = {rhs:.6e}")
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    # <A s', g> = <s', ds>
    s2, _ = workloads.make_signal_filters(wl.Ns, 1, 1, seed=98)
    y3 = plan.forward(dev(s2)).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y3.ravel(), g.astype(np.complex128).ravel())
    rhs = np.vdot(s2.astype(np.complex128), ds.cpu().numpy().astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    plan.close()
    plan2.close()


def test_grad_workload_full_elementwise(ols, loops):
    """The full differentiable workload (2^22 samples, 16 filters of 512 taps,
    N = 4096) on the persistent grid the library launches: every sample of ds
    and every row of dh against the float64 adjoint of eq. (1) (plain loops),
    relative L2 <= 1e-5 per row; ds written into a guarded NaN buffer."""
    wl = workloads.WORKLOADS["grad_2p22_k16_m512"]
    say(f"full adjoint {wl.name}")
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    g = workloads.make_grad(wl.K, wl.Ns, seed=wl.seed)
    plan = ols.OLSPlan(dev(h), N=wl.N)
    ds, dh = backward_guarded(plan, dev(s), dev(g), wl.Ns)
    ds_h, dh_h = ds.cpu().numpy(), dh.cpu().numpy()
    plan.close()
    r_ds = rel(ds_h, loops.grad_signal(g, h))
    r_dh = rel_rows(dh_h, loops.grad_filters(g, s, wl.M))
    say(f"  ds rel {r_ds:.3e}  dh worst row rel {r_dh.max():.3e}")
    assert r_ds <= TOL
    assert np.all(r_dh <= TOL), r_dh


@pytest.mark.parametrize("Ns,K,M,N,hop", [(1_500_001, 5, 700, 4096, 3000), (2_000_003, 3, 1500, 8192, None),
                                          (1_000_001, 7, 200, 2048, None)])
def test_backward_fills_grid_elementwise(ols, loops, Ns, K, M, N, hop):
    """Signals long enough that every persistent workgroup gets work and tiles
    are split between workgroups (odd K, a hop that is not the default):
    ds and every dh row element-wise against the float64 adjoint."""
    say(f"grid-filling backward Ns={Ns} K={K} M={M} N={N} hop={hop}")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=Ns % 1000)
    g = workloads.make_grad(K, Ns, seed=Ns % 1000)
    plan = ols.OLSPlan(dev(h), N=N)
    if hop is not None:
        plan.set_hop(hop)
    ds, dh = backward_guarded(plan, dev(s), dev(g), Ns)
    plan.close()
    assert rel(ds.cpu().numpy(), loops.grad_signal(g, h)) <= TOL
    assert np.all(rel_rows(dh.cpu().numpy(), loops.grad_filters(g, s, M)) <= TOL)


def test_finite_differences_on_slice(ols):
    """L = Re sum conj(w) y is linear in s and h, so central differences of the
    GPU forward are exact up to float32 rounding; compared with the GPU
    gradients on a 2^12-sample slice (16 filters of 512 taps, N = 4096)."""
    Ns, K, M = 1 << 12, 16, 512
    s, h = workloads.make_signal_filters(Ns, K, M, seed=55)
    w = workloads.make_grad(K, Ns, seed=55)
    plan = ols.OLSPlan(dev(h), N=4096)
    ds, dh = plan.backward(dev(s), dev(w))
    ds, dh = ds.cpu().numpy(), dh.cpu().numpy()
    wd = w.astype(np.complex128)

    def loss(s_, h_):
        plan.update_filters(dev(h_))
        y = plan.forward(dev(s_)).cpu().numpy().astype(np.complex128)
        return float(np.real(np.vdot(wd.ravel(), y.ravel())))

    eps = 1.0
    scale = np.abs(ds).max()
    for m in (0, 1, 511, 512, 2047, Ns - 1):
        for unit, part in ((1.0, 0), (1j, 1)):
            e = np.zeros(Ns, dtype=np.complex64)
            e[m] = unit * eps
            fd = (loss(s + e, h) - loss(s - e, h)) / (2 * eps)
            want = (ds[m].real, ds[m].imag)[part]
            assert abs(fd - want) <= 1e-4 * scale, (m, part, fd, want)
    scale = np.abs(dh).max()
    for r, k in ((0, 0), (3, 17), (15, M - 1)):
        for unit, part in ((1.0, 0), (1j, 1)):
            e = np.zeros((K, M), dtype=np.complex64)
            e[r, k] = unit * eps
            fd = (loss(s, h + e) - loss(s, h - e)) / (2 * eps)
            want = (dh[r, k].real, dh[r, k].imag)[part]
            assert abs(fd - want) <= 1e-4 * scale, (r, k, part, fd, want)
    plan.close()


def test_autograd_module(ols):
    from paper_1910_01972_amd.ols import OLSConv
    Ns, K, M = 20000, 4, 128
    s, h = workloads.make_signal_filters(Ns, K, M, seed=21)
    w = workloads.make_grad(K, Ns, seed=21)
    mod = OLSConv(dev(h), N=1024)
    sd = dev(s).requires_grad_(True)
    y = mod(sd)
    L = (torch.conj(dev(w)) * y).real.sum()
    L.backward()
    assert rel(sd.grad.cpu().numpy(), adjoint.grad_signal(w, h)) <= TOL
    assert rel(mod.h.grad.cpu().numpy(), adjoint.grad_filters(w, s, M)) <= TOL
    # a step on the filters changes the forward accordingly
    with torch.no_grad():
        mod.h -= 0.01 * mod.h.grad
    y2 = mod(dev(s))
    ref = conv.direct_conv(s, mod.h.detach().cpu().numpy())
    assert np.all(np.linalg.norm(y2.detach().cpu().numpy() - ref, axis=1) <= TOL * np.linalg.norm(ref, axis=1))
