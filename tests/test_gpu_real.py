"""GPU parity of the real-to-real (R2R) path: two real segments per complex
transform, against the oracle's real-data eq. (1) (bar: relative L2 error
<= 1e-5 per filter row)."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conv, post  # noqa: E402
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
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-300)


def reference(s, h, derivative=False, power=False):
    y = conv.direct_conv_real(s, h)
    if derivative:
        y = post.derivative(y).real
    if power:
        y = y * y
    return y


CASES = [
    # (Ns, K, M, N, derivative, power)
    (1, 1, 1, 256, False, False),
    (255, 2, 3, 256, False, False),
    (3001, 4, 40, 256, False, False),        # odd segment count
    (9000, 4, 100, 1024, False, True),
    (20000, 5, 513, 2048, False, False),
    (20000, 6, 300, 2048, True, False),
    (65536, 32, 256, 2048, False, False),
    (65536, 7, 256, 2048, False, False),     # odd K: one filter per unit
    (30000, 3, 1000, 4096, False, False),
    (40000, 8, 1500, 4096, False, False),
    (40000, 2, 700, 8192, True, True),
    (100001, 16, 64, 512, False, False),
    # rows off the 64-byte grid (N_s not a multiple of 16) on whole-wave transforms
    (20001, 3, 300, 2048, False, False),
    (30005, 4, 1000, 4096, False, True),
    (40003, 2, 700, 8192, False, False),
]


@pytest.mark.parametrize("Ns,K,M,N,derivative,power", CASES)
def test_real_full(ols, Ns, K, M, N, derivative, power):
    say(f"r2r Ns={Ns} K={K} M={M} N={N} derivative={derivative} power={power}")
    s, h = workloads.make_real_signal_filters(Ns, K, M, seed=Ns + 3 * K)
    plan = ols.OLSPlan(dev(h), N=N, derivative=derivative, power=power)
    sbuf = torch.full((Ns + 2 * GUARD,), float("nan"), dtype=torch.float32, device="cuda")
    sbuf[GUARD:GUARD + Ns] = dev(s)
    buf = torch.full((K * Ns + 2 * GUARD,), float("nan"), dtype=torch.float32, device="cuda")
    y = buf[GUARD:GUARD + K * Ns].view(K, Ns)
    plan.forward(sbuf[GUARD:GUARD + Ns], y=y)
    torch.cuda.synchronize()
    b = buf.cpu().numpy()
    assert np.isnan(b[:GUARD]).all() and np.isnan(b[GUARD + K * Ns:]).all(), "guard band written"
    got = y.cpu().numpy()
    assert not np.isnan(got).any(), "unwritten output or a read outside the signal"
    r = rel_rows(got, reference(s, h, derivative, power))
    assert np.all(r <= TOL), r
    plan.close()


def test_real_hop_invariance_and_update(ols):
    Ns, K, M = 12000, 3, 100
    s, h = workloads.make_real_signal_filters(Ns, K, M, seed=81)
    ref = reference(s, h)
    for N, H in ((256, 157), (256, 1), (512, 300), (1024, 925)):
        plan = ols.OLSPlan(dev(h), N=N)
        plan.set_hop(H)
        got = plan.forward(dev(s)).cpu().numpy()
        assert np.all(rel_rows(got, ref) <= TOL), (N, H)
        plan.close()
    plan = ols.OLSPlan(dev(h), N=1024)
    _, h2 = workloads.make_real_signal_filters(1, K, M, seed=82)
    plan.update_filters(dev(h2))
    got = plan.forward(dev(s)).cpu().numpy()
    assert np.all(rel_rows(got, reference(s, h2)) <= TOL)
    with pytest.raises(TypeError):
        plan.forward(dev(s.astype(np.complex64)))
    with pytest.raises(TypeError):
        plan.backward(dev(s), torch.zeros((K, Ns), device="cuda"))
    plan.close()


def test_real_full_size_sampled(ols):
    """2^23 real samples, 32 real filters of 256 taps, N = 2048: sampled
    outputs against eq. (1) evaluated one by one, including pair and segment
    edges."""
    wl = workloads.WORKLOADS["filter_bank_real_2p23_k32_m256"]
    s, h = workloads.make_real_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    plan = ols.OLSPlan(dev(h), N=wl.N)
    H = plan.info()["H"]
    rng = np.random.default_rng(91)
    idx = np.unique(np.concatenate([np.arange(0, 700), np.arange(wl.Ns - 300, wl.Ns)] +
                                   [np.arange(j * H - 2, j * H + 2) for j in rng.integers(1, wl.Ns // H, 64)] +
                                   [rng.integers(0, wl.Ns, 2000)]))
    y = plan.forward(dev(s))
    got = y[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    ref = conv.direct_conv_real_at(s, h, idx)
    assert np.all(rel_rows(got, ref) <= TOL), rel_rows(got, ref)
    # a contiguous block spanning many segment pairs, element by element
    blk = slice(1 << 20, (1 << 20) + 50000)
    ref_blk = conv.direct_conv_real(s[(1 << 20) - wl.M + 1:(1 << 20) + 50000], h)[:, wl.M - 1:]
    assert np.all(rel_rows(y[:, blk].cpu().numpy(), ref_blk) <= TOL)
    plan.close()
