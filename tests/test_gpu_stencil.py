"""GPU parity of the non-local post-processing stage (sec. 4: outputs combined
with their neighbours, e.g. the numerical derivative or interpolation): each
segment's outputs staged in LDS and combined by a stencil with J outputs per
sample, against the oracle's stencil of eq. (1) and its tail (bar: relative
L2 error <= 1e-5 per filter row)."""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conv, post  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
GUARD = 4096

_RNG_W = np.random.default_rng(2025)
STENCILS = {
    "difference": (np.array([[-1.0, 1.0]]), 1),
    "central": (np.array([[-0.5, 0.0, 0.5]]), 1),
    "midpoint_cubic": post.midpoint_interpolation_stencil(1, 2),
    "midpoint_linear": post.midpoint_interpolation_stencil(0, 1),
    "wide3": (_RNG_W.uniform(-1, 1, (3, 6)), 2),    # J = 3, taps -2 .. 3
    "ahead4": (_RNG_W.uniform(-1, 1, (4, 8)), 0),   # J = 4, taps 0 .. 7
    "behind": (_RNG_W.uniform(-1, 1, (2, 8)), 7),   # taps -7 .. 0
}


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


def reference(s, h, flags, w, left):
    """Oracle: derivative (as the filter followed by [1, -1]) first, then the
    stencil of eq. (1) and its tail, then the power."""
    real = bool(flags & 4)
    hh = h.astype(np.float64 if real else np.complex128)
    if flags & 1:
        hh = np.concatenate([hh, np.zeros((h.shape[0], 1), hh.dtype)], axis=1)
        hh[:, 1:] -= h
    ref = post.conv_stencil_real(s, hh, w, left) if real else post.conv_stencil(s, hh, w, left)
    if flags & 2:
        ref = ref * ref if real else post.power(ref)
    return ref


def make_plan(ols, h, N, flags, stencil):
    return ols.OLSPlan(dev(h), N=N, derivative=bool(flags & 1), power=bool(flags & 2), stencil=stencil)


def run_guarded(plan, s, K, cols, float_out, offset=0):
    """forward into a NaN-filled buffer with guard bands (y starting `offset`
    elements past an aligned address); returns (y, bands intact)."""
    dt = torch.float32 if float_out else torch.complex64
    fill = float("nan") if float_out else complex(float("nan"), float("nan"))
    buf = torch.full((K * cols + 2 * GUARD + offset,), fill, dtype=dt, device="cuda")
    lo = GUARD + offset
    y = buf[lo:lo + K * cols].view(K, cols)
    plan.forward(dev(s), y=y)
    torch.cuda.synchronize()
    b = buf.cpu().numpy()
    return y.cpu().numpy(), bool(np.isnan(b[:lo]).all() and np.isnan(b[lo + K * cols:]).all())


CASES = [
    # (Ns, K, M, N, flags, stencil); flags: 1 derivative, 2 power, 4 R2R
    (1, 1, 1, 256, 0, "midpoint_cubic"),
    (2, 2, 5, 256, 0, "ahead4"),                # every tap past the sample reads the tail
    (200, 2, 3, 256, 0, "ahead4"),              # fewer samples than one segment
    (5001, 3, 40, 256, 0, "wide3"),
    (5001, 3, 40, 256, 2, "midpoint_cubic"),
    (7000, 2, 248, 256, 0, "difference"),       # M - 1 + left + right = N - 8
    (9000, 3, 64, 512, 1, "central"),
    (20000, 4, 100, 1024, 0, "behind"),
    (20003, 3, 100, 1024, 2, "midpoint_cubic"),  # rows off the 64-byte grid
    (65536, 8, 256, 2048, 0, "midpoint_cubic"),
    (65536, 9, 513, 2048, 0, "difference"),     # odd K: padded last filter group
    (30001, 3, 700, 2048, 1 | 2, "wide3"),
    (40000, 4, 1000, 4096, 0, "ahead4"),
    (40005, 3, 1000, 4096, 2, "midpoint_linear"),
    (50000, 2, 2000, 8192, 0, "midpoint_cubic"),
    (50001, 2, 8185, 8192, 0, "difference"),    # hop 1
    # R2R: two real segments per transform, each with its own stencil outputs
    (1, 2, 3, 256, 4, "midpoint_cubic"),        # one real sample: the pair's second segment is empty
    (3, 1, 2, 256, 4 | 2, "behind"),            # all taps before the sample: zero history
    (3001, 3, 40, 256, 4, "midpoint_cubic"),
    (20000, 4, 100, 1024, 4 | 2, "wide3"),
    (65536, 6, 256, 2048, 4, "midpoint_cubic"),
    (40001, 3, 1000, 4096, 4 | 1, "central"),
    (50000, 2, 2000, 8192, 4, "behind"),
]


@pytest.mark.parametrize("Ns,K,M,N,flags,name", CASES)
def test_stencil_full(ols, Ns, K, M, N, flags, name):
    say(f"stencil Ns={Ns} K={K} M={M} N={N} flags={flags} stencil={name}")
    w, left = STENCILS[name]
    real = bool(flags & 4)
    if real:
        s, h = workloads.make_real_signal_filters(Ns, K, M, seed=Ns + K)
    else:
        s, h = workloads.make_signal_filters(Ns, K, M, seed=Ns + K)
    plan = make_plan(ols, h, N, flags, (w, left))
    J = w.shape[0]
    got, bands = run_guarded(plan, s, K, J * Ns, real or bool(flags & 2))
    assert bands, "guard band written"
    assert not np.isnan(got).any(), "an output was not written"
    r = rel_rows(got, reference(s, h, flags, w, left))
    assert np.all(r <= TOL), r
    plan.close()


@pytest.mark.parametrize("N,flags,name", [(1024, 0, "midpoint_cubic"), (2048, 0, "midpoint_cubic"),
                                          (512, 2, "midpoint_linear"), (4096, 4, "midpoint_cubic"),
                                          (2048, 0, "central")])
def test_stencil_unaligned_output(ols, N, flags, name):
    """y not aligned to the J phases of a sample (or to a float pair): the
    per-phase store form, same results."""
    Ns, K, M = 30001, 3, 200
    w, left = STENCILS[name]
    real = bool(flags & 4)
    mk = workloads.make_real_signal_filters if real else workloads.make_signal_filters
    s, h = mk(Ns, K, M, seed=N + 7)
    plan = make_plan(ols, h, N, flags, (w, left))
    J = w.shape[0]
    say(f"stencil unaligned N={N} flags={flags} stencil={name}")
    got, bands = run_guarded(plan, s, K, J * Ns, real or bool(flags & 2), offset=1)
    assert bands and not np.isnan(got).any()
    assert np.all(rel_rows(got, reference(s, h, flags, w, left)) <= TOL)
    plan.close()


def test_stencil_difference_equals_folded_derivative(ols):
    """The backward difference computed from neighbours in LDS and the one
    folded into the filter spectra are the same operation (sec. 4)."""
    Ns, K, M, N = 70001, 5, 300, 2048
    s, h = workloads.make_signal_filters(Ns, K, M, seed=81)
    ref = post.conv_derivative(s, h)
    staged = make_plan(ols, h, N, 0, STENCILS["difference"])
    folded = ols.OLSPlan(dev(h), N=N, derivative=True)
    a = staged.forward(dev(s)).cpu().numpy()
    b = folded.forward(dev(s)).cpu().numpy()
    assert np.all(rel_rows(a, ref) <= TOL) and np.all(rel_rows(b, ref) <= TOL)
    assert np.all(rel_rows(a, b) <= 2 * TOL)
    staged.close()
    folded.close()


def test_stencil_hop_tiling_and_removal(ols):
    """Every hop the reach allows and every tiling give the oracle's result;
    removing the stencil restores the plain convolution."""
    Ns, K, M, N = 30000, 4, 200, 2048
    w, left = STENCILS["wide3"]
    right = w.shape[1] - 1 - left
    s, h = workloads.make_signal_filters(Ns, K, M, seed=82)
    ref = reference(s, h, 0, w, left)
    plan = make_plan(ols, h, N, 0, (w, left))
    info = plan.info()
    assert info["D"] >= M - 1 + left and info["D"] + info["H"] + right <= N
    assert info["H"] % 16 == 0 and N - info["D"] - right - info["H"] < 16
    Hmax = N - (M - 1 + left) - right
    with pytest.raises(ols.OLSError):
        plan.set_hop(Hmax + 1)
    for H in (Hmax, 1000, 257):
        plan.set_hop(H)
        say(f"stencil hop {H}")
        assert np.all(rel_rows(plan.forward(dev(s)).cpu().numpy(), ref) <= TOL), H
    plan.set_hop(0)
    for nf, wpc in ((1, 0), (2, 0), (2, 1), (1, 1)):
        plan.set_tiling(nf, wpc)
        say(f"stencil tiling nf={nf} wpc={wpc}")
        assert np.all(rel_rows(plan.forward(dev(s)).cpu().numpy(), ref) <= TOL), (nf, wpc)
    plan.set_stencil(None)
    y = plan.forward(dev(s))
    assert tuple(y.shape) == (K, Ns)
    assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s, h)) <= TOL)
    plan.close()


def test_stencil_argument_errors(ols):
    from paper_1910_01972_amd._lib import lib
    s, h = workloads.make_signal_filters(3000, 2, 30, seed=83)
    plan = ols.OLSPlan(dev(h), N=256)
    raw = lib().ols_plan_set_stencil
    w = (ctypes.c_float * 32)(*([0.25] * 32))
    OK = 0
    assert raw(plan.handle, 5, 0, 0, w) != OK          # more than 4 phases
    assert raw(plan.handle, 1, 4, 4, w) != OK          # 9 taps
    assert raw(plan.handle, 1, -1, 1, w) != OK         # negative reach
    assert raw(plan.handle, 2, 1, 2, None) != OK       # no weights
    assert plan.info()["H"] == 256 - 32               # a refused call changes nothing
    long_h = workloads.make_signal_filters(1, 1, 250, seed=84)[1]
    p2 = ols.OLSPlan(dev(long_h), N=256)
    assert raw(p2.handle, 1, 3, 4, w) != OK            # M - 1 + 7 > N - 1
    assert raw(p2.handle, 1, 3, 3, w) == OK            # M - 1 + 6 = N - 1: hop 1
    assert p2.info()["H"] == 1
    p2.close()
    plan.set_stencil(*STENCILS["midpoint_cubic"])
    with pytest.raises(ValueError):
        plan.forward(dev(s), y=torch.empty((2, 3000), dtype=torch.complex64, device="cuda"))
    with pytest.raises(ols.OLSError):
        plan.backward(dev(s), dev(workloads.make_grad(2, 3000, seed=83)))
    plan.close()


def test_stencil_empty_signal(ols):
    """N_s = 0 through the C ABI on a stencil plan: a successful no-op that
    writes nothing (a sentinel buffer stays as it was)."""
    from paper_1910_01972_amd._lib import lib
    say("stencil empty signal")
    w, left = STENCILS["midpoint_cubic"]
    _, h = workloads.make_signal_filters(1, 2, 16, seed=85)
    plan = ols.OLSPlan(dev(h), N=256, stencil=(w, left))
    s = torch.zeros(8, dtype=torch.complex64, device="cuda")
    y = torch.full((64,), complex(3.0, -1.0), dtype=torch.complex64, device="cuda")
    P = ctypes.c_void_p
    assert lib().ols_forward(plan.handle, P(s.data_ptr()), 0, P(y.data_ptr()), None) == 0
    torch.cuda.synchronize()
    assert bool((y == complex(3.0, -1.0)).all()), "an empty call wrote outputs"
    plan.close()


def test_stencil_full_size(ols):
    """The 2^23-sample, 32-filter, 256-tap filter bank at N = 2048 with the
    cubic midpoint interpolation (2^24 outputs per filter, 4 GiB), and its
    power: every output written (NaN prefill), sampled outputs against the
    oracle evaluated one by one, including segment edges and the tail."""
    wl = workloads.WORKLOADS["filter_bank_2p23_k32_m256"]
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    sd = dev(s)
    w, left = STENCILS["midpoint_cubic"]
    rng = np.random.default_rng(85)
    for power in (False, True):
        say(f"stencil full size power={power}")
        plan = make_plan(ols, h, wl.N, 2 if power else 0, (w, left))
        H = plan.info()["H"]
        cols = 2 * wl.Ns
        dt = torch.float32 if power else torch.complex64
        y = torch.full((wl.K, cols), float("nan"), dtype=dt, device="cuda")
        plan.forward(sd, y=y)
        torch.cuda.synchronize()
        assert not bool(torch.isnan(y).any()), "an output was not written"
        n = np.unique(np.concatenate([np.arange(0, 400), np.arange(wl.Ns - 300, wl.Ns)] +
                                     [np.arange(j * H - 3, j * H + 3) for j in rng.integers(1, wl.Ns // H, 64)] +
                                     [rng.integers(0, wl.Ns, 1500)]))
        idx = np.unique(np.concatenate([2 * n, 2 * n + 1]))
        got = y[:, torch.from_numpy(idx).cuda()].cpu().numpy()
        del y
        ref = post.stencil_at(s, h, w, left, idx)
        if power:
            ref = post.power(ref)
        assert np.all(rel_rows(got, ref) <= TOL), rel_rows(got, ref)
        plan.close()
