"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bar (per filter row): relative L2 error <= 1e-5, the tolerance stated for this
path.  Small cases compare every output; the full-size workloads compare
sampled outputs that eq. (1) gives one by one (segment boundaries, the start,
the tail and random windows), because eq. (1) is local.  Every output buffer
is NaN-prefilled inside NaN guard bands: no NaN may survive inside, every guard
must survive outside (each output written, nothing written out of bounds).
"""

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


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def ols():
    _need_gpu()
    from paper_1910_01972_amd import ols as m
    return m


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def guarded_output(K, Ns):
    buf = torch.full((K * Ns + 2 * GUARD,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    y = buf[GUARD:GUARD + K * Ns].view(K, Ns)
    return buf, y


def check_guards(buf, K, Ns):
    assert bool(torch.isnan(buf[:GUARD].real).all()), "front guard written"
    assert bool(torch.isnan(buf[GUARD + K * Ns:].real).all()), "back guard written"
    inner = buf[GUARD:GUARD + K * Ns]
    assert not bool(torch.isnan(inner.real).any() or torch.isnan(inner.imag).any()), "output not fully written"


def rel_rows(y, yr):
    return np.linalg.norm(y - yr, axis=1) / np.maximum(np.linalg.norm(yr, axis=1), 1e-300)


def sample_indices(Ns, M, H, rng, windows=16, wlen=1024, boundaries=64):
    idx = [np.arange(0, min(Ns, M + 2)), np.arange(max(0, Ns - 2 * M), Ns)]
    nseg = -(-Ns // H)
    for j in rng.choice(nseg, size=min(boundaries, nseg), replace=False):
        idx.append(np.arange(max(0, j * H - 2), min(Ns, j * H + 3)))
    for st in rng.integers(0, max(1, Ns - wlen), size=windows):
        idx.append(np.arange(st, min(Ns, st + wlen)))
    return np.unique(np.concatenate(idx))


def run_case(ols, s, h, N, hop=None):
    K, M = h.shape
    Ns = s.shape[0]
    plan = ols.OLSPlan(dev(h), N=N)
    if hop is not None:
        plan.set_hop(hop)
    buf, y = guarded_output(K, Ns)
    plan.forward(dev(s), y)
    torch.cuda.synchronize()
    check_guards(buf, K, Ns)
    info = plan.info()
    plan.close()
    return y.cpu().numpy(), info


# ---------------------------------------------------------------- spectra

@pytest.mark.parametrize("N", [256, 512, 1024, 2048, 4096, 8192])
def test_spectra_natural_order(ols, N):
    rng = np.random.default_rng(N)
    for M in (1, 33, N):
        h = (rng.standard_normal((5, M)) + 1j * rng.standard_normal((5, M))).astype(np.complex64)
        say(f"spectra N={N} M={M}")
        plan = ols.OLSPlan(dev(h), N=N)
        got = plan.spectra().cpu().numpy()
        plan.close()
        ref = conv.fft(np.concatenate([h.astype(np.complex128), np.zeros((5, N - M))], axis=1)) / N
        err = np.abs(got - ref).max() / np.abs(ref).max()
        assert err < 2e-6, err


# ---------------------------------------------------------------- small, full comparison

SMALL = [
    # (Ns, K, M, N, hop)
    (1, 1, 1, 256, None),
    (10, 2, 40, 256, None),           # Ns < M
    (200, 1, 256, 256, None),         # M = N
    (5000, 5, 1, 512, None),          # M = 1
    (4097, 2, 100, 1024, 57),         # odd hop
    (70000, 3, 33, 1024, None),       # ragged tail, many tiles
    (9000, 4, 513, 2048, None),
    (12345, 2, 2048, 4096, 1),        # tiny hop
    (30000, 2, 3000, 8192, None),     # long filter
    (100003, 7, 64, 256, None),
    (65536, 16, 255, 512, None),
    (250000, 3, 129, 2048, None),
    (123457, 2, 1000, 4096, None),
    (300001, 2, 4097, 8192, None),
    (50000, 9, 100, 1024, None),      # odd K >= 9: two filters per unit, ragged last group
    (20001, 11, 300, 4096, 1000),
    (33333, 6, 1, 256, None),         # even K, N = 256 (16 transforms per workgroup)
    (40000, 3, 500, 2048, None),      # odd K < 9 at N = 2048: one filter per unit, double-buffered LDS
    (40000, 7, 500, 4096, 2000),      # odd K < 9 at N = 4096
    (262147, 64, 32, 256, None),      # many filters on single-wave transforms (no barriers)
    (70001, 10, 200, 1024, 333),      # N = 1024, odd hop, even K
]


@pytest.mark.parametrize("Ns,K,M,N,hop", SMALL)
def test_forward_small_full(ols, Ns, K, M, N, hop):
    say(f"small Ns={Ns} K={K} M={M} N={N} hop={hop}")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=Ns + M)
    y, _ = run_case(ols, s, h, N, hop)
    rel = rel_rows(y, conv.direct_conv(s, h))
    assert np.all(rel <= TOL), rel


def test_auto_fft_length(ols):
    s, h = workloads.make_signal_filters(50000, 3, 300, seed=77)
    y, info = run_case(ols, s, h, 0)
    assert info["N"] in (256, 512, 1024, 2048, 4096, 8192) and info["N"] >= 300
    assert np.all(rel_rows(y, conv.direct_conv(s, h)) <= TOL)


@pytest.mark.parametrize("K,N_expected", [(23, 1024), (24, 2048), (31, 2048)])
def test_auto_fft_length_many_filters(ols, K, N_expected):
    """The library's length for short filters: N = 1024 up to 23 filters,
    N = 2048 from 24 on (two filters per unit; K = 31 leaves a ragged last
    group); every row matches eq. (1) in guarded outputs."""
    s, h = workloads.make_signal_filters(30011, K, 32, seed=K)
    y, info = run_case(ols, s, h, 0)
    assert info["N"] == N_expected, info
    assert np.all(rel_rows(y, conv.direct_conv(s, h)) <= TOL)


def test_hop_invariance(ols):
    """sec. 3.2: the result does not depend on the segment size or hop."""
    s, h = workloads.make_signal_filters(40000, 2, 200, seed=5)
    ref = conv.direct_conv(s, h)
    for N, hop in ((256, None), (256, 57), (1024, 825), (1024, 1), (8192, None), (8192, 4000)):
        say(f"hop N={N} hop={hop}")
        y, info = run_case(ols, s, h, N, hop)
        if hop is not None:
            assert info["H"] == hop
        assert np.all(rel_rows(y, ref) <= TOL), (N, hop)


def test_delta_identity_and_shift(ols):
    s, _ = workloads.make_signal_filters(100000, 1, 1, seed=6)
    h = np.zeros((3, 64), dtype=np.complex64)
    h[0, 0] = 1
    h[1, 17] = 1
    h[2, 63] = 2 - 1j
    y, _ = run_case(ols, s, h, 1024)
    assert np.max(np.abs(y[0] - s)) < 1e-5
    assert np.max(np.abs(y[1, 17:] - s[:-17])) < 1e-5 and np.max(np.abs(y[1, :17])) < 1e-5
    assert np.max(np.abs(y[2, 63:] - (2 - 1j) * s[:-63])) < 1e-5


def test_update_filters_and_streams(ols):
    s, h = workloads.make_signal_filters(60000, 4, 100, seed=8)
    _, h2 = workloads.make_signal_filters(1, 4, 100, seed=9)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        plan = ols.OLSPlan(dev(h), N=1024, stream=stream)
        sd = dev(s)
        y1 = plan.forward(sd, stream=stream)
        plan.update_filters(dev(h2), stream=stream)
        y2 = plan.forward(sd, stream=stream)
    stream.synchronize()
    assert np.all(rel_rows(y1.cpu().numpy(), conv.direct_conv(s, h)) <= TOL)
    assert np.all(rel_rows(y2.cpu().numpy(), conv.direct_conv(s, h2)) <= TOL)
    plan.close()


def test_deterministic(ols):
    s, h = workloads.make_signal_filters(200000, 8, 256, seed=10)
    plan = ols.OLSPlan(dev(h), N=2048)
    sd = dev(s)
    a = plan.forward(sd)
    b = plan.forward(sd)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    plan.close()


def test_forward_validation(ols):
    from paper_1910_01972_amd._lib import OLSError, lib
    s, h = workloads.make_signal_filters(1000, 2, 16, seed=11)
    plan = ols.OLSPlan(dev(h), N=256)
    sd = dev(s)
    big = torch.empty(3000, dtype=torch.complex64, device="cuda")
    L = lib()
    P = ctypes.c_void_p
    # y overlapping s
    assert L.ols_forward(plan.handle, P(big.data_ptr()), 1000, P(big.data_ptr() + 8 * 500), None) == 1
    # misaligned
    assert L.ols_forward(plan.handle, P(sd.data_ptr() + 4), 100, P(big.data_ptr()), None) == 1
    # negative length, empty signal
    assert L.ols_forward(plan.handle, P(sd.data_ptr()), -1, P(big.data_ptr()), None) == 1
    assert L.ols_forward(plan.handle, P(sd.data_ptr()), 0, P(big.data_ptr()), None) == 0
    # bad hop
    with pytest.raises(OLSError):
        plan.set_hop(256 - 16 + 2)
    with pytest.raises(OLSError):
        plan.set_hop(-3)
    plan.close()


# ---------------------------------------------------------------- full-size workloads (sampled)

def sampled_check(ols, wl, N=None, windows=16):
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    K, M, Ns = wl.K, wl.M, wl.Ns
    plan = ols.OLSPlan(dev(h), N=wl.N if N is None else N)
    info = plan.info()
    say(f"{wl.name}: N={info['N']} H={info['H']} D={info['D']} launch={plan.launch()}")
    buf, y = guarded_output(K, Ns)
    plan.forward(dev(s), y)
    torch.cuda.synchronize()
    check_guards(buf, K, Ns)
    rng = np.random.default_rng(wl.seed)
    idx = sample_indices(Ns, M, info["H"], rng, windows=windows)
    got = y[:, torch.from_numpy(idx).to("cuda")].cpu().numpy()
    ref = conv.direct_conv_at(s, h, idx)
    rel = rel_rows(got, ref)
    plan.close()
    del buf, y
    torch.cuda.empty_cache()
    return rel, len(idx)


def test_single_filter_2p20_full(ols):
    wl = workloads.WORKLOADS["single_filter_2p20"]
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    say("single_filter_2p20 full comparison")
    y, info = run_case(ols, s, h, wl.N)
    assert info["N"] == 1024
    rel = rel_rows(y, conv.direct_conv(s, h))
    say(f"  rel L2 {rel}")
    assert np.all(rel <= TOL), rel


def test_filter_bank_2p23_sampled(ols):
    rel, n = sampled_check(ols, workloads.WORKLOADS["filter_bank_2p23_k32_m256"], windows=32)
    say(f"  filter_bank_2p23: {n} sampled outputs per row, max rel L2 {rel.max():.3e}")
    assert np.all(rel <= TOL), rel


@pytest.mark.parametrize("extra", [1, 4, 8])
def test_filter_bank_off_grid_rows_sampled(ols, extra):
    """The benchmark filter bank with N_s = 2^23 + extra: rows of the output
    start 8, 32 or 64 bytes off the 64-byte grid, so part of every store goes
    through the default-policy branch.  Guards around y, sampled outputs."""
    import dataclasses
    wl = workloads.WORKLOADS["filter_bank_2p23_k32_m256"]
    wl = dataclasses.replace(wl, Ns=wl.Ns + extra)
    rel, n = sampled_check(ols, wl, windows=8)
    say(f"  filter_bank 2^23+{extra}: {n} sampled outputs per row, max rel L2 {rel.max():.3e}")
    assert np.all(rel <= TOL), rel


ROW_PHASE_CASES = [
    # (Ns, K, M, N, derivative); from 2^22 outputs on, rows are re-aligned per row
    ((1 << 20) + 1, 4, 64, 1024, False),
    ((1 << 20) + 5, 4, 300, 2048, True),
    (20001, 3, 256, 2048, False),
    (20003, 3, 250, 2048, False),
    (9999, 5, 40, 256, False),      # transforms narrower than a wave (per-lane stores)
    (30001, 2, 100, 1024, False),   # one wave per transform
    (40005, 4, 513, 4096, False),
    (7001, 2, 1000, 1024, False),   # D = 1008, H = 16
    (25001, 3, 255, 2048, True),    # derivative (effective M = 256)
    (5, 2, 7, 256, False),          # a single segment, shorter than a granule
]


@pytest.mark.parametrize("Ns,K,M,N,deriv", ROW_PHASE_CASES)
@pytest.mark.parametrize("phase", [1, 3, 7])
def test_row_phase_aligned_boundaries_full(ols, Ns, K, M, N, deriv, phase):
    """Output rows that start off the 64-byte grid, at several granule
    phases: part of every store goes through the default-policy branch of the
    granule-aware store.  y starts `phase` samples past a granule boundary of
    a NaN-filled buffer; every output and both guard bands are checked."""
    say(f"row phase {phase}: Ns={Ns} K={K} M={M} N={N} deriv={deriv}")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=Ns + phase)
    plan = ols.OLSPlan(dev(h), N=N, derivative=deriv)
    buf = torch.full((K * Ns + 2 * GUARD,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    assert buf.data_ptr() % 64 == 0
    y = buf[GUARD + phase:GUARD + phase + K * Ns].view(K, Ns)
    plan.forward(dev(s), y)
    torch.cuda.synchronize()
    assert bool(torch.isnan(buf[:GUARD + phase].real).all()), "guard before y written"
    assert bool(torch.isnan(buf[GUARD + phase + K * Ns:].real).all()), "guard after y written"
    got = y.cpu().numpy()
    assert not np.isnan(got).any(), "output not written everywhere"
    ref = post.conv_derivative(s, h) if deriv else conv.direct_conv(s, h)
    rel = rel_rows(got, ref)
    assert np.all(rel <= TOL), rel
    plan.close()


def test_filter_bank_2p23_prefix_full(ols):
    """Full comparison of the first 2^16 outputs of every row, in the same
    plan and launch configuration as the benchmark."""
    wl = workloads.WORKLOADS["filter_bank_2p23_k32_m256"]
    s, h = workloads.make_signal_filters(wl.Ns, wl.K, wl.M, seed=wl.seed)
    plan = ols.OLSPlan(dev(h), N=wl.N)
    y = plan.forward(dev(s))
    torch.cuda.synchronize()
    n = 1 << 16
    got = y[:, :n].cpu().numpy()
    ref = conv.direct_conv(s[:n], h)
    plan.close()
    assert np.all(rel_rows(got, ref) <= TOL)


def test_grad_workload_forward_sampled(ols):
    rel, n = sampled_check(ols, workloads.WORKLOADS["grad_2p22_k16_m512"])
    assert np.all(rel <= TOL), rel


@pytest.mark.parametrize("cell", range(12))
def test_sweep_cells_sampled(ols, cell):
    wl = workloads.sweep_cells()[cell]
    rel, n = sampled_check(ols, wl, N=0, windows=8)
    say(f"  {wl.name}: max rel {rel.max():.3e}")
    assert np.all(rel <= TOL), rel


def test_signal_longer_than_2p31_sampled(ols):
    """N_s = 2^31 + 4099 samples, 2 filters (outputs beyond 2^32 elements):
    64-bit indexing end to end; sampled outputs against eq. (1) at indices
    around 2^31, the segment edges there and the end."""
    Ns, K, M, N = (1 << 31) + 4099, 2, 33, 512
    say(f"huge Ns={Ns} K={K} M={M} N={N}")
    _, h = workloads.make_signal_filters(1, K, M, seed=2024)
    s = torch.empty(Ns, dtype=torch.complex64, device="cuda")
    step = 1 << 28
    for a in range(0, Ns, step):
        s[a:min(Ns, a + step)] = workloads.exact_signal(a, min(Ns, a + step), "cuda")
    plan = ols.OLSPlan(dev(h), N=N)
    H = plan.info()["H"]
    # output rows in a NaN-filled buffer with guard bands on both sides
    G = 4096
    buf = torch.full((K * Ns + 2 * G,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    y = buf[G:G + K * Ns].view(K, Ns)
    plan.forward(s, y)
    torch.cuda.synchronize()
    assert bool(torch.isnan(buf[:G].real).all()) and bool(torch.isnan(buf[G + K * Ns:].real).all()), "guard written"
    assert not bool(torch.isnan(y).any()), "an output sample was not written"
    j = (1 << 31) // H
    idx = np.unique(np.concatenate([np.arange(0, 50), np.arange((1 << 31) - 40, (1 << 31) + 40),
                                    np.arange(j * H - 3, j * H + 3), np.arange(Ns - 60, Ns)]))
    got = y[:, torch.from_numpy(idx).cuda()].cpu().numpy()
    del y, s, buf
    torch.cuda.empty_cache()
    # the oracle sees the same exact values, rebuilt on the host window by window
    ref = np.zeros((K, idx.size), dtype=np.complex128)
    for c, n0 in enumerate(idx):
        w0 = max(0, int(n0) - M + 1)
        win = workloads.exact_signal(w0, int(n0) + 1, "cpu").numpy().astype(np.complex128)
        ref[:, c] = conv.direct_conv_at(win, h, [int(n0) - w0])[:, 0]
    rel = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert np.all(rel <= TOL), rel
    plan.close()


@pytest.mark.parametrize("hop", [900, 500, 100])
def test_row_realignment_with_chosen_hop(ols, hop):
    """A plan with a chosen hop and output rows off the 128-byte grid, large
    enough (>= 2^22 outputs) to be re-aligned: the call runs with the hop
    rounded down to the line grid, and every output matches eq. (1)."""
    Ns, K, M, N = (1 << 20) + 7, 4, 64, 1024
    say(f"row re-alignment, hop {hop}")
    s, h = workloads.make_signal_filters(Ns, K, M, seed=hop)
    plan = ols.OLSPlan(dev(h), N=N)
    plan.set_hop(hop)
    buf, y = guarded_output(K, Ns)
    plan.forward(dev(s), y)
    torch.cuda.synchronize()
    check_guards(buf, K, Ns)
    assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s, h)) <= TOL)
    plan.close()


def test_forward_concurrent_streams_rows_off_grid(ols):
    """ols_forward only reads its plan: two calls of one plan with different
    row phases (both re-aligned) run concurrently on two streams and both
    match eq. (1)."""
    K, M, N = 4, 64, 1024
    NsA, NsB = (1 << 20) + 9, (1 << 20) + 3  # both >= 2^22 outputs with K = 4
    s, h = workloads.make_signal_filters(NsA, K, M, seed=404)
    plan = ols.OLSPlan(dev(h), N=N)
    sd = dev(s)
    bufA = torch.full((K * NsA + 16,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    bufB = torch.full((K * NsB + 16,), complex(float("nan"), float("nan")), dtype=torch.complex64, device="cuda")
    yA = bufA[1:1 + K * NsA].view(K, NsA)
    yB = bufB[3:3 + K * NsB].view(K, NsB)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        plan.forward(sd, y=yA, stream=s1)
        plan.forward(sd[:NsB], y=yB, stream=s2)
    torch.cuda.synchronize()
    ref = conv.direct_conv(s, h)
    assert np.all(rel_rows(yA.cpu().numpy(), ref) <= TOL)
    assert np.all(rel_rows(yB.cpu().numpy(), ref[:, :NsB]) <= TOL)
    plan.close()
