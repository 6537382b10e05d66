"""GPU parity of the batched persistent launch (ols_batch_plan / ols_batched)
against the FP64 oracle, including hipGraph capture and replay."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import conv  # noqa: E402
import workloads  # noqa: E402

pytestmark = pytest.mark.gpu
TOL = 1e-5
GUARD = 2048


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


def rel_rows(y, yr):
    return np.linalg.norm(y - yr, axis=1) / np.maximum(np.linalg.norm(yr, axis=1), 1e-300)


SPECS = [(5000, 3, 40, 256), (0, 2, 10, 512), (20000, 1, 100, 1024), (9000, 4, 513, 2048),
         (30000, 2, 300, 4096), (1, 1, 1, 256), (7777, 5, 64, 512), (100000, 16, 1024, 0), (60000, 9, 17, 0)]


def make_batch(ols, specs, seed0=1):
    items, host = [], []
    # outputs carved from one NaN-filled buffer with guard gaps between them
    sizes = [K * Ns for Ns, K, M, N in specs]
    buf = torch.full((sum(sizes) + GUARD * (len(specs) + 1),), complex(float("nan"), float("nan")),
                     dtype=torch.complex64, device="cuda")
    outs, off = [], GUARD
    for i, (Ns, K, M, N) in enumerate(specs):
        s, h = workloads.make_signal_filters(Ns, K, M, seed=seed0 + i)
        host.append((s, h))
        items.append((dev(s), dev(h), N))
        outs.append(buf[off:off + K * Ns].view(K, Ns))
        off += K * Ns + GUARD
    return items, host, outs, buf


def check_guards(buf, specs):
    off = 0
    for Ns, K, M, N in specs:
        assert bool(torch.isnan(buf[off:off + GUARD].real).all()), "guard written"
        off += GUARD + K * Ns
    assert bool(torch.isnan(buf[off:off + GUARD].real).all())


def test_batched_small_full(ols):
    items, host, outs, buf = make_batch(ols, SPECS)
    b = ols.OLSBatch(items, outputs=outs)
    say("batch", b.info(), [b.item(i) for i in range(len(SPECS))])
    b.run()
    torch.cuda.synchronize()
    check_guards(buf, SPECS)
    for (s, h), y in zip(host, outs):
        if s.shape[0] == 0:
            continue
        yy = y.cpu().numpy()
        assert not np.isnan(yy).any()
        assert np.all(rel_rows(yy, conv.direct_conv(s, h)) <= TOL)
    b.close()


def test_batched_graph_capture_replays(ols):
    """The launch allocates nothing and is captured once; every replay reads
    the inputs' current contents and matches an eager launch."""
    specs = SPECS[:5]
    items, host, outs, buf = make_batch(ols, specs, seed0=30)
    b = ols.OLSBatch(items, outputs=outs)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.run(stream=stream)  # warm-up on the capture stream
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b.run(stream=stream)
    for rep in range(3):
        # eager work between replays: new signal values written in place
        new = []
        for (sd, hd, N), (s, h) in zip(items, host):
            s2, _ = workloads.make_signal_filters(s.shape[0], 1, 1, seed=500 + rep)
            sd.copy_(torch.from_numpy(s2).cuda())
            new.append((s2, h))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for (s2, h), y in zip(new, outs):
            if s2.shape[0] == 0:
                continue
            assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s2, h)) <= TOL), rep
        eager = [y.clone() for y in outs]
        b.run()
        torch.cuda.synchronize()
        for e, y in zip(eager, outs):
            assert torch.equal(e, y)
    b.close()


def test_batched_custom_fft_length_and_validation(ols):
    from paper_1910_01972_amd._lib import OLSError
    items, host, outs, _ = make_batch(ols, [(20000, 3, 100, 0), (10000, 2, 50, 0)], seed0=60)
    b = ols.OLSBatch(items, outputs=outs, fft_length=lambda M, K: 512)
    assert b.item(0)["N"] == 512 and b.item(1)["N"] == 512
    b.run()
    torch.cuda.synchronize()
    for (s, h), y in zip(host, outs):
        assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s, h)) <= TOL)
    b.close()
    s, h = items[0][0], items[0][1]
    with pytest.raises(OLSError):
        ols.OLSBatch([(s, h, 8192)])          # batched N is at most 4096
    with pytest.raises(OLSError):
        ols.OLSBatch([(s, h, 300)])           # not a power of two
    long_h = torch.zeros((1, 5000), dtype=torch.complex64, device="cuda")
    with pytest.raises(OLSError):
        ols.OLSBatch([(s, long_h, 0)])        # needs N > 4096


def test_uneven_batch_workload_sampled(ols):
    """The uneven batch: 256 signals, N_s log-uniform in [2^14, 2^22],
    K ~ U{1..16}, M log-uniform in [16, 1024], one persistent launch; a few
    hundred sampled outputs per item against eq. (1)."""
    shapes = workloads.batched_items()
    items, host = [], []
    total = 0
    for Ns, K, M, seed in shapes:
        s, h = workloads.make_signal_filters(Ns, K, M, seed=seed)
        host.append((s, h))
        items.append((dev(s), dev(h), 0))
        total += K * Ns
    say(f"uneven batch: {len(shapes)} signals, {total:.3e} output samples")
    b = ols.OLSBatch(items)
    b.run()
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    worst = 0.0
    for i, ((s, h), y) in enumerate(zip(host, b.outputs)):
        Ns, M = s.shape[0], h.shape[1]
        H = b.item(i)["H"]
        idx = np.unique(np.concatenate([np.arange(min(Ns, M + 2)), np.arange(max(0, Ns - 64), Ns),
                                        rng.integers(0, Ns, 64),
                                        np.clip(np.arange(1, 9) * H - 1, 0, Ns - 1)]))
        got = y[:, torch.from_numpy(idx).cuda()].cpu().numpy()
        r = rel_rows(got, conv.direct_conv_at(s, h, idx))
        worst = max(worst, float(r.max()))
    say(f"  worst sampled rel L2 {worst:.3e}")
    assert worst <= TOL
    b.close()
