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
    specs = [(Ns, K, M, 0) for Ns, K, M, _ in shapes]
    items, host = [], []
    total = sum(K * Ns for Ns, K, M, _ in shapes)
    say(f"uneven batch: {len(shapes)} signals, {total:.3e} output samples")
    # outputs carved from one NaN-filled buffer with guard bands between them
    buf = torch.full((total + GUARD * (len(shapes) + 1),), complex(float("nan"), float("nan")),
                     dtype=torch.complex64, device="cuda")
    outs, off = [], GUARD
    for Ns, K, M, seed in shapes:
        s, h = workloads.make_signal_filters(Ns, K, M, seed=seed)
        host.append((s, h))
        items.append((dev(s), dev(h), 0))
        outs.append(buf[off:off + K * Ns].view(K, Ns))
        off += K * Ns + GUARD
    b = ols.OLSBatch(items, outputs=outs)
    b.run()
    torch.cuda.synchronize()
    check_guards(buf, specs)
    for y in outs:
        assert not bool(torch.isnan(y).any()), "an output sample was not written"
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


# ---------------------------------------------------------------------------
# The single-call path: ols_batched(dev_items, n, workspace, ws_bytes, stream)
# ---------------------------------------------------------------------------
ITEM_BYTES = 48  # sizeof(ols_batch_item_t); K at byte 24, N at byte 32


def set_item_field(dev_items, i, offset, value):
    b = np.frombuffer(np.int32(value).tobytes(), dtype=np.uint8)
    dev_items[i * ITEM_BYTES + offset:i * ITEM_BYTES + offset + 4] = torch.from_numpy(b.copy()).cuda()


def test_batched_device_call_full(ols):
    items, host, outs, buf = make_batch(ols, SPECS, seed0=70)
    b = ols.OLSBatched(items, outputs=outs)
    say("device batch, workspace bytes", b.workspace_bytes)
    b.run()
    torch.cuda.synchronize()
    assert b.status() == (0, -1)
    check_guards(buf, SPECS)
    for (s, h), y in zip(host, outs):
        if s.shape[0] == 0:
            continue
        yy = y.cpu().numpy()
        assert not np.isnan(yy).any()
        assert np.all(rel_rows(yy, conv.direct_conv(s, h)) <= TOL)


def test_batched_device_matches_plan(ols):
    """The single call and a batch plan run the same setup, spectra and
    forward kernels (twiddles from the device vs the host in float64)."""
    items, host, outs, buf = make_batch(ols, SPECS, seed0=80)
    b = ols.OLSBatched(items, outputs=outs)
    b.run()
    p = ols.OLSBatch(items)
    p.run()
    torch.cuda.synchronize()
    for y1, y2 in zip(outs, p.outputs):
        if y1.numel():
            d = (y1 - y2).abs().max().item()
            assert d <= 1e-6 * max(y2.abs().max().item(), 1.0), d
    p.close()


def test_batched_device_graph_replays_see_new_inputs_and_filters(ols):
    """One captured ols_batched call (setup, spectra, forward; no allocation)
    replayed three times; between replays the signals AND the filters change
    in place, and every replay matches the oracle for the current values."""
    specs = SPECS[:5] + [(40000, 6, 200, 0)]
    items, host, outs, buf = make_batch(ols, specs, seed0=90)
    b = ols.OLSBatched(items, outputs=outs)
    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        b.run(stream=stream)
    stream.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=stream):
        b.run(stream=stream)
    for rep in range(3):
        new = []
        for (sd, hd, N), (s, h) in zip(items, host):
            s2, h2 = workloads.make_signal_filters(s.shape[0], h.shape[0], h.shape[1], seed=700 + rep)
            sd.copy_(torch.from_numpy(s2).cuda())
            hd.copy_(torch.from_numpy(h2).cuda())
            new.append((s2, h2))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        check_guards(buf, specs)
        for (s2, h2), y in zip(new, outs):
            if s2.shape[0] == 0:
                continue
            assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s2, h2)) <= TOL), rep
    assert b.status() == (0, -1)
    del graph


def test_batched_device_rejects_bad_items_without_writing(ols):
    """Items that fail the device-side checks make the whole call write
    nothing: an item with K = 0 (status INVALID_VALUE, its index reported),
    then an FFT length whose spectra exceed the workspace."""
    specs = SPECS[:4]
    items, host, outs, buf = make_batch(ols, specs, seed0=100)
    b = ols.OLSBatched(items, outputs=outs)
    set_item_field(b.dev_items, 2, 24, 0)  # K = 0
    b.run()
    torch.cuda.synchronize()
    assert b.status() == (1, 2)
    assert bool(torch.isnan(buf.real).all()), "an output was written"
    set_item_field(b.dev_items, 2, 24, specs[2][1])  # valid again
    set_item_field(b.dev_items, 0, 32, 4096)  # item 0: N 256 -> 4096, 16x the spectrum bytes
    b.run()
    torch.cuda.synchronize()
    assert b.status() == (1, -1)
    assert bool(torch.isnan(buf.real).all()), "an output was written"
    set_item_field(b.dev_items, 0, 32, specs[0][3])
    b.run()
    torch.cuda.synchronize()
    assert b.status() == (0, -1)
    check_guards(buf, specs)
    for (s, h), y in zip(host, outs):
        if s.shape[0]:
            assert np.all(rel_rows(y.cpu().numpy(), conv.direct_conv(s, h)) <= TOL)


def test_batch_output_shape_checked(ols):
    items, host, outs, buf = make_batch(ols, SPECS[:2], seed0=110)
    K0, Ns0 = outs[0].shape
    # contiguous but one sample short per row (item 0 is the non-empty one)
    bad = [outs[0].reshape(-1)[:K0 * (Ns0 - 1)].view(K0, Ns0 - 1), outs[1]]
    with pytest.raises(ValueError):
        ols.OLSBatch(items, outputs=bad)
    with pytest.raises(ValueError):
        ols.OLSBatched(items, outputs=bad)
    with pytest.raises(ValueError):
        ols.OLSBatch(items, outputs=outs[:1])
