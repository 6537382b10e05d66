"""CPU oracle pinned to the paper and to mathematics (no GPU needed)."""

import numpy as np
import pytest

from oracle import adjoint, conv, post
import oracle_pins as P
import workloads


def test_fft_golden():
    P.pin_fft_golden(conv.fft)


def test_dft_definition_golden():
    P.pin_fft_golden(conv.dft)


def test_fft_vs_bruteforce():
    P.pin_fft_vs_bruteforce(conv.fft)


def test_fft_closed_forms_and_parseval():
    P.pin_fft_closed_forms(conv.fft)


def test_fft_vs_library():
    P.pin_fft_library(conv.fft)


def test_ifft_roundtrip():
    P.pin_ifft_roundtrip(conv.fft, conv.ifft)


def test_fft_rejects_bad_length():
    with pytest.raises(ValueError):
        conv.fft(np.ones(6))


@pytest.mark.parametrize("impl", ["direct_conv", "direct_conv_loops", "full_fft_conv"])
def test_conv_golden(impl):
    P.pin_conv_golden(getattr(conv, impl))


def test_ols_golden_small_segments():
    P.pin_conv_golden(lambda s, h: conv.ols_conv(s, h, 2))
    P.pin_ols_golden(conv.ols_conv)


@pytest.mark.parametrize("impl", ["direct_conv", "full_fft_conv"])
def test_conv_bruteforce(impl):
    P.pin_conv_bruteforce(getattr(conv, impl))


def test_direct_conv_loops_is_bruteforce():
    P.pin_conv_bruteforce(conv.direct_conv_loops)


@pytest.mark.parametrize("impl", ["direct_conv", "full_fft_conv"])
def test_conv_library(impl):
    P.pin_conv_library(getattr(conv, impl))


@pytest.mark.parametrize("impl", ["direct_conv", "full_fft_conv"])
def test_conv_closed_forms(impl):
    P.pin_conv_closed_forms(getattr(conv, impl))


def test_conv_linearity():
    P.pin_conv_linearity(conv.direct_conv)


def test_direct_conv_chunking():
    rng = np.random.default_rng(3)
    s = P.rand_c(rng, 1000)
    h = P.rand_c(rng, 2, 33)
    P._close(conv.direct_conv(s, h, chunk=7), conv.direct_conv(s, h), 1e-13, "chunked")


def test_direct_conv_at():
    rng = np.random.default_rng(4)
    s = P.rand_c(rng, 2000)
    h = P.rand_c(rng, 3, 50)
    idx = np.array([0, 1, 48, 49, 50, 777, 1999])
    P._close(conv.direct_conv_at(s, h, idx), conv.direct_conv(s, h)[:, idx], 1e-13, "direct_conv_at")
    with pytest.raises(IndexError):
        conv.direct_conv_at(s, h, [2000])


def test_circular_alias_golden():
    P.pin_circular_alias(conv.fft, conv.ifft)


def test_ols_discard_count_bruteforce():
    """A causal filter of length M corrupts exactly circular positions 0..M-2
    (sec. 3.2: M-1 discarded samples; footnote to eq. 2: causal filters alias
    the start).  Brute force on a tiny segment."""
    rng = np.random.default_rng(8)
    N = 16
    for M in (1, 2, 5, 16):
        x = P.rand_c(rng, N)
        h = P.rand_c(rng, M)
        circ = np.zeros(N, dtype=np.complex128)
        lin = np.zeros(N, dtype=np.complex128)
        for n in range(N):
            for k in range(M):
                circ[n] += x[(n - k) % N] * h[k]
                if n - k >= 0:
                    lin[n] += x[n - k] * h[k]
        P._close(conv.ifft(conv.fft(x) * conv.fft(np.concatenate([h, np.zeros(N - M)]))), circ, 1e-12, "fft circ")
        bad = np.abs(circ - lin) > 1e-9
        assert list(np.nonzero(bad)[0]) == list(range(M - 1)), (M, np.nonzero(bad)[0])


def test_ols_matches_definition():
    P.pin_ols_matches_definition(conv.ols_conv, None)


def test_ols_segment_invariance():
    P.pin_ols_segment_invariance(conv.ols_conv)


def test_ols_filters_independent():
    P.pin_ols_filters_independent(conv.ols_conv)


def test_ols_rejects_bad_geometry():
    s = np.ones(10)
    with pytest.raises(ValueError):
        conv.ols_conv(s, np.ones((1, 9)), 8)
    with pytest.raises(ValueError):
        conv.ols_conv(s, np.ones((1, 4)), 12)
    with pytest.raises(ValueError):
        conv.ols_conv(s, np.ones((1, 4)), 8, 6)


def test_direct_vs_ols_medium_fp64():
    """Two independent FP64 routes agree to ~1e-13 on a workload-shaped input."""
    s, h = workloads.make_signal_filters(1 << 15, 4, 256, seed=123)
    a = conv.direct_conv(s, h)
    b = conv.ols_conv(s, h, 2048)
    rel = np.linalg.norm(a - b, axis=1) / np.linalg.norm(a, axis=1)
    assert np.all(rel < 1e-13), rel


def test_adjoint_loops_vs_vectorised():
    rng = np.random.default_rng(9)
    s = P.rand_c(rng, 40)
    h = P.rand_c(rng, 2, 7)
    g = P.rand_c(rng, 2, 40)
    P._close(adjoint.grad_signal(g, h), adjoint.grad_signal_loops(g, h), 1e-12, "ds")
    P._close(adjoint.grad_filters(g, s, 7), adjoint.grad_filters_loops(g, s, 7), 1e-12, "dh")
    P._close(adjoint.grad_signal(g, h, chunk=3), adjoint.grad_signal(g, h), 1e-13, "ds chunk")
    P._close(adjoint.grad_filters(g, s, 7, chunk=3), adjoint.grad_filters(g, s, 7), 1e-13, "dh chunk")


@pytest.mark.parametrize("pair", ["vectorised", "loops"])
def test_adjoint_dot_product(pair):
    if pair == "vectorised":
        P.pin_adjoint_dot_product(conv.direct_conv, adjoint.grad_signal, adjoint.grad_filters)
    else:
        P.pin_adjoint_dot_product(conv.direct_conv_loops, adjoint.grad_signal_loops, adjoint.grad_filters_loops)


def test_adjoint_finite_differences():
    P.pin_adjoint_finite_differences(conv.direct_conv, adjoint.grad_signal, adjoint.grad_filters)


def test_workload_generator_recipe():
    s, h = workloads.make_signal_filters(1000, 3, 64, seed=7)
    assert s.dtype == np.complex64 and h.dtype == np.complex64
    assert s.shape == (1000,) and h.shape == (3, 64)
    assert np.all(np.abs(s.real) <= 1) and np.all(np.abs(s.imag) <= 1)
    s2, h2 = workloads.make_signal_filters(1000, 3, 64, seed=7)
    assert np.array_equal(s, s2) and np.array_equal(h, h2)
    # filter variance per component ~ 1/M
    big = workloads.make_signal_filters(10, 64, 1024, seed=8)[1]
    v = np.var(big.real) * 1024
    assert 0.9 < v < 1.1


def test_adjoint_matches_torch_autograd_convention():
    """Library cross-check: PyTorch's own complex autograd of eq. (1) (computed
    by zero-padded FFTs in complex128) gives the oracle's adjoint for
    L = Re sum conj(w) y, i.e. the gradient convention of ols_backward."""
    torch = pytest.importorskip("torch")
    torch.manual_seed(0)
    Ns, K, M = 64, 3, 7
    s = torch.randn(Ns, dtype=torch.complex128, requires_grad=True)
    h = torch.randn(K, M, dtype=torch.complex128, requires_grad=True)
    w = torch.randn(K, Ns, dtype=torch.complex128)
    P = 128
    Sf = torch.fft.fft(torch.nn.functional.pad(s, (0, P - Ns)))
    Hf = torch.fft.fft(torch.nn.functional.pad(h, (0, P - M)), dim=1)
    y = torch.fft.ifft(Sf[None, :] * Hf, dim=1)[:, :Ns]
    (torch.conj(w) * y).real.sum().backward()
    P_ = adjoint.grad_signal(w.numpy(), h.detach().numpy())
    Q_ = adjoint.grad_filters(w.numpy(), s.detach().numpy(), M)
    assert np.abs(s.grad.numpy() - P_).max() < 1e-12
    assert np.abs(h.grad.numpy() - Q_).max() < 1e-12


def test_grad_signal_at():
    rng = np.random.default_rng(12)
    g = P.rand_c(rng, 3, 500)
    h = P.rand_c(rng, 3, 40)
    idx = np.array([0, 1, 100, 459, 460, 461, 499])
    P._close(adjoint.grad_signal_at(g, h, idx), adjoint.grad_signal(g, h)[idx], 1e-12, "grad_signal_at")
    with pytest.raises(IndexError):
        adjoint.grad_signal_at(g, h, [500])


def test_post_golden():
    P.pin_post_golden(post.power, post.derivative, conv.direct_conv)
    P.pin_post_golden(post.power, post.derivative, conv.direct_conv_loops)


def test_post_closed_forms():
    P.pin_power_closed_forms(post.power)
    P.pin_derivative_closed_forms(post.derivative, conv.direct_conv)


def test_post_composed_and_sampled():
    rng = np.random.default_rng(33)
    s = P.rand_c(rng, 3000)
    h = P.rand_c(rng, 3, 40)
    y = conv.direct_conv(s, h)
    P._close(post.conv_power(s, h), post.power(y), 1e-14, "conv_power")
    P._close(post.conv_derivative(s, h), post.derivative(y), 1e-14, "conv_derivative")
    idx = np.array([0, 1, 2, 39, 40, 41, 1234, 2999])
    P._close(post.derivative_at(s, h, idx), post.derivative(y)[:, idx], 1e-12, "derivative_at")


def test_stencil_pins():
    P.pin_stencil_golden(post.stencil, post.conv_stencil)
    P.pin_stencil_closed_forms(post.stencil, post.derivative)
    P.pin_lagrange(post.lagrange_weights, post.midpoint_interpolation_stencil)


def test_stencil_composed_and_sampled():
    rng = np.random.default_rng(43)
    s = P.rand_c(rng, 2000)
    h = P.rand_c(rng, 3, 40)
    w, L = post.midpoint_interpolation_stencil()
    z = post.conv_stencil(s, h, w, L)
    assert z.shape == (3, 4000)
    # the stencil of the convolution continued by zeros, by hand
    y = conv.direct_conv(np.concatenate([s, np.zeros(2)]), h)
    P._close(z, post.stencil(y, w, L, 2000), 1e-14, "conv_stencil")
    # phase 0 is eq. (1); the backward difference is the derivative
    P._close(z[:, 0::2], conv.direct_conv(s, h), 1e-12, "phase 0")
    P._close(post.conv_stencil(s, h, [[-1.0, 1.0]], 1), post.conv_derivative(s, h), 1e-12, "difference")
    idx = np.array([0, 1, 2, 3, 78, 79, 80, 81, 1234, 3997, 3998, 3999])
    P._close(post.stencil_at(s, h, w, L, idx), z[:, idx], 1e-12, "stencil_at")
    with pytest.raises(IndexError):
        post.stencil_at(s, h, w, L, [4000])
    # R2R: the real stencil of the real convolution
    sr = rng.uniform(-1, 1, 1500)
    hr = rng.uniform(-1, 1, (2, 33))
    zr = post.conv_stencil_real(sr, hr, w, L)
    yr = conv.direct_conv_real(np.concatenate([sr, np.zeros(2)]), hr)
    P._close(zr, post.stencil(yr, w, L, 1500).real, 1e-14, "conv_stencil_real")
    P._close(post.stencil_at(sr, hr, w, L, idx[:-3], real=True), zr[:, idx[:-3]], 1e-12, "stencil_at real")


def test_real_conv_pins():
    P.pin_real_conv(conv.direct_conv_real)


def test_real_conv_at_and_complex_agreement():
    rng = np.random.default_rng(42)
    s = rng.standard_normal(5000)
    h = rng.standard_normal((4, 300))
    y = conv.direct_conv_real(s, h)
    idx = np.array([0, 1, 298, 299, 300, 4999, 2500])
    P._close(conv.direct_conv_real_at(s, h, idx), y[:, idx], 1e-12, "real_at")
    yc = conv.direct_conv(s.astype(complex), h.astype(complex))
    P._close(yc.real, y, 1e-12, "complex path real part")
    assert np.abs(yc.imag).max() == 0.0


def test_exact_signal_generator_is_window_consistent():
    """The long-signal generator rebuilds any window identically (it is used
    for the GPU input and, window by window, for the oracle's)."""
    pytest.importorskip("torch")
    full = workloads.exact_signal(0, 5000).numpy()
    assert full.dtype == np.complex64
    for a, b in ((0, 10), (1234, 1300), (4990, 5000)):
        assert np.array_equal(workloads.exact_signal(a, b).numpy(), full[a:b])
    big = workloads.exact_signal((1 << 31) - 2, (1 << 31) + 2).numpy()
    n = np.arange((1 << 31) - 2, (1 << 31) + 2, dtype=np.int64)
    want = ((n * 40503) % (1 << 20)) / (1 << 20) - 0.5 + 1j * (((n * 65537) % (1 << 20)) / (1 << 20) - 0.5)
    assert np.array_equal(big.astype(np.complex128), want)
