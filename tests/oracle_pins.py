"""Pins for the CPU oracle: checks against things other than the oracle itself.

Each ``pin_*`` takes the implementation under check as an argument and raises
AssertionError when a pin fails, so the same checks run on the real oracle
(tests/test_oracle.py) and on copies with planted mistakes
(tests/test_oracle_mutations.py), which must be caught.

Sources of truth used here:
* hand-derived fixtures in tests/golden/ (eq. 1, eq. 2, sec. 3.2);
* closed forms: delta, shifted delta, boxcar (prefix sums), complex exponential
  (eigenfunction of a linear time-invariant filter), Parseval;
* brute force on tiny inputs (explicit loops, the O(N^2) DFT);
* library routines as cross-checks (numpy.fft.fft, numpy.convolve);
* the paper's statement that the OLS result does not depend on the segment
  size (sec. 3.2).
"""

from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def _c(d, re, im=None):
    r = np.asarray(d[re], dtype=np.float64)
    i = np.zeros_like(r) if im is None or im not in d else np.asarray(d[im], dtype=np.float64)
    return r + 1j * i


def _close(a, b, tol, what):
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, f"{what}: shape {a.shape} != {b.shape}"
    err = np.max(np.abs(a - b)) if a.size else 0.0
    scale = max(1.0, np.max(np.abs(b)) if b.size else 1.0)
    assert err <= tol * scale, f"{what}: max abs err {err:.3e} > {tol:.1e} (scale {scale:.3g})"


def rand_c(rng, *shape):
    return rng.uniform(-1, 1, shape) + 1j * rng.uniform(-1, 1, shape)


# ---------------------------------------------------------------- FFT pins

def pin_fft_golden(fft):
    for name in ("dft4.json", "dft8_rect.json"):
        d = load_golden(name)
        _close(fft(_c(d, "x_re", "x_im")), _c(d, "X_re", "X_im"), 1e-13, name)


def pin_fft_vs_bruteforce(fft):
    rng = np.random.default_rng(11)
    for N in (1, 2, 4, 8, 16, 32, 64):
        x = rand_c(rng, 3, N)
        n = np.arange(N)
        ref = np.zeros((3, N), dtype=np.complex128)
        for m in range(N):  # written out, independent of the oracle's dft()
            ref[:, m] = np.sum(x * np.exp(-2j * np.pi * m * n / N), axis=1)
        _close(fft(x), ref, 1e-12, f"fft vs brute force N={N}")


def pin_fft_closed_forms(fft):
    for N in (8, 64, 1024):
        d = np.zeros(N, dtype=np.complex128)
        d[0] = 1
        _close(fft(d), np.ones(N), 1e-13, "fft(delta) = ones")
        for k0 in (1, 3, N // 2 - 1):
            e = np.exp(2j * np.pi * k0 * np.arange(N) / N)
            want = np.zeros(N, dtype=np.complex128)
            want[k0] = N
            _close(fft(e), want, 1e-11, f"fft(exp) = N delta, N={N}, k0={k0}")
        x = rand_c(np.random.default_rng(N), N)
        X = fft(x)
        assert abs(np.sum(np.abs(x) ** 2) - np.sum(np.abs(X) ** 2) / N) < 1e-10 * N, "Parseval"


def pin_fft_library(fft):
    rng = np.random.default_rng(5)
    for N in (128, 2048, 8192):
        x = rand_c(rng, 2, N)
        _close(fft(x), np.fft.fft(x, axis=-1), 1e-12, f"fft vs numpy.fft N={N}")


def pin_ifft_roundtrip(fft, ifft):
    rng = np.random.default_rng(6)
    for N in (2, 16, 4096):
        x = rand_c(rng, 2, N)
        _close(ifft(fft(x)), x, 1e-13, f"ifft(fft(x)) = x N={N}")
        _close(ifft(x), np.fft.ifft(x, axis=-1), 1e-13, f"ifft vs numpy N={N}")


# ---------------------------------------------------------------- eq. (1) pins

def pin_conv_golden(conv):
    d = load_golden("conv_complex_small.json")
    _close(conv(_c(d, "s_re", "s_im"), _c(d, "h_re", "h_im")), _c(d, "y_re", "y_im"), 1e-13, "conv golden")


def pin_conv_bruteforce(conv):
    rng = np.random.default_rng(21)
    for Ns, M in ((1, 1), (5, 3), (17, 16), (64, 7), (9, 12)):
        s = rand_c(rng, Ns)
        h = rand_c(rng, 2, M)
        ref = np.zeros((2, Ns), dtype=np.complex128)
        for r in range(2):
            for n in range(Ns):
                for k in range(M):
                    if n - k >= 0:
                        ref[r, n] += s[n - k] * h[r, k]
        _close(conv(s, h), ref, 1e-12, f"conv brute force Ns={Ns} M={M}")


def pin_conv_library(conv):
    rng = np.random.default_rng(22)
    s = rand_c(rng, 3000)
    h = rand_c(rng, 3, 45)
    ref = np.stack([np.convolve(s, h[r])[:3000] for r in range(3)])
    _close(conv(s, h), ref, 1e-11, "conv vs numpy.convolve")


def pin_conv_closed_forms(conv):
    rng = np.random.default_rng(23)
    Ns = 500
    s = rand_c(rng, Ns)
    # delta: y = s exactly
    for M in (1, 9, 64):
        h = np.zeros((1, M), dtype=np.complex128)
        h[0, 0] = 1
        _close(conv(s, h)[0], s, 1e-13, f"delta identity M={M}")
    # shifted delta: y[n] = s[n-d]
    for d in (1, 7, 31):
        h = np.zeros((1, 32), dtype=np.complex128)
        h[0, d] = 1
        want = np.concatenate([np.zeros(d), s[:-d]])
        _close(conv(s, h)[0], want, 1e-13, f"shift d={d}")
    # M = 1: scaling
    _close(conv(s, np.array([[2 - 3j]]))[0], (2 - 3j) * s, 1e-13, "M=1 scaling")
    # boxcar: y[n] = sum_{m=max(0,n-M+1)}^{n} s[m]  (prefix sums)
    for M in (2, 13, 100):
        c = np.concatenate([[0], np.cumsum(s)])
        n = np.arange(Ns)
        want = c[n + 1] - c[np.maximum(0, n - M + 1)]
        _close(conv(s, np.ones((1, M)))[0], want, 1e-11, f"boxcar M={M}")
    # complex exponential is an eigenfunction: y[n] = e^{i w n} * sum_k h[k] e^{-i w k}, n >= M-1
    for M, w in ((16, 0.3), (33, 2.0), (64, -1.1)):
        h = rand_c(rng, 1, M)
        e = np.exp(1j * w * np.arange(Ns))
        Hw = np.sum(h[0] * np.exp(-1j * w * np.arange(M)))
        y = conv(e, h)[0]
        _close(y[M - 1:], e[M - 1:] * Hw, 1e-11, f"eigenfunction M={M}")


def pin_conv_linearity(conv):
    rng = np.random.default_rng(24)
    s1, s2 = rand_c(rng, 400), rand_c(rng, 400)
    h1, h2 = rand_c(rng, 2, 20), rand_c(rng, 2, 20)
    a, b = 0.7 - 0.2j, -1.3 + 0.5j
    _close(conv(a * s1 + b * s2, h1), a * conv(s1, h1) + b * conv(s2, h1), 1e-12, "linear in s")
    _close(conv(s1, a * h1 + b * h2), a * conv(s1, h1) + b * conv(s1, h2), 1e-12, "linear in h")


# ---------------------------------------------------------------- OLS pins

def pin_ols_golden(ols):
    d = load_golden("ols_boxcar_n4.json")
    _close(ols(_c(d, "s_re", "s_im"), _c(d, "h_re", "h_im"), d["N"]), _c(d, "y_re", "y_im"), 1e-12, "ols golden")


def pin_circular_alias(fft, ifft):
    d = load_golden("circular_alias_n4.json")
    x = np.asarray(d["x_re"], dtype=np.complex128)
    h = np.zeros(4, dtype=np.complex128)
    h[:2] = d["h_re"]
    circ = ifft(fft(x) * fft(h))
    _close(circ, np.asarray(d["circular_re"], dtype=np.complex128), 1e-13, "circular conv golden")
    lin = np.asarray(d["linear_re"], dtype=np.complex128)
    a = d["aliased_count"]
    _close(circ[a:], lin[a:], 1e-13, "unaliased part equals linear conv")
    assert abs(circ[a - 1] - lin[a - 1]) > 1.0, "aliased sample differs"


def pin_ols_matches_definition(ols, conv_ref):
    """OLS equals eq. (1) (computed by brute-force loops or a library)."""
    rng = np.random.default_rng(31)
    cases = [
        # (Ns, K, M, N, H)
        (1000, 2, 17, 64, None),
        (1000, 1, 64, 64, None),      # M = N: one valid sample per segment
        (999, 3, 1, 32, None),        # M = 1
        (10, 2, 30, 64, None),        # Ns < M
        (40, 1, 16, 64, None),        # Ns < L
        (1, 1, 5, 8, None),           # single sample
        (0, 2, 5, 8, None),           # empty signal
        (4097, 2, 100, 256, 157),     # Ns = 1 mod H... and a non-default hop
        (4095, 2, 100, 256, 91),
        (6000, 2, 200, 1024, 825),    # H = L
    ]
    for Ns, K, M, N, H in cases:
        s = rand_c(rng, Ns)
        h = rand_c(rng, K, M)
        ref = np.stack([np.convolve(s, h[r])[:Ns] for r in range(K)]) if Ns else np.zeros((K, 0))
        got = ols(s, h, N) if H is None else ols(s, h, N, H)
        _close(got, ref, 1e-11, f"ols vs definition Ns={Ns} K={K} M={M} N={N} H={H}")


def pin_ols_segment_invariance(ols):
    """sec. 3.2: the convolved signal does not depend on the segment size."""
    rng = np.random.default_rng(32)
    s = rand_c(rng, 5000)
    h = rand_c(rng, 2, 60)
    base = ols(s, h, 64)
    for N in (128, 256, 1024, 8192):
        _close(ols(s, h, N), base, 1e-11, f"segment invariance N={N}")
    for H in (1, 5, 64, 196):
        _close(ols(s, h, 256, H), base, 1e-11, f"hop invariance H={H}")


def pin_ols_filters_independent(ols):
    """Reading of Alg. 2: each filter multiplies the unchanged segment spectrum."""
    rng = np.random.default_rng(33)
    s = rand_c(rng, 700)
    h = np.zeros((3, 8), dtype=np.complex128)
    h[0] = rand_c(rng, 8)
    h[1, 0] = 1.0          # delta: must return s itself
    h[2, 3] = 1.0          # shift by 3
    y = ols(s, h, 32)
    _close(y[1], s, 1e-12, "second filter (delta) sees the raw spectrum")
    _close(y[2], np.concatenate([np.zeros(3), s[:-3]]), 1e-12, "third filter (shift)")


# ---------------------------------------------------------------- adjoint pins

def pin_adjoint_dot_product(conv, grad_signal, grad_filters):
    """<A s, g> = <s, A^H g> and <B h, g> = <h, B^H g>."""
    rng = np.random.default_rng(41)
    for Ns, K, M in ((300, 3, 20), (50, 2, 64), (1, 1, 1)):
        s = rand_c(rng, Ns)
        h = rand_c(rng, K, M)
        g = rand_c(rng, K, Ns)
        y = conv(s, h)
        lhs = np.vdot(g.ravel(), y.ravel())
        rhs_s = np.vdot(grad_signal(g, h), s)
        rhs_h = np.vdot(grad_filters(g, s, M).ravel(), h.ravel())
        assert abs(lhs - rhs_s) <= 1e-10 * max(1, abs(lhs)), f"adjoint in s {lhs} vs {rhs_s}"
        assert abs(lhs - rhs_h) <= 1e-10 * max(1, abs(lhs)), f"adjoint in h {lhs} vs {rhs_h}"


def pin_adjoint_finite_differences(conv, grad_signal, grad_filters):
    """L = Re sum conj(g) y is linear in s and h, so central differences are exact."""
    rng = np.random.default_rng(42)
    Ns, K, M = 64, 2, 9
    s = rand_c(rng, Ns)
    h = rand_c(rng, K, M)
    g = rand_c(rng, K, Ns)

    def loss(s_, h_):
        return float(np.real(np.vdot(g.ravel(), conv(s_, h_).ravel())))

    ds = grad_signal(g, h)
    dh = grad_filters(g, s, M)
    eps = 0.5
    for m in (0, 5, Ns - 1):
        for unit, part in ((1.0, "re"), (1j, "im")):
            e = np.zeros(Ns, dtype=np.complex128)
            e[m] = unit * eps
            fd = (loss(s + e, h) - loss(s - e, h)) / (2 * eps)
            want = ds[m].real if part == "re" else ds[m].imag
            assert abs(fd - want) < 1e-10, f"ds[{m}].{part}: fd {fd} vs {want}"
    for r, k in ((0, 0), (1, M - 1), (1, 4)):
        for unit, part in ((1.0, "re"), (1j, "im")):
            e = np.zeros((K, M), dtype=np.complex128)
            e[r, k] = unit * eps
            fd = (loss(s, h + e) - loss(s, h - e)) / (2 * eps)
            want = dh[r, k].real if part == "re" else dh[r, k].imag
            assert abs(fd - want) < 1e-10, f"dh[{r},{k}].{part}: fd {fd} vs {want}"


# ---------------------------------------------------------- post-processing

def pin_post_golden(power, derivative, conv):
    d = load_golden("post_small.json")
    s = _c(d, "s_re", "s_im")
    h = _c(d, "h_re", "h_im")
    y = conv(s, h)
    _close(y, _c(d, "y_re", "y_im"), 1e-14, "post_small y")
    _close(derivative(y), _c(d, "d_re", "d_im"), 1e-14, "post_small derivative")
    _close(power(y), np.asarray(d["p"], dtype=np.float64), 1e-14, "post_small power")


def pin_power_closed_forms(power):
    rng = np.random.default_rng(31)
    w = rng.uniform(-np.pi, np.pi, 64)
    _close(power(np.exp(1j * w)), np.ones(64), 1e-14, "unit circle")
    r = rng.uniform(-3, 3, 64)
    _close(power(r + 0j), r * r, 1e-14, "real axis")
    _close(power(1j * r), r * r, 1e-14, "imaginary axis")
    z = rand_c(rng, 3, 50)
    assert np.asarray(power(z)).dtype.kind == "f" and np.all(power(z) >= 0)
    # Parseval: the summed power equals the summed power of the spectrum / N
    _close(np.sum(power(z), axis=-1), np.sum(power(np.fft.fft(z)), axis=-1) / 50, 1e-12, "Parseval")


def pin_derivative_closed_forms(derivative, conv):
    rng = np.random.default_rng(32)
    # boxcar on a constant: y[n] = min(n+1, M), so d[n] = 1 for n < M, else 0
    M, Ns = 9, 40
    d = derivative(conv(np.ones(Ns), np.ones((1, M))))
    _close(d, (np.arange(Ns) < M).astype(float)[None, :], 1e-13, "boxcar step")
    # telescoping: the running sum of the difference gives back y
    y = rand_c(rng, 2, 77)
    _close(np.cumsum(derivative(y), axis=-1), y, 1e-13, "telescoping")
    # complex exponential: once the filter is full, d[n] = y[n] (1 - e^{-iw})
    w = 0.37
    n = np.arange(200)
    h = rand_c(rng, 1, 16)
    y = conv(np.exp(1j * w * n), h)
    d = derivative(y)
    _close(d[:, 16:], y[:, 16:] * (1 - np.exp(-1j * w)), 1e-12, "exponential")
    # a delta at m: y = h shifted, d is h[k] - h[k-1] shifted
    s = np.zeros(30, dtype=complex)
    s[5] = 1
    h = rand_c(rng, 1, 6)
    want = np.zeros((1, 30), dtype=complex)
    want[0, 5:12] = np.concatenate([h[0], [0]]) - np.concatenate([[0], h[0]])
    _close(derivative(conv(s, h)), want, 1e-13, "delta")


# ------------------------------------------------------- non-local stencil

def pin_stencil_golden(stencil, conv_stencil):
    """Hand-worked fixture: cubic midpoint interpolation, backward and central
    differences on a given sequence, and interpolation of a convolution whose
    tail (samples past N_s) the stencil reads."""
    d = load_golden("stencil_small.json")
    y = _c(d, "y_re", "y_im")
    w = np.asarray(d["interp_w"], dtype=np.float64)
    L = d["interp_left"]
    _close(stencil(y, w, L, 4), _c(d, "interp_re", "interp_im"), 1e-14, "stencil_small interp")
    _close(stencil(y[:4], np.array([[-1.0, 1.0]]), 1, 4), _c(d, "diff_re", "diff_im"), 1e-14, "stencil_small diff")
    _close(stencil(y[:5], np.array([[-0.5, 0.0, 0.5]]), 1, 4), _c(d, "central_re", "central_im"), 1e-14,
           "stencil_small central")
    s = _c(d, "s_re", "s_im")
    h = _c(d, "h_re", "h_im")
    _close(conv_stencil(s, h, w, L), _c(d, "conv_interp_re", "conv_interp_im"), 1e-14, "stencil_small conv interp")


def pin_stencil_closed_forms(stencil, derivative):
    rng = np.random.default_rng(41)
    Ns = 60
    # identity stencil
    y = rand_c(rng, 2, Ns)
    _close(stencil(y, np.array([[1.0]]), 0, Ns), y, 1e-15, "identity")
    # the backward-difference stencil is the (separately pinned) derivative
    _close(stencil(y, np.array([[-1.0, 1.0]]), 1, Ns), derivative(y), 1e-14, "difference = derivative")
    # impulse response: y = delta at m gives z[J n + j] = w[j][m - n + L] for the n it reaches
    J, L, R = 3, 2, 1
    w = rng.uniform(-1, 1, (J, L + 1 + R))
    m = 30
    yd = np.zeros(Ns + R, dtype=complex)
    yd[m] = 1
    want = np.zeros(J * Ns, dtype=complex)
    for n in range(m - R, m + L + 1):
        for j in range(J):
            want[J * n + j] = w[j, m - n + L]
    _close(stencil(yd, w, L, Ns), want, 1e-15, "impulse response")
    # complex exponential: z[J n + j] = e^{i a n} sum_d w[j][d + L] e^{i a d} once every tap is at n + d >= 0
    a = 0.41
    ye = np.exp(1j * a * np.arange(Ns + R))
    resp = np.array([sum(w[j, d + L] * np.exp(1j * a * d) for d in range(-L, R + 1)) for j in range(J)])
    ze = stencil(ye, w, L, Ns).reshape(Ns, J)
    _close(ze[L:], np.exp(1j * a * np.arange(L, Ns))[:, None] * resp[None, :], 1e-13, "exponential response")
    # zero history: the first outputs drop the taps before sample 0
    _close(ze[0], [w[j, L:] @ ye[: R + 1] for j in range(J)], 1e-13, "zero history")
    # Lagrange midpoint weights reproduce a cubic exactly, phase 0 returns the samples
    c = rand_c(rng, 4)
    t = np.arange(Ns + 2, dtype=float)
    yp = c[0] + c[1] * t + c[2] * t**2 + c[3] * t**3
    wi = np.array([[0, 1, 0, 0], [-1 / 16, 9 / 16, 9 / 16, -1 / 16]])
    zi = stencil(yp, wi, 1, Ns).reshape(Ns, 2)
    tm = t[1:Ns] + 0.5
    _close(zi[1:, 1], c[0] + c[1] * tm + c[2] * tm**2 + c[3] * tm**3, 1e-11, "cubic midpoint exact")
    _close(zi[:, 0], yp[:Ns], 1e-15, "phase 0")


def pin_lagrange(lagrange_weights, midpoint_stencil):
    # the textbook cubic midpoint weights (derived by hand in stencil_small.json)
    _close(lagrange_weights([-1, 0, 1, 2], 0.5), np.array([-1, 9, 9, -1]) / 16, 1e-15, "cubic midpoint weights")
    # at a node the weights pick that sample
    _close(lagrange_weights([-2, -1, 0, 1, 2], 1.0), [0, 0, 0, 1, 0], 1e-15, "node")
    # exact for every power x^k, k < T, at any offset
    rng = np.random.default_rng(42)
    nodes = np.array([-3, -1, 0, 2, 5], dtype=float)
    for x in rng.uniform(-3, 5, 4):
        wts = lagrange_weights(nodes, x)
        for k in range(nodes.shape[0]):
            _close(wts @ nodes**k, x**k, 1e-10, f"x^{k} at {x:.3f}")
    w, L = midpoint_stencil(1, 2)
    assert L == 1 and w.shape == (2, 4)
    _close(w[0], [0, 1, 0, 0], 0, "midpoint phase 0")
    _close(w[1], np.array([-1, 9, 9, -1]) / 16, 1e-15, "midpoint phase 1")
    # linear interpolation through offsets 0, 1
    w, L = midpoint_stencil(0, 1)
    _close(w, [[1, 0], [0.5, 0.5]], 1e-15, "linear midpoint")


# ------------------------------------------------------------------ R2R

def pin_real_conv(conv_real):
    """Real-data convolution (R2R): hand-worked fixture, library cross-check,
    brute force, closed forms."""
    d = load_golden("ols_boxcar_n4.json")
    _close(conv_real(np.asarray(d["s_re"], float), np.asarray(d["h_re"], float)),
           np.asarray(d["y_re"], float), 1e-14, "boxcar fixture")
    rng = np.random.default_rng(41)
    s = rng.standard_normal(300)
    h = rng.standard_normal((3, 17))
    y = conv_real(s, h)
    assert y.dtype == np.float64 and y.shape == (3, 300)
    for r in range(3):
        _close(y[r], np.convolve(s, h[r])[:300], 1e-12, "np.convolve")
    # brute force on a tiny case
    s = rng.standard_normal(9)
    h = rng.standard_normal((2, 4))
    want = np.zeros((2, 9))
    for r in range(2):
        for n in range(9):
            want[r, n] = sum(h[r, k] * s[n - k] for k in range(4) if n - k >= 0)
    _close(conv_real(s, h), want, 1e-14, "brute force")
    # delta filter is the identity; a shifted delta delays by the shift
    s = rng.standard_normal(50)
    e = np.zeros((1, 6))
    e[0, 5] = 1
    _close(conv_real(s, e)[0], np.concatenate([np.zeros(5), s[:45]]), 1e-15, "shifted delta")
