"""The pins must catch plausible mistakes planted in (copies of) the oracle.

Every mutant below is a copy of an oracle routine with one planted mistake (a
wrong sign, a dropped term, an off-by-one index, a transposed operand).  Each
must fail at least one pin.  CPU only; nothing here touches the GPU path.
"""

import numpy as np
import pytest

from oracle import adjoint, conv
import oracle_pins as P


def _fft_mutant(sign_flip=False, skip_bitrev=False, twiddle_half=False):
    def core(x, sign):
        x = np.asarray(x, dtype=np.complex128)
        N = x.shape[-1]
        if N & (N - 1):
            raise ValueError
        if sign_flip:
            sign = -sign
        y = x.copy() if skip_bitrev else x[..., conv._bit_reverse_indices(N)].copy()
        m = 2
        while m <= N:
            half = m // 2
            k = np.arange(half)
            w = np.exp(sign * 2j * np.pi * k / (2 * m if twiddle_half else m))
            b = y.reshape(y.shape[:-1] + (N // m, m))
            u = b[..., :half].copy()
            t = b[..., half:] * w
            b[..., :half] = u + t
            b[..., half:] = u - t
            y = b.reshape(y.shape)
            m *= 2
        return y
    return (lambda x: core(x, -1.0)), (lambda X: core(X, 1.0) / np.shape(X)[-1])


def _ols_mutant(discard_shift=0, compound=False, no_history=False, hop_fix=0):
    def ols(s, h, N, hop=None):
        s = np.asarray(s, dtype=np.complex128)
        h = np.atleast_2d(np.asarray(h, dtype=np.complex128))
        K, M = h.shape
        Ns = s.shape[0]
        L = N - M + 1
        H = (L if hop is None else hop) + hop_fix
        H = max(H, 1)
        y = np.zeros((K, Ns), dtype=np.complex128)
        if Ns == 0:
            return y
        nseg = -(-Ns // H)
        F = np.fft.fft(np.concatenate([h, np.zeros((K, N - M))], axis=1))
        hist = 0 if no_history else M - 1
        xp = np.zeros((nseg - 1) * H + N + M, dtype=np.complex128)
        xp[hist:hist + Ns] = s
        segs = xp[np.arange(nseg)[:, None] * H + np.arange(N)[None, :]]
        A = np.fft.fft(segs)
        d = M - 1 + discard_shift
        for r in range(K):
            if compound:
                A = A * F[r]
                a = np.fft.ifft(A)
            else:
                a = np.fft.ifft(A * F[r])
            out = a[:, d:d + H]
            if out.shape[1] < H:
                out = np.concatenate([out, np.zeros((nseg, H - out.shape[1]))], axis=1)
            y[r] = out.reshape(-1)[:Ns]
        return y
    return ols


def _expect_caught(*checks):
    caught = 0
    for fn in checks:
        try:
            fn()
        except (AssertionError, ValueError, IndexError):
            caught += 1
    assert caught > 0, "planted mistake was not caught by any pin"


@pytest.mark.parametrize("kw", [dict(sign_flip=True), dict(skip_bitrev=True), dict(twiddle_half=True)])
def test_fft_mutants_caught(kw):
    f, fi = _fft_mutant(**kw)
    _expect_caught(lambda: P.pin_fft_golden(f), lambda: P.pin_fft_vs_bruteforce(f),
                   lambda: P.pin_fft_closed_forms(f))


def test_fft_mutant_control():
    f, fi = _fft_mutant()
    P.pin_fft_golden(f)
    P.pin_fft_vs_bruteforce(f)
    P.pin_ifft_roundtrip(f, fi)


def _conv_correlation(s, h):
    s = np.asarray(s, dtype=np.complex128)
    h = np.atleast_2d(h)
    K, M = h.shape
    Ns = len(s)
    y = np.zeros((K, Ns), dtype=np.complex128)
    for r in range(K):
        for n in range(Ns):
            for k in range(M):
                if n + k < Ns:
                    y[r, n] += s[n + k] * h[r, k]
    return y


def _conv_dropped_tap(s, h):
    h = np.atleast_2d(np.asarray(h, dtype=np.complex128)).copy()
    h[:, -1] = 0
    return conv.direct_conv(s, h)


def _conv_transposed_filter(s, h):
    return conv.direct_conv(s, np.atleast_2d(h)[:, ::-1])


def _conv_conjugated(s, h):
    return conv.direct_conv(s, np.conj(np.atleast_2d(h)))


@pytest.mark.parametrize("mut", [_conv_correlation, _conv_dropped_tap, _conv_transposed_filter, _conv_conjugated])
def test_conv_mutants_caught(mut):
    _expect_caught(lambda: P.pin_conv_golden(mut), lambda: P.pin_conv_bruteforce(mut),
                   lambda: P.pin_conv_closed_forms(mut))


@pytest.mark.parametrize("kw", [dict(discard_shift=-1), dict(discard_shift=1), dict(compound=True),
                                dict(no_history=True), dict(hop_fix=1)])
def test_ols_mutants_caught(kw):
    ols = _ols_mutant(**kw)
    _expect_caught(lambda: P.pin_ols_golden(ols), lambda: P.pin_ols_matches_definition(ols, None),
                   lambda: P.pin_ols_filters_independent(ols), lambda: P.pin_ols_segment_invariance(ols))


def test_ols_mutant_control():
    ols = _ols_mutant()
    P.pin_ols_golden(ols)
    P.pin_ols_matches_definition(ols, None)
    P.pin_ols_filters_independent(ols)


def _ds_no_conj(g, h):
    return adjoint.grad_signal(g, np.conj(h))


def _ds_wrong_dir(g, h):
    g = np.asarray(g)
    K, Ns = g.shape
    out = np.zeros(Ns, dtype=np.complex128)
    y = conv.direct_conv(np.zeros(Ns), h)  # placeholder shape
    for r in range(K):
        out += conv.direct_conv(g[r], np.conj(h[r:r + 1]))[0]  # convolution instead of correlation
    return out + 0 * y[0]


def _dh_shift(g, s, M):
    s = np.asarray(s)
    return adjoint.grad_filters(g, np.concatenate([s[1:], [0]]), M)


@pytest.mark.parametrize("ds,dh", [(_ds_no_conj, adjoint.grad_filters), (_ds_wrong_dir, adjoint.grad_filters),
                                   (adjoint.grad_signal, _dh_shift)])
def test_adjoint_mutants_caught(ds, dh):
    _expect_caught(lambda: P.pin_adjoint_dot_product(conv.direct_conv, ds, dh),
                   lambda: P.pin_adjoint_finite_differences(conv.direct_conv, ds, dh))


def _fails(fn, *args):
    try:
        fn(*args)
    except AssertionError:
        return True
    return False


def _deriv_forward(y):
    y = np.asarray(y, dtype=np.complex128)
    d = np.zeros_like(y)
    d[..., :-1] = y[..., 1:] - y[..., :-1]
    return d


def _deriv_sign(y):
    y = np.asarray(y, dtype=np.complex128)
    d = y.copy()
    d[..., 1:] += y[..., :-1]
    return d


def _deriv_wrap(y):
    y = np.asarray(y, dtype=np.complex128)
    return y - np.roll(y, 1, axis=-1)


def _deriv_no_first(y):
    y = np.asarray(y, dtype=np.complex128)
    d = np.zeros_like(y)
    d[..., 1:] = y[..., 1:] - y[..., :-1]
    return d


@pytest.mark.parametrize("mutant", [_deriv_forward, _deriv_sign, _deriv_wrap, _deriv_no_first])
def test_derivative_mutants_fail(mutant):
    from oracle import post
    assert (_fails(P.pin_post_golden, post.power, mutant, conv.direct_conv)
            or _fails(P.pin_derivative_closed_forms, mutant, conv.direct_conv))


@pytest.mark.parametrize("mutant", [
    lambda y: np.asarray(y).real ** 2,
    lambda y: np.abs(np.asarray(y)),
    lambda y: (np.asarray(y) ** 2).real,
])
def test_power_mutants_fail(mutant):
    from oracle import post
    assert (_fails(P.pin_post_golden, mutant, post.derivative, conv.direct_conv)
            or _fails(P.pin_power_closed_forms, mutant))


def _real_corr(s, h):
    # correlation instead of convolution (filter not reversed)
    s = np.asarray(s, float)
    h = np.atleast_2d(np.asarray(h, float))
    K, M = h.shape
    padded = np.concatenate([np.zeros(M - 1), s])
    win = np.lib.stride_tricks.sliding_window_view(padded, M)
    return (win @ h.T).T


def _real_no_history(s, h):
    s = np.asarray(s, float)
    h = np.atleast_2d(np.asarray(h, float))
    y = conv.direct_conv_real(s, h)
    y[:, : h.shape[1] - 1] = 0
    return y


@pytest.mark.parametrize("mutant", [_real_corr, _real_no_history])
def test_real_conv_mutants_fail(mutant):
    assert _fails(P.pin_real_conv, mutant)


# ---------------------------------------------------------- stencil mutants

def _stencil_mutant(flip_d=False, transpose_phases=False, shift_tap=0, wrap_history=False):
    def stencil(y, w, left, Ns):
        y = np.asarray(y, dtype=np.complex128)
        w = np.atleast_2d(np.asarray(w, dtype=np.float64))
        J, T = w.shape
        right = T - 1 - left
        z = np.zeros(y.shape[:-1] + (Ns, J), dtype=np.complex128)
        for j in range(J):
            for d in range(-left, right + 1):
                dd = -d if flip_d else d + shift_tap
                for n in range(Ns):
                    m = n + dd
                    if m < 0 and not wrap_history:
                        continue
                    if m >= y.shape[-1]:
                        continue
                    z[..., n, j] += w[j, d + left] * y[..., m]
        if transpose_phases:
            return np.moveaxis(z, -1, -2).reshape(y.shape[:-1] + (J * Ns,))
        return z.reshape(y.shape[:-1] + (J * Ns,))
    return stencil


def _conv_stencil_with(stencil, zero_tail=False):
    def conv_stencil(s, h, w, left):
        s = np.asarray(s, dtype=np.complex128).ravel()
        R = np.atleast_2d(w).shape[1] - 1 - left
        if zero_tail:
            y = conv.direct_conv(s, h)
            y = np.concatenate([y, np.zeros((y.shape[0], R))], axis=1)
        else:
            y = conv.direct_conv(np.concatenate([s, np.zeros(R)]), h)
        return stencil(y, w, left, s.shape[0])
    return conv_stencil


@pytest.mark.parametrize("kw", [dict(flip_d=True), dict(transpose_phases=True), dict(shift_tap=1),
                                dict(shift_tap=-1), dict(wrap_history=True)])
def test_stencil_mutants_fail(kw):
    from oracle import post
    m = _stencil_mutant(**kw)
    assert (_fails(P.pin_stencil_golden, m, _conv_stencil_with(m))
            or _fails(P.pin_stencil_closed_forms, m, post.derivative))


def test_stencil_zero_tail_mutant_fails():
    from oracle import post
    assert _fails(P.pin_stencil_golden, post.stencil, _conv_stencil_with(post.stencil, zero_tail=True))


def test_unmutated_stencil_copy_passes():
    from oracle import post
    m = _stencil_mutant()
    P.pin_stencil_golden(m, _conv_stencil_with(m))
    P.pin_stencil_closed_forms(m, post.derivative)


def _lagrange_mutant(swap=False, skip_last=False):
    def weights(nodes, x):
        t = np.asarray(nodes, dtype=np.float64)
        out = np.ones(t.shape[0])
        for k in range(t.shape[0]):
            for i in range(t.shape[0] - (1 if skip_last else 0)):
                if i != k:
                    out[k] *= (x - t[i]) / ((t[i] - t[k]) if swap else (t[k] - t[i]))
        return out
    return weights


@pytest.mark.parametrize("kw", [dict(swap=True), dict(skip_last=True)])
def test_lagrange_mutants_fail(kw):
    from oracle import post
    assert _fails(P.pin_lagrange, _lagrange_mutant(**kw), post.midpoint_interpolation_stencil)
