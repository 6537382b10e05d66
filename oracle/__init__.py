"""CPU oracle for overlap-and-save (OLS) convolution -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously correct reference that the HIP path
is checked against.  Only the test suite, the smoke check in the repository's
entry module and the CPU-baseline leg of the benchmark may import it.  The
product path (the C-ABI library and its Python binding) never imports, links or
calls anything here, and nothing here imports the product package: the two
share no code.  The only thing both sides use is the seeded input generator in
``workloads.py``, which contains none of the method's arithmetic.

Everything is computed in float64 / complex128.

What is here (paper: Adamek, Dimoudi, Giles, Armour, "GPU Fast Convolution via
the Overlap-and-Save Method in Shared Memory"):

* ``conv.direct_conv``     -- eq. (1), discrete linear convolution, zero history.
* ``conv.direct_conv_at``  -- eq. (1) evaluated at chosen output indices only.
* ``conv.direct_conv_loops`` -- eq. (1) as explicit Python loops (tiny inputs).
* ``conv.direct_conv_real`` / ``direct_conv_real_at`` -- eq. (1) for a real
  signal and real filters (R2R), float64.
* ``conv.fft`` / ``conv.ifft`` -- hand-written iterative radix-2 Cooley-Tukey
  FFT with explicit bit reversal (the FFT named in the introduction and sec. 3.4).
* ``conv.dft``             -- the O(N^2) DFT definition (tiny inputs).
* ``conv.full_fft_conv``   -- eq. (2) with the zero padding its footnote asks
  for (length >= N_s + M - 1).
* ``conv.ols_conv``        -- overlap-and-save as described in sec. 3.2 and
  Alg. 2: overlapping segments, forward FFT, point-wise product with each
  filter spectrum, inverse FFT, discard of the M-1 aliased samples.
* ``adjoint``              -- the adjoint (gradient) of eq. (1) with respect to
  the signal and to the filters, by direct correlation.
* ``post``                 -- post-processing of the output (sec. 4): the
  power |y|^2, the numerical derivative (backward difference) and the
  non-local stencil with J outputs per sample (derivative, Lagrange
  interpolation) applied to eq. (1)'s output and its tail.

Every function is pinned by tests in ``tests/test_oracle*.py`` against things
other than itself: hand-derived fixtures under ``tests/golden/``, closed forms
(delta, shift, boxcar, complex exponential), Parseval, brute force on tiny
inputs, numpy's own FFT/convolve as library cross-checks, and the invariance of
the OLS result under the segment length (sec. 3.2).
"""

from . import conv, adjoint, post  # noqa: F401
