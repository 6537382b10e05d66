"""The C loops of the oracle (oracle/adjoint_loops.c) pinned to the paper's
definitions: brute force on tiny inputs (including the edge cases N_s < M,
M = 1, N_s = 1), the adjoint identities with eq. (1), exact finite
differences, the closed forms of eq. (1), and the numpy definitions at
medium size.  No GPU needed."""

import numpy as np
import pytest

from oracle import adjoint, conv, loops
import oracle_pins as P
import workloads


@pytest.fixture(scope="module", autouse=True)
def built():
    if not loops.available():
        loops.build()


TINY = [(1, 1, 1), (7, 2, 3), (5, 3, 9), (40, 4, 1), (64, 2, 16), (33, 1, 33)]


@pytest.mark.parametrize("Ns,K,M", TINY)
def test_loops_vs_bruteforce(Ns, K, M):
    rng = np.random.default_rng(Ns * 100 + K * 10 + M)
    s = P.rand_c(rng, Ns)
    h = P.rand_c(rng, K, M)
    g = P.rand_c(rng, K, Ns)
    P._close(loops.direct_conv(s, h), conv.direct_conv_loops(s, h), 1e-13, "eq. (1)")
    P._close(loops.grad_signal(g, h), adjoint.grad_signal_loops(g, h), 1e-13, "ds")
    P._close(loops.grad_filters(g, s, M), adjoint.grad_filters_loops(g, s, M), 1e-13, "dh")


def test_loops_conv_golden_and_closed_forms():
    P.pin_conv_golden(loops.direct_conv)
    P.pin_conv_bruteforce(loops.direct_conv)
    P.pin_conv_closed_forms(loops.direct_conv)
    P.pin_conv_linearity(loops.direct_conv)


def test_loops_adjoint_identities():
    P.pin_adjoint_dot_product(loops.direct_conv, loops.grad_signal, loops.grad_filters)
    P.pin_adjoint_finite_differences(loops.direct_conv, loops.grad_signal, loops.grad_filters)


def test_loops_vs_numpy_definitions_medium():
    """Sizes that span several of the C code's output blocks (4096 for ds, the
    sum over n in blocks of 16384 for dh) with ragged ends."""
    Ns, K, M = 40001, 3, 300
    s, h = workloads.make_signal_filters(Ns, K, M, seed=17)
    g = workloads.make_grad(K, Ns, seed=17)
    P._close(loops.grad_signal(g, h), adjoint.grad_signal(g, h), 1e-11, "ds")
    P._close(loops.grad_filters(g, s, M), adjoint.grad_filters(g, s, M), 1e-11, "dh")
    P._close(loops.direct_conv(s, h), conv.direct_conv(s, h), 1e-11, "eq. (1)")


def test_loops_reject_shape_mismatch():
    with pytest.raises(ValueError):
        loops.grad_signal(np.zeros((2, 5)), np.zeros((3, 2)))
    with pytest.raises(ValueError):
        loops.grad_filters(np.zeros((2, 5)), np.zeros(4), 2)
