"""Pins for the Gauss-Chebyshev rule and adaptive order sequence (Section 4.1, 5.1)."""
import numpy as np
import pytest

from oracle import quadrature as quad


def test_order_sequence_contains_printed_orders(golden):
    g = golden("quadrature_orders.txt")
    seq = quad.order_sequence()
    assert int(g["order_sec51"][0]) in seq
    assert int(g["order_sec53"][0]) in seq
    assert seq[:7] == [32, 45, 63, 89, 125, 176, 248]
    for a, b in zip(seq[1:], seq[2:]):
        assert b == int(np.floor(np.sqrt(2.0) * a))


def test_chebyshev_nodes_integrate_polynomials():
    """First-kind Gauss-Chebyshev is exact for T_j, j < 2l: sum T_j(x_i) = 0."""
    l = 17
    t, w = quad.gauss_chebyshev_invsqrt(l)
    x = (1 - t) / (1 + t)
    assert np.allclose((2.0 / l) / (1 + x), w)
    for j in range(1, 2 * l):
        assert abs(np.sum(np.cos(j * np.arccos(x)))) < 1e-12
    assert abs(np.sum(np.cos(2 * l * np.arccos(x))) + l) < 1e-10


@pytest.mark.parametrize("l", [32, 45, 63])
def test_rule_reproduces_invsqrt(l):
    z = np.logspace(-1, 1, 101)
    err = np.abs(quad.scalar_invsqrt_rule(z, l) - z ** -0.5) * np.sqrt(z)
    assert err.max() < 2e-15 * l


def test_scaling_is_exact_identity():
    z = np.array([3e3, 7e4, 2.5e5])
    sigma = np.sqrt(3e3 * 2.5e5)
    approx = quad.scalar_invsqrt_rule(z, 176, sigma)
    assert np.max(np.abs(approx * np.sqrt(z) - 1)) < 1e-13


def test_complex_right_half_plane_converges():
    z = np.array([1 + 2j, 0.5 - 0.3j, 4 + 4j])
    exact = 1 / np.sqrt(z)  # principal branch
    approx = quad.scalar_invsqrt_rule(z, 176)
    assert np.max(np.abs(approx - exact) / np.abs(exact)) < 1e-12


def test_rule_is_integral_of_measure():
    """w_i/(t_i + z) approximates int (t+z)^-1 t^-1/2 dt / pi computed by scipy."""
    from scipy.integrate import quad as squad
    z = 2.7
    exact, _ = squad(lambda t: 1.0 / ((t + z) * np.sqrt(t) * np.pi), 0, np.inf, limit=200)
    assert abs(quad.scalar_invsqrt_rule(np.array([z]), 63)[0] - exact) < 1e-9


def _rule_from_diffs(diffs):
    """eval_rule whose consecutive results differ (relatively) by the given amounts,
    indexed by the order sequence 32, 45, 63, ..."""
    orders = [32]
    while len(orders) < len(diffs) + 1:
        orders.append(quad.next_order(orders[-1]))
    vals = {orders[0]: np.array([1.0, 0.0])}
    for l_prev, l, d in zip(orders, orders[1:], diffs):
        vals[l] = vals[l_prev] + np.array([0.0, d])   # ||q_l - q_prev|| / ||q_l|| ~ d
    return lambda l: vals[l], orders


def test_adaptive_accepts_at_tolerance():
    from oracle.methods import _adaptive
    rule, orders = _rule_from_diffs([1e-2, 1e-5, 1e-9, 1e-14, 1e-15])
    _, l = _adaptive(rule, 1e-13, 32, 45, 10_000)
    assert l == orders[4]          # first difference below 1e-13


def test_adaptive_accepts_at_rounding_floor():
    """Differences stop falling at 3e-13 (above tol = 1e-13): the order where the
    decrease stops (d > d_prev / 2, d <= 1e-10) is accepted."""
    from oracle.methods import QUAD_FLOOR, _adaptive
    rule, orders = _rule_from_diffs([1e-2, 1e-5, 1e-9, 4e-13, 3e-13, 5e-13, 2e-13])
    _, l = _adaptive(rule, 1e-13, 32, 45, 10_000)
    assert l == orders[5]
    assert 3e-13 <= QUAD_FLOOR


def test_adaptive_no_floor_acceptance_above_floor():
    """A stagnation above the floor is a failure, not convergence."""
    from oracle.methods import QuadratureError, _adaptive
    rule, orders = _rule_from_diffs([1e-2, 1e-5, 1e-6, 1e-6, 1e-6, 1e-6])
    with pytest.raises(QuadratureError):
        _adaptive(rule, 1e-13, 32, 45, orders[-1])


def test_adaptive_final_order_below_floor_is_accepted():
    """Still falling fast, but the sequence ends (l_max): below the floor is accepted
    at the last order, above it is a failure."""
    from oracle.methods import QUAD_FLOOR, QuadratureError, _adaptive
    rule, orders = _rule_from_diffs([1e-2, 1e-6, 1e-9, 4e-11])
    _, l = _adaptive(rule, 1e-13, 32, 45, orders[4])
    assert l == orders[4] and 4e-11 <= QUAD_FLOOR
    rule, orders = _rule_from_diffs([1e-2, 1e-6, 1e-9, 4e-10])
    with pytest.raises(QuadratureError):
        _adaptive(rule, 1e-13, 32, 45, orders[4])


def test_adaptive_fast_decrease_is_not_stagnation():
    """Below the floor but still falling faster than 2x per order: keep refining."""
    from oracle.methods import _adaptive
    rule, orders = _rule_from_diffs([1e-2, 1e-6, 1e-11, 1e-12, 9e-14])
    _, l = _adaptive(rule, 1e-13, 32, 45, 10_000)
    assert l == orders[5]


def test_reference_invsqrt_matches_dense():
    """The sparse-direct reference A^(-1/2) b equals the dense Schur square root on a
    small grid of the paper's operator family."""
    import scipy.linalg as sla
    import scipy.sparse as sp
    from oracle import reference
    from workloads import convdiff_csr, ones_rhs
    rp, col, val = convdiff_csr(12, 2, 1e-3, 1.0, paper_direction=True)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = ones_rhs(N)
    ref = np.real(np.linalg.solve(sla.sqrtm(A.toarray()), b))
    x = reference.invsqrt_apply(A, b, tol=1e-13)
    assert np.linalg.norm(x - ref) / np.linalg.norm(ref) < 1e-11
