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
