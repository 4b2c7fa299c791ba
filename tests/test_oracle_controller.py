"""Pins of the controller's oracle parts: the MLP gradient (finite differences,
closed-form special cases), the Adam update, the Gershgorin bounds (Gershgorin's
theorem, hand example) and the adaptive-m loop of Section 4.3."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as oarn
from oracle import features as ofeat
from oracle import methods as ometh
from oracle import mlp
from oracle import sketch as osk
from workloads import convdiff_csr, gaussian_rhs


def test_mlp_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    p = mlp.init_params(3) + 0.01 * rng.standard_normal(mlp.N_PARAMS)
    p[mlp.N_PARAMS - 3:] = rng.standard_normal(3)
    X = rng.standard_normal((8, mlp.N_IN))
    T = rng.standard_normal((8, mlp.N_OUT))
    _, g = mlp.loss_grad(p, X, T)
    h = 1e-6
    idx = rng.choice(mlp.N_PARAMS, 200, replace=False)
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        fd = (mlp.loss(p + e, X, T) - mlp.loss(p - e, X, T)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), i


def test_mlp_constant_output_closed_form():
    """W3 = 0: the output is b3 for every input; dL/db3 = 2 mean_b (b3 - t_b) / 3."""
    p = mlp.init_params(0)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    W3[:] = 0.0
    b3[:] = [1.0, -2.0, 0.5]
    X = np.random.default_rng(2).standard_normal((5, mlp.N_IN))
    T = np.arange(15, dtype=float).reshape(5, 3)
    Y, _ = mlp.forward(p, X)
    assert np.array_equal(Y, np.tile(b3, (5, 1)))
    L, g = mlp.loss_grad(p, X, T)
    assert L == pytest.approx(np.mean((b3 - T) ** 2))
    assert g[-3:] == pytest.approx(2.0 * (b3 - T).mean(axis=0) / 3.0)
    # with W3 = 0 nothing upstream receives a gradient
    assert np.all(g[:-3 - 3 * 64] == 0.0)


def test_mlp_dead_relu_blocks_gradient():
    p = mlp.init_params(4)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    b1[:] = -1e6   # every first-layer unit inactive
    X = np.random.default_rng(5).standard_normal((4, mlp.N_IN))
    T = np.ones((4, 3))
    _, g = mlp.loss_grad(p, X, T)
    n1 = 64 * 16 + 64 + 64 * 64
    assert np.all(g[:n1] == 0.0)


def test_adam_first_step_is_signed_learning_rate():
    """t = 1 from m = v = 0: p - lr g / (|g| + eps)."""
    g = np.array([3.0, -0.5, 0.0, 1e-3])
    p = np.zeros(4)
    q, m, v = mlp.adam_step(p, g, np.zeros(4), np.zeros(4), 1, lr=0.1, eps=1e-8)
    assert q == pytest.approx(-0.1 * g / (np.abs(g) + 1e-8))
    assert m == pytest.approx(0.1 * g) and v == pytest.approx(0.001 * g * g)


def test_gershgorin_hand_example_and_theorem():
    A = sp.csr_matrix(np.array([[4.0, -1.0, 0.5], [2.0, 6.0, 0.0], [0.0, -3.0, 1.0]]))
    lo, hi = ofeat.gershgorin_bounds(A)
    assert (lo, hi) == (-2.0, 8.0)   # rows: [2.5, 5.5], [4, 8], [-2, 4]
    rng = np.random.default_rng(6)
    for _ in range(5):
        M = rng.standard_normal((20, 20)) + 5 * np.eye(20)
        lo, hi = ofeat.gershgorin_bounds(M)
        ev = np.linalg.eigvals(M)
        assert np.all(ev.real >= lo - 1e-12) and np.all(ev.real <= hi + 1e-12)


def _problem(n=30, c=40.0, m=60, s=150):
    rp, col, val = convdiff_csr(n, 2, 1.0, c)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    return A, gaussian_rhs(N, 3), osk.sparse_sign_matrix(N, s, 8, 0)


def test_prefix_equals_shorter_run():
    A, b, S = _problem()
    big = oarn.truncated_arnoldi(A, b, 60, 2, S)
    small = oarn.truncated_arnoldi(A, b, 25, 2, S)
    pre = ometh._prefix(big, 25)
    for a, c in ((pre.V, small.V), (pre.SV, small.SV), (pre.SAV, small.SAV), (pre.H[:25, :24], small.H[:25, :24])):
        assert np.array_equal(a, c)


def test_relative_estimate_is_exact_difference_without_sketch():
    """S = I, k = m (orthonormal basis, eps = 0): the estimate is exactly
    ||f_m - f_prev|| / ||f_m||."""
    A, b, _ = _problem(n=12, s=144)
    N = b.size
    I = sp.identity(N, format="csr")
    arn = oarn.truncated_arnoldi(A, b, 30, 30, I)
    a20, a30 = ometh._prefix(arn, 20), ometh._prefix(arn, 30)
    r20, r30 = ometh.sfom_closed(a20, "invsqrt"), ometh.sfom_closed(a30, "invsqrt")
    est = ometh.relative_stopping_estimate(a30, r30.y, r20.y)
    truth = np.linalg.norm(r30.x - r20.x) / np.linalg.norm(r30.x)
    assert est == pytest.approx(truth, rel=1e-9)


def test_adaptive_m_stops_at_first_passing_checkpoint_and_is_monotone():
    A, b, S = _problem(m=120, s=300)
    stops = []
    for tol in (1e-3, 1e-5, 1e-7):
        res, m_stop, est = ometh.adaptive_m(A, b, "invsqrt", 2, S, 10, 5, 120, tol)
        assert est <= tol
        direct = ometh.sfom_closed(oarn.truncated_arnoldi(A, b, m_stop, 2, S), "invsqrt")
        assert np.allclose(res.x, direct.x, rtol=0, atol=1e-12 * np.linalg.norm(direct.x))
        prev = ometh.sfom_closed(oarn.truncated_arnoldi(A, b, m_stop - 5, 2, S), "invsqrt")
        if m_stop - 5 > 10:   # the checkpoint before did not pass
            pprev = ometh.sfom_closed(oarn.truncated_arnoldi(A, b, m_stop - 10, 2, S), "invsqrt")
            arn_p = ometh._prefix(oarn.truncated_arnoldi(A, b, m_stop - 5, 2, S), m_stop - 5)
            assert ometh.relative_stopping_estimate(arn_p, prev.y, pprev.y) > tol
        stops.append(m_stop)
    assert stops == sorted(stops)
