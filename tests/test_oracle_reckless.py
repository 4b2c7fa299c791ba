"""Pins of the s-adaptive solve (methods.solve_reckless) and of the Cortinovis-
Kressner form's interpolation property.

* s-adaptivity: on a batched-workload problem whose sketched Ritz values reach the
  branch cut at s = 2m, doubling s once gives an admissible projected matrix, and
  the result equals the fixed-s solve at that s; a problem that is fine at s0
  returns at s0 with the fixed-s result; the loop stops at s_max.
* Corollary (interp) in Section 2.2: the sketched FOM approximant (the form
  V_m f(H_hat) ||b|| e_1 of the Cortinovis-Kressner remark) equals q(A) b for the
  polynomial q of degree m-1 that interpolates f at the eigenvalues of H_hat,
  evaluated here in Newton form with A itself -- a route that shares nothing
  with the whitening or with f(M).
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as oarn
from oracle import methods as ometh
from oracle import sketch as osk
from workloads import batched_problem_params, convdiff_csr, gaussian_rhs


def batch_pair(pi, r):
    q = batched_problem_params(64)[pi]
    rp, col, val = convdiff_csr(q["n"], 2, 1.0, q["c"])
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = np.random.default_rng(q["rhs_seedseq"]).standard_normal((4, N))[r]
    return A, b, q


def test_reckless_recovers_branch_failure():
    A, b, q = batch_pair(7, 1)
    res, s_used, trail = ometh.solve_reckless(A, b, "invsqrt", q["m"], 2, q["s"], min(4 * q["s"], 1024),
                                              seed=q["sketch_seed"])
    assert [t[1] for t in trail] == ["branch", "ok"]
    assert s_used == 2 * q["s"]
    S = osk.sparse_sign_matrix(A.shape[0], s_used, 8, q["sketch_seed"])
    fixed = ometh.sfom_closed(oarn.truncated_arnoldi(A, b, q["m"], 2, S), "invsqrt")
    assert np.array_equal(res.x, fixed.x)


def test_reckless_keeps_good_s_and_caps():
    rp, col, val = convdiff_csr(30, 2, 1.0, 50.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = gaussian_rhs(N, 1)
    res, s_used, trail = ometh.solve_reckless(A, b, "invsqrt", 40, 2, 120, 480, seed=2)
    assert s_used == 120 and len(trail) == 1
    # an unreachable monitor threshold walks s up to the cap and stops there
    res, s_used, trail = ometh.solve_reckless(A, b, "invsqrt", 40, 2, 60, 200, eps_max=1e-6, seed=2)
    assert [t[0] for t in trail] == [60, 120, 200] and s_used == 200
    assert all(t[1] == "eps" for t in trail)


def newton_interp_apply(A, b, nodes, f):
    """q(A) b for the interpolant of f at the (distinct) nodes, Newton form; complex
    nodes come in conjugate pairs, so the result is real up to rounding."""
    x = np.asarray(nodes, dtype=np.complex128)
    c = f(x).astype(np.complex128)
    n = x.size
    for j in range(1, n):  # divided differences
        c[j:] = (c[j:] - c[j - 1:-1]) / (x[j:] - x[:-j])
    v = b.astype(np.complex128)
    acc = c[0] * v
    for j in range(1, n):
        v = A @ v - x[j - 1] * v
        acc = acc + c[j] * v
    return acc


@pytest.mark.parametrize("f,tau,m", [("exp", 0.5, 6), ("invsqrt", 0.0, 7), ("exp", 0.2, 8)])
def test_cortinovis_form_interpolates_at_hhat_eigenvalues(f, tau, m):
    rp, col, val = convdiff_csr(8, 2, 1.0, 5.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N)) / 30.0
    b = gaussian_rhs(N, 5)
    S = osk.sparse_sign_matrix(N, 24, 8, 3)
    arn = oarn.truncated_arnoldi(A, b, m, 2, S, extend=True)
    arn.S = S
    mm = arn.m_used
    Sv = S @ arn.v_next
    xhat = np.linalg.lstsq(arn.SV, Sv, rcond=None)[0]
    Hhat = arn.H[:mm, :mm].copy()
    Hhat[:, mm - 1] += arn.H[mm, mm - 1] * xhat
    nodes = np.linalg.eigvals(Hhat)
    fz = (lambda z: np.exp(-tau * z)) if f == "exp" else (lambda z: 1.0 / np.sqrt(z))
    q = newton_interp_apply(A, b, nodes, fz)
    assert np.max(np.abs(q.imag)) < 1e-8 * np.linalg.norm(q)
    x_ck = ometh.cortinovis_form(arn, f, tau)
    x_cl = ometh.sfom_closed(arn, f, tau).x
    assert np.linalg.norm(q.real - x_ck) / np.linalg.norm(x_ck) < 1e-9
    assert np.linalg.norm(x_cl - x_ck) / np.linalg.norm(x_ck) < 1e-10


def test_interpolation_pin_rejects_uncorrected_hessenberg():
    """Planted mistake: interpolating at the eigenvalues of H_m (the Arnoldi matrix
    without the sketched correction x_hat) does not reproduce the approximant."""
    rp, col, val = convdiff_csr(8, 2, 1.0, 5.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N)) / 30.0
    b = gaussian_rhs(N, 5)
    S = osk.sparse_sign_matrix(N, 24, 8, 3)
    arn = oarn.truncated_arnoldi(A, b, 7, 2, S, extend=True)
    arn.S = S
    q = newton_interp_apply(A, b, np.linalg.eigvals(arn.H[:7, :7]), lambda z: np.exp(-0.5 * z))
    x_ck = ometh.cortinovis_form(arn, "exp", 0.5)
    assert np.linalg.norm(q.real - x_ck) / np.linalg.norm(x_ck) > 1e-6
