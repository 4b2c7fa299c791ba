"""Pins for the ill-conditioned-R remedy of Section 2.1 (remark after eq. sFOM''').

The oracle replaces R_m^-1 by the truncated QR pseudoinverse in basis order:
the approximant is formed from the longest prefix of the basis whose sketched
basis has a Frobenius condition number of at most COND_MAX.  In exact
arithmetic the sketched approximants depend only on span(V_m) (Section 2.1), so
the fully orthogonalised basis (k = m), whose sketch stays well conditioned,
fixes what the truncated basis (k = 2) must give once it has converged.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as arn_mod
from oracle import methods, sketch
from workloads import convdiff_csr, gaussian_rhs


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def conv2d_m300():
    """2D convection-diffusion n = 100, m = 300, s = 600: the k = 2 basis becomes
    numerically dependent after convergence (cond(SV_m) ~ 1e16)."""
    rp, col, val = convdiff_csr(100, 2, 1.0, 50.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = gaussian_rhs(N, 0)
    S = sketch.sparse_sign_matrix(N, 600, 8, 0)
    a2 = arn_mod.truncated_arnoldi(A, b, 300, 2, S)
    am = arn_mod.truncated_arnoldi(A, b, 300, 300, S)
    return a2, am


def test_case_is_ill_conditioned(conv2d_m300):
    a2, am = conv2d_m300
    assert np.linalg.cond(a2.SV) > 1e15
    assert np.linalg.cond(am.SV) < 1e8
    assert methods.conditioned_prefix(am) == 300


@pytest.mark.parametrize("f,tau", [("invsqrt", 0.0), ("exp", 0.01)])
def test_truncated_k2_equals_full_orthogonalisation(conv2d_m300, f, tau):
    """Section 2.1 basis independence restored by the remedy: k = 2 (truncated at
    its conditioned prefix) equals k = m (no truncation needed)."""
    a2, am = conv2d_m300
    r2 = methods.sfom_closed(a2, f, tau)
    rm = methods.sfom_closed(am, f, tau)
    assert r2.m_used < 300 and rm.m_used == 300
    assert rel(r2.x, rm.x) < 1e-10


def test_sgmres_truncated_k2_equals_full_orthogonalisation(conv2d_m300):
    a2, am = conv2d_m300
    assert rel(methods.sgmres(a2, "invsqrt").x, methods.sgmres(am, "invsqrt").x) < 1e-10


def test_without_remedy_exp_is_not_determined(conv2d_m300):
    """The case needs the remedy: R^-1 taken literally gives an exp(-0.01 A) b
    whose norm is off by orders of magnitude."""
    a2, am = conv2d_m300
    full = methods.sfom_closed(am, "exp", 0.01).x
    w = methods.whiten(a2)
    import scipy.linalg as sla
    g = sla.expm(-0.01 * w.M) @ w.c
    x_lit = a2.V @ sla.solve_triangular(w.R, g)
    assert rel(x_lit, full) > 1.0


def test_prefix_conditions_match_definition():
    """kappa_F of every leading block, from the prefix sums, equals the definition
    ||R_j||_F ||R_j^-1||_F computed block by block."""
    rng = np.random.default_rng(7)
    m = 40
    R = np.triu(rng.standard_normal((m, m))) + np.diag(np.logspace(0, -9, m))
    c = methods.prefix_conditions(R)
    ref = np.array([np.linalg.cond(R[:j, :j], "fro") for j in range(1, m + 1)])
    assert np.allclose(c, np.maximum.accumulate(ref), rtol=1e-8)
    assert np.all(np.diff(ref) >= -1e-9 * ref[1:])   # the definition itself never decreases


def test_remedy_is_identity_when_conditioned():
    rp, col, val = convdiff_csr(12, 2, 1.0, 50.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = gaussian_rhs(N, 0)
    S = sketch.sparse_sign_matrix(N, 64, 8, 0)
    arn = arn_mod.truncated_arnoldi(A, b, 20, 2, S)
    reg, mp = methods.regularize(arn)
    assert reg is arn and mp == 20
