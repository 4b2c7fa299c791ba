"""Pins of the oracle's contour quadrature for exp(-tau A) b (oracle/contour.py).

* The rule with the exact resolvent reproduces exp(-tau A) b (dense expm) on a
  convection-diffusion operator, on a nonnormal matrix with complex spectrum and
  on a diagonal matrix (closed form exp(-tau lambda)): this fixes the nodes, the
  weights, the orientation of the contour and the conjugate-symmetry folding.
* With S = I and the full Krylov space (k = m = N) sketched GMRES is exact, so
  its contour form must equal expm.
* Sketched FOM by the contour rule equals the closed form exp(-tau M) c
  (SciPy's expm, another algorithm).
* Sketched GMRES with S = I and full orthogonalisation (k = m < N) equals the
  same rule applied to least-squares solutions computed from an orthonormal
  basis of the Krylov space made independently (QR of the Krylov matrix), with
  no whitening.
* The chosen parabola encloses every relevant negated Ritz value.
* Mutations (weights conjugated, wrong sign of t') fail the first pin.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import arnoldi as oarn
from oracle import contour as C
from oracle import methods as ometh
from oracle import sketch as osk
from workloads import convdiff_csr, gaussian_rhs


def dense_convdiff(n, conv):
    rp, col, val = convdiff_csr(n, 2, 1.0, conv)
    N = rp.size - 1
    return sp.csr_matrix((val, col, rp), shape=(N, N))


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


def nonnormal(n, seed):
    """Upper triangular plus a rotation block: complex eigenvalues in the right
    half-plane, strongly nonnormal."""
    rng = np.random.default_rng(seed)
    T = np.triu(rng.standard_normal((n, n)), 1) * 2.0
    d = 1.0 + 20.0 * rng.random(n)
    T[np.arange(n), np.arange(n)] = d
    for i in range(0, n - 1, 4):  # 2x2 rotation blocks: eigenvalues d_i +- i w
        T[i + 1, i] = -(3.0 + i)
        T[i, i + 1] = 3.0 + i
        T[i + 1, i + 1] = T[i, i]
    Qm, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return Qm @ T @ Qm.T


@pytest.mark.parametrize("case,tau", [("convdiff", 1e-2), ("convdiff", 1e-3), ("nonnormal", 0.1),
                                      ("diag", 0.5)])
def test_resolvent_rule_reproduces_expm(case, tau):
    if case == "convdiff":
        A = dense_convdiff(12, 50.0).toarray()
    elif case == "nonnormal":
        A = nonnormal(24, 1)
    else:
        A = np.diag(np.linspace(0.1, 40.0, 30))
    b = gaussian_rhs(A.shape[0], 1)
    ref = sla.expm(-tau * A) @ b if case != "diag" else np.exp(-tau * np.diag(A)) * b
    theta = np.linalg.eigvals(A)
    a, c, tm = C.parabola(theta, tau)
    assert C.encloses(theta, tau, a, c)
    x = C.resolvent_rule(A, b, tau, a, c, tm, 256)
    assert rel(x, ref) < 1e-12


def test_parabola_encloses_with_margin():
    rng = np.random.default_rng(3)
    theta = rng.uniform(1, 500, 40) + 1j * rng.uniform(-80, 80, 40)
    theta = np.concatenate([theta, theta.conj()])
    for tau in (1e-3, 1e-2, 1e-1):
        a, c, tm = C.parabola(theta, tau)
        assert C.encloses(theta, tau, a, c)
        lam = -theta
        # at least half of the parabola's horizontal room: Re lam <= (a + (a - c Im^2)) / 2 - ...
        relv = lam[tau * lam.real >= tau * lam.real.max() - C.L_DECAY]
        assert np.all(relv.real <= a - 0.5 * c * relv.imag ** 2 - 0.5 / tau + 1e-9)


@pytest.mark.parametrize("tau", [1e-3, 1e-2, 5e-2])
def test_sgmres_contour_full_space_is_exact(tau):
    A = dense_convdiff(6, 50.0)
    N = A.shape[0]
    b = gaussian_rhs(N, 2)
    arn = oarn.truncated_arnoldi(A, b, N, N, np.eye(N))
    ref = sla.expm(-tau * A.toarray()) @ b
    assert rel(C.sgmres_contour(arn, tau).x, ref) < 1e-12
    assert rel(C.sfom_contour(arn, tau).x, ref) < 1e-12


@pytest.mark.parametrize("tau,m", [(1e-3, 40), (1e-2, 60)])
def test_sfom_contour_equals_closed_form(tau, m):
    A = dense_convdiff(30, 50.0)
    N = A.shape[0]
    b = gaussian_rhs(N, 2)
    S = osk.sparse_sign_matrix(N, 160, 8, 3)
    arn = oarn.truncated_arnoldi(A, b, m, 2, S)
    r = C.sfom_contour(arn, tau)
    assert rel(r.x, ometh.sfom_closed(arn, "exp", tau).x) < 1e-11
    assert r.info["quad_diff"] <= 1e-13 or r.info["floor"]


@pytest.mark.parametrize("tau,m", [(1e-2, 8), (5e-2, 12)])
def test_sgmres_contour_against_unwhitened_gmres(tau, m):
    A = dense_convdiff(8, 30.0)
    N = A.shape[0]
    b = gaussian_rhs(N, 4)
    arn = oarn.truncated_arnoldi(A, b, m, m, np.eye(N))
    r = C.sgmres_contour(arn, tau, tol=1e-12)
    # orthonormal basis of K_m(A, b) from the Krylov matrix itself
    Kry = np.empty((N, m))
    v = b / np.linalg.norm(b)
    for j in range(m):
        Kry[:, j] = v
        v = A @ v
        v /= np.linalg.norm(v)
    Vo, _ = np.linalg.qr(Kry)
    AV = A @ Vo
    a, c, tm = r.info["a"], r.info["c"], r.info["theta_max"]
    t, W = C.trapezoid(a, c, tm, r.l_used - 1, tau)
    acc = np.zeros(m)
    for tk, Wk in zip(t, W):
        acc += np.imag(Wk * np.linalg.lstsq(tk * Vo + AV, b.astype(np.complex128), rcond=None)[0])
    assert rel(r.x, Vo @ acc) < 1e-10


@pytest.mark.parametrize("mutation", ["conj", "dt_sign"])
def test_contour_mutations_fail(monkeypatch, mutation):
    orig = C.trapezoid

    def bad(a, c, theta_max, K, tau):
        t, W = orig(a, c, theta_max, K, tau)
        if mutation == "conj":
            return t, np.conj(W)
        h = theta_max / K
        th = h * np.arange(K + 1)
        return t, W * (-1j - 2.0 * c * th) / (1j - 2.0 * c * th)

    monkeypatch.setattr(C, "trapezoid", bad)
    A = dense_convdiff(12, 50.0).toarray()
    b = gaussian_rhs(A.shape[0], 1)
    tau = 1e-2
    theta = np.linalg.eigvals(A)
    a, c, tm = C.parabola(theta, tau)
    x = C.resolvent_rule(A, b, tau, a, c, tm, 256)
    assert rel(x, sla.expm(-tau * A) @ b) > 1e-3
