"""Contour quadrature for f(z) = exp(-tau z) (Section 1, Sections 4.1 and 5.2).

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Integral form.  The paper writes f(A)b as an integral of the solutions x(t) of
the shifted systems (t I + A) x(t) = b against a measure on a contour Gamma that
encloses the negated spectrum; with dmu(t) = dt / (2 pi i) this is Cauchy's
formula for g(-A) with g = exp(tau .):

    exp(-tau A) b = 1/(2 pi i) int_Gamma exp(tau t) (t I + A)^-1 b dt,

Gamma traversed counterclockwise around -Lambda(A).  Sketched GMRES (eq.
sGMRES) and sketched FOM (eq. sFOM) replace x(t) by V_m y(t) with
y(t) = (t SV_m + SAV_m)^+ S b, respectively by the sketched Galerkin solution
(t I + M) g(t) = c in whitened coordinates.

Contour.  Section 5.2 integrates over the parabola

    t(theta) = a + i theta - c theta^2,  theta real,

with a, c chosen so that the sketched Ritz values are enclosed (Algorithm 2:
eigenvalues of the rectangular pencil SAV_m x = -lambda SV_m x, which are the
negated eigenvalues of M).  The paper fixes no rule for a and c; the reading
taken here, in units where tau = 1 (u = tau t):
  * mu_j = -tau theta_j for the Ritz values theta_j, X = max_j Re mu_j; only
    those with Re mu_j >= X - L matter (L = 45: an unenclosed one would lose a
    weight below exp(-45) ~ 3e-20 times the largest, exp(X));
  * apex alpha = X + 1;
  * curvature kappa = min(KAPPA_MAX, min_j (alpha - Re mu_j) / (2 (Im mu_j)^2))
    over the relevant mu_j with Im mu_j != 0 (each such value lies halfway
    between the axis of the parabola and the parabola itself);
  * truncation |v| <= v_max with alpha - kappa v_max^2 = X - L (the integrand
    has fallen below exp(-L) of its largest scale there);
  * back in t: a = alpha / tau, c = kappa tau, theta_max = v_max / tau.

Rule.  The trapezoidal rule in theta with step h = theta_max / K, nodes
theta_k = k h (k = 0..K).  A, b and S are real, so the integrand at -theta is
minus the conjugate of the one at theta, and

    1/(2 pi i) sum_{|k| <= K} h exp(tau t_k) t'_k x(t_k)
        = (h / pi) sum_{k = 0}^{K} c_k Im(exp(tau t_k) t'_k x(t_k)),

c_0 = 1/2, c_k = 1 otherwise, t'(theta) = i - 2 c theta.  Adaptive order as in
Section 4.1, with K doubled (32, 64, ..., KMAX) in place of the Gauss-Chebyshev
order sequence, the relative test in whitened coordinates, and the same
rounding floor (methods.QUAD_FLOOR).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import methods as M_
from .arnoldi import ArnoldiResult

L_DECAY = 45.0
KAPPA_MAX = 0.25
K_FIRST = 32
K_MAX = 1024  # the largest level the library evaluates


def parabola(theta: np.ndarray, tau: float):
    """(a, c, theta_max) of the contour for the Ritz values theta (reading above)."""
    mu = -tau * np.asarray(theta, dtype=np.complex128)
    top = float(mu.real.max())
    rel = mu[mu.real >= top - L_DECAY]
    alpha = top + 1.0
    kappa = KAPPA_MAX
    cplx = np.abs(rel.imag) > 0.0
    if np.any(cplx):
        kappa = min(kappa, float(np.min((alpha - rel.real[cplx]) / (2.0 * rel.imag[cplx] ** 2))))
    vmax = np.sqrt((alpha - top + L_DECAY) / kappa)
    return alpha / tau, kappa * tau, vmax / tau


def encloses(theta: np.ndarray, tau: float, a: float, c: float) -> bool:
    """Every relevant -theta_j lies strictly inside the parabola (left of it)."""
    lam = -np.asarray(theta, dtype=np.complex128)
    rel = lam[tau * lam.real >= tau * lam.real.max() - L_DECAY]
    return bool(np.all(rel.real < a - c * rel.imag ** 2))


def trapezoid(a: float, c: float, theta_max: float, K: int, tau: float):
    """Nodes t_k and complex weights W_k with f ~ sum_k Im(W_k x(t_k))."""
    h = theta_max / K
    th = h * np.arange(K + 1)
    t = a + 1j * th - c * th ** 2
    dt = 1j - 2.0 * c * th
    ck = np.ones(K + 1)
    ck[0] = 0.5
    W = (h / np.pi) * ck * np.exp(tau * t) * dt
    return t, W


def resolvent_rule(A: np.ndarray, b: np.ndarray, tau: float, a: float, c: float, theta_max: float,
                   K: int) -> np.ndarray:
    """The rule with the exact resolvent (dense solves): exp(-tau A) b up to the
    quadrature error, for any contour that encloses -Lambda(A)."""
    t, W = trapezoid(a, c, theta_max, K, tau)
    n = A.shape[0]
    acc = np.zeros(n)
    for tk, Wk in zip(t, W):
        acc += np.imag(Wk * np.linalg.solve(tk * np.eye(n) + A, b.astype(np.complex128)))
    return acc


def _contour_solve(arn: ArnoldiResult, tau: float, node, tol: float, kmax: int, cond_max: float):
    full = arn
    arn, mp = M_.regularize(full, cond_max)
    w = M_.whiten(arn)
    theta = np.linalg.eigvals(w.M)
    a, c, tmax = parabola(theta, tau)

    def rule(K):
        t, W = trapezoid(a, c, tmax, K, tau)
        acc = np.zeros(w.M.shape[0])
        for tk, Wk in zip(t, W):
            acc += np.imag(Wk * node(w, tk))
        return acc

    # Section 4.1's test in whitened coordinates: g is already whitened here
    st = {}
    K1, K2 = K_FIRST, 2 * K_FIRST
    q1, q2 = rule(K1), rule(K2)
    d_prev = np.inf
    while True:
        n2 = np.linalg.norm(q2)
        d = np.linalg.norm(q1 - q2) / n2 if n2 > 0 else 0.0
        st["quad_diff"], st["floor"] = d, False
        if d <= tol:
            break
        if d <= M_.QUAD_FLOOR and d > 0.5 * d_prev:
            st["floor"] = True
            break
        if 2 * K2 > kmax:
            if d <= M_.QUAD_FLOOR:
                st["floor"] = True
                break
            raise M_.QuadratureError(f"contour rule: no convergence up to K = {K2}")
        q1, K1, K2, d_prev = q2, K2, 2 * K2, d
        q2 = rule(K2)
    y = M_._pad(sla.solve_triangular(w.R, q2, lower=False), full.m_used)
    return M_.SolveResult(M_._assemble(full, y), y, mp, K2 + 1,
                          info=dict(a=a, c=c, theta_max=tmax, ritz=theta, **st))


def sgmres_contour(arn: ArnoldiResult, tau: float, tol: float = 1e-13, kmax: int = K_MAX,
                   cond_max: float = M_.COND_MAX) -> M_.SolveResult:
    """Sketched GMRES approximant (eq. sGMRES) to exp(-tau A) b: at each node the
    least-squares solution of min ||S b - (t Q + B) g|| (complex t), whitened."""
    if arn.m_used == 0:
        return M_._empty(arn)

    def node(w, t):
        return np.linalg.lstsq(t * w.Q + w.B, w.Sb.astype(np.complex128), rcond=None)[0]

    return _contour_solve(arn, tau, node, tol, kmax, cond_max)


def sfom_contour(arn: ArnoldiResult, tau: float, tol: float = 1e-13, kmax: int = K_MAX,
                 cond_max: float = M_.COND_MAX) -> M_.SolveResult:
    """Sketched FOM approximant by the same contour rule: (t I + M) g = c at each
    node.  Equals the closed form exp(-tau M) c up to the quadrature error."""
    if arn.m_used == 0:
        return M_._empty(arn)

    def node(w, t):
        return np.linalg.solve(t * np.eye(w.M.shape[0]) + w.M, w.c.astype(np.complex128))

    return _contour_solve(arn, tau, node, tol, kmax, cond_max)
