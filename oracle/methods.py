"""Sketched FOM and sketched GMRES approximants of f(A)b (plain FP64).

Section 2 defines the sketched FOM approximant by the integral (sFOM) over the
sketched Galerkin solutions (eq. ym_hat) and derives the closed forms (sFOM'),
(sFOM'') and, after retrospective basis whitening SV_m = Q_m R_m, (sFOM''') --
the form Algorithm 1 evaluates.  Section 3 defines the sketched GMRES
approximant (sGMRES), evaluated by quadrature as in Algorithm 2 and Section 4.1.

Functions f (the ``f`` argument):
  "invsqrt"  f(z) = z^(-1/2)       (Stieltjes; principal branch)
  "exp"      f(z) = exp(-tau z)    (``fparam`` = tau)
  "inv"      f(z) = 1/z            (Stieltjes with a point mass at t = 0)
  "poly"     f(z) = sum_i p[i] z^i (``poly`` = coefficients, lowest first)

Readings (listed in the design notes):
  * S b is taken as ||b|| * S v_1, the first column of SV_m (Section 4's
    algorithm never sketches b itself).
  * Extremely ill-conditioned R (remark after eq. sfom3): the numerical
    pseudoinverse is the truncated QR one in basis order, i.e. the longest
    prefix of the basis whose sketch has kappa_F(R_j) <= COND_MAX is used.
  * Whitened coordinates: c = Q^T S b, B = SAV R^-1, M = Q^T B.
  * Quadrature uses the spectral scaling sigma = sqrt(|theta|_min |theta|_max)
    over the eigenvalues theta of M (an exact identity for z^(-1/2)).
  * An eigenvalue of M on (-inf, 0] makes z^(-1/2) undefined: BranchError.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from . import quadrature as quad
from .arnoldi import ArnoldiResult


class BranchError(ArithmeticError):
    """An eigenvalue of the projected matrix lies on f's branch cut."""


class QuadratureError(ArithmeticError):
    """Adaptive quadrature reached the maximum order without converging."""


@dataclass
class Whitened:
    Q: np.ndarray
    R: np.ndarray
    B: np.ndarray     # SAV R^-1
    M: np.ndarray     # Q^T SAV R^-1
    c: np.ndarray     # Q^T S b
    Sb: np.ndarray    # S b = beta * SV[:, 0]


# ------------------------------------------- ill-conditioned R (Section 2.1) ---
# The remark after eq. (sFOM''') suggests a numerical pseudoinverse in place of
# R_m^-1 when SV_m, and hence R_m, is extremely ill-conditioned.  Reading taken
# here: the pseudoinverse is the truncated (basic) one of the QR factor in the
# order of the Krylov basis.  The leading blocks R_j = R[:j, :j] are the QR
# factors of the prefixes SV_j, and their condition numbers never decrease with
# j, so the columns to drop are the trailing ones: the approximant is formed
# from the longest prefix V_j whose sketch has a Frobenius-norm condition number
# ||R_j||_F ||R_j^-1||_F of at most COND_MAX.  A basis that meets the bound is
# used whole, so the remedy changes nothing for well-conditioned problems.
COND_MAX = 1e10


def prefix_conditions(R: np.ndarray) -> np.ndarray:
    """kappa_F(R_j) = ||R_j||_F ||R_j^-1||_F for j = 1..m (R upper triangular).
    R_j^-1 is the leading block of R^-1, so both norms are prefix sums over
    columns; a zero pivot gives inf from its column on."""
    m = R.shape[0]
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        Rinv = sla.solve_triangular(R, np.eye(m), lower=False)
        inv2 = np.cumsum(np.sum(Rinv ** 2, axis=0))
        fro2 = np.cumsum(np.sum(np.triu(R) ** 2, axis=0))
        c = np.sqrt(fro2 * inv2)
    c[~np.isfinite(c)] = np.inf
    return np.maximum.accumulate(c)


def conditioned_prefix(arn: ArnoldiResult, cond_max: float = COND_MAX) -> int:
    """Largest j with kappa_F(R_j) <= cond_max, R the QR factor of SV_m."""
    if arn.m_used == 0:
        return 0
    R = np.linalg.qr(arn.SV, mode="r")
    c = prefix_conditions(R)
    return max(1, int(np.count_nonzero(c <= cond_max)))


def regularize(arn: ArnoldiResult, cond_max: float = COND_MAX):
    """The data the whitening uses: arn itself, or its conditioned prefix."""
    mp = conditioned_prefix(arn, cond_max)
    if mp >= arn.m_used:
        return arn, arn.m_used
    return _prefix(arn, mp), mp


def _pad(y: np.ndarray, m: int) -> np.ndarray:
    """Coefficients over the whole basis: dropped trailing vectors get 0."""
    if y.size >= m:
        return y
    out = np.zeros(m)
    out[: y.size] = y
    return out


def whiten(arn: ArnoldiResult) -> Whitened:
    """Thin QR of SV_m and the whitened quantities (Section 2.1, eq. sfom3)."""
    Q, R = np.linalg.qr(arn.SV, mode="reduced")
    # B = SAV R^-1  <=>  R^T B^T = SAV^T
    B = sla.solve_triangular(R, arn.SAV.T, trans="T", lower=False).T
    M = Q.T @ B
    Sb = arn.beta * arn.SV[:, 0]
    c = Q.T @ Sb
    return Whitened(Q, R, B, M, c, Sb)


# ---------------------------------------------------------------- f(M) c ---
def check_branch(M: np.ndarray):
    ev = np.linalg.eigvals(M)
    bad = (np.abs(ev.imag) <= 1e-12 * np.max(np.abs(ev))) & (ev.real <= 0.0)
    if np.any(bad):
        raise BranchError("eigenvalue of the projected matrix on (-inf, 0]")
    return ev


def matfun_apply(M: np.ndarray, c: np.ndarray, f: str, fparam: float = 0.0,
                 poly=None) -> np.ndarray:
    """g = f(M) c with dense Schur-based routines (SciPy)."""
    if f == "invsqrt":
        check_branch(M)
        X = sla.sqrtm(M)
        g = np.linalg.solve(X, c)
        return np.real_if_close(g, tol=1e6).real
    if f == "exp":
        return sla.expm(-fparam * M) @ c
    if f == "inv":
        return np.linalg.solve(M, c)
    if f == "poly":
        p = np.asarray(poly, dtype=np.float64)
        g = p[-1] * c
        for coef in p[-2::-1]:
            g = M @ g + coef * c
        return g
    raise ValueError(f"unknown function {f!r}")


def spectral_scale(M: np.ndarray) -> float:
    ev = np.abs(np.linalg.eigvals(M))
    return float(np.sqrt(ev.min() * ev.max()))


# ------------------------------------------------------------ results -----
@dataclass
class SolveResult:
    x: np.ndarray
    y: np.ndarray             # coefficients in the (unwhitened) basis V_m
    m_used: int
    l_used: int = 0
    info: dict = field(default_factory=dict)


def _assemble(arn: ArnoldiResult, y: np.ndarray) -> np.ndarray:
    """f_m = V_m y  (Algorithm 1, last step)."""
    return arn.V @ y


def _empty(arn: ArnoldiResult) -> SolveResult:
    return SolveResult(np.zeros(arn.V.shape[0]), np.zeros(0), 0)


def sfom_closed(arn: ArnoldiResult, f: str, fparam: float = 0.0, poly=None) -> SolveResult:
    """Closed form (sFOM''') of Algorithm 1: V_m R^-1 f(Q^T SAV R^-1) Q^T S b."""
    if arn.m_used == 0:
        return _empty(arn)
    full = arn
    arn, mp = regularize(full)
    w = whiten(arn)
    g = matfun_apply(w.M, w.c, f, fparam, poly)
    y = _pad(sla.solve_triangular(w.R, g, lower=False), full.m_used)
    return SolveResult(_assemble(full, y), y, mp,
                       info=dict(rcond_R=1.0 / np.linalg.cond(w.R)))


# Rounding floor of the adaptive test.  This is NOT part of Section 4.1's rule,
# which refines until ||q_l1 - q_l2|| < tol: it is an addition of this
# implementation.  When the requested tolerance lies below what the node solves
# can resolve, the relative differences of consecutive orders stop falling at
# the rounding level of the node solves; an order whose difference is below
# QUAD_FLOOR and larger than half the previous difference is then accepted
# instead of refining up to l_max.  At the last order the sequence allows (the
# next one would exceed l_max), a difference below QUAD_FLOOR is accepted even
# while it is still falling: no further order exists to show the floor, and the
# difference already bounds the change at that level.  Results accepted this
# way report ``floor=True`` in their info and the accepted difference.
QUAD_FLOOR = 1e-10


def _adaptive(eval_rule, tol: float, l1: int, l2: int, lmax: int, stats: dict | None = None):
    """Adaptive order loop of Section 4.1 (relative test ||q1-q2|| <= tol ||q2||),
    with the rounding-floor acceptance described at QUAD_FLOOR.  ``stats``
    receives the accepted difference and whether the floor accepted it."""
    q1 = eval_rule(l1)
    q2 = eval_rule(l2)
    d_prev = np.inf
    st = stats if stats is not None else {}
    while True:
        n2 = np.linalg.norm(q2)
        d = np.linalg.norm(q1 - q2) / n2 if n2 > 0 else (0.0 if np.linalg.norm(q1) == 0 else np.inf)
        st["quad_diff"] = d
        st["floor"] = False
        if d <= tol:
            return q2, l2
        if d <= QUAD_FLOOR and d > 0.5 * d_prev:
            st["floor"] = True
            return q2, l2
        nxt = quad.next_order(l2)
        if nxt > lmax:
            if d <= QUAD_FLOOR:
                st["floor"] = True
                return q2, l2
            raise QuadratureError(f"no convergence up to l = {l2}")
        q1, l1, l2, d_prev = q2, l2, nxt, d
        q2 = eval_rule(l2)


def sfom_quad(arn: ArnoldiResult, f: str = "invsqrt", tol: float = 1e-13,
              l1: int = quad.L1_DEFAULT, l2: int = quad.L2_DEFAULT,
              lmax: int = quad.LMAX_DEFAULT) -> SolveResult:
    """Integral form (sFOM) in whitened coordinates: the sketched Galerkin
    solutions of eq. (ym_hat) satisfy (t I + M) y_hat(t) = c, integrated by the
    Gauss-Chebyshev rule."""
    if arn.m_used == 0:
        return _empty(arn)
    full = arn
    arn, mp = regularize(full)
    w = whiten(arn)
    m = w.M.shape[0]
    if f == "inv":
        g = np.linalg.solve(w.M, w.c)
        y = _pad(sla.solve_triangular(w.R, g, lower=False), full.m_used)
        return SolveResult(_assemble(full, y), y, mp, 1)
    if f != "invsqrt":
        raise ValueError("quadrature forms support the Stieltjes functions invsqrt and inv")
    check_branch(w.M)
    sigma = spectral_scale(w.M)

    def rule(l):
        t, wt = quad.gauss_chebyshev_invsqrt(l)
        acc = np.zeros(m)
        for ti, wi in zip(t, wt):
            acc += wi * np.linalg.solve(ti * np.eye(m) + w.M / sigma, w.c)
        return acc / np.sqrt(sigma)

    st = {}
    g, l_used = _adaptive(rule, tol, l1, l2, lmax, st)
    y = _pad(sla.solve_triangular(w.R, g, lower=False), full.m_used)
    return SolveResult(_assemble(full, y), y, mp, l_used, info=dict(sigma=sigma, **st))


def sgmres(arn: ArnoldiResult, f: str = "invsqrt", tol: float = 1e-13,
           l1: int = quad.L1_DEFAULT, l2: int = quad.L2_DEFAULT,
           lmax: int = quad.LMAX_DEFAULT) -> SolveResult:
    """Sketched GMRES approximant (sGMRES), Section 3 / Algorithm 2:
    V_m R^-1 int (t Q + B)^+ dmu(t) S b, the pseudo-inverse applied by a
    least-squares solve at every quadrature node (Section 4.1, eq.
    quadrature_rule)."""
    if arn.m_used == 0:
        return _empty(arn)
    full = arn
    arn, mp = regularize(full)
    w = whiten(arn)
    if f == "inv":
        # point mass at t = 0: the textbook sketched GMRES solution of A x = b
        g = np.linalg.lstsq(w.B, w.Sb, rcond=None)[0]
        y = _pad(sla.solve_triangular(w.R, g, lower=False), full.m_used)
        return SolveResult(_assemble(full, y), y, mp, 1)
    if f != "invsqrt":
        raise ValueError("sGMRES needs a Stieltjes function (invsqrt or inv)")
    sigma = spectral_scale(w.M)

    def rule(l):
        t, wt = quad.gauss_chebyshev_invsqrt(l)
        acc = np.zeros(w.M.shape[0])
        for ti, wi in zip(t, wt):
            acc += wi * np.linalg.lstsq(ti * w.Q + w.B / sigma, w.Sb, rcond=None)[0]
        return acc / np.sqrt(sigma)

    st = {}
    g, l_used = _adaptive(rule, tol, l1, l2, lmax, st)
    y = _pad(sla.solve_triangular(w.R, g, lower=False), full.m_used)
    return SolveResult(_assemble(full, y), y, mp, l_used, info=dict(sigma=sigma, **st))


# ---------------------------------------------- equivalent forms (pins) ---
def sfom_gram_form(arn: ArnoldiResult, f: str, fparam: float = 0.0, poly=None) -> np.ndarray:
    """(sFOM'): V (V^H S^H S V)^-1 f(V^H S^H S A V (V^H S^H S V)^-1) (SV)^H (S b),
    evaluated without any QR (Section 2.1)."""
    G = arn.SV.T @ arn.SV
    K = arn.SV.T @ arn.SAV
    Kg = np.linalg.solve(G.T, K.T).T          # K G^-1
    rhs = arn.SV.T @ (arn.beta * arn.SV[:, 0])
    g = matfun_apply(Kg, rhs, f, fparam, poly)
    return arn.V @ np.linalg.solve(G, g)


def cortinovis_form(arn: ArnoldiResult, f: str, fparam: float = 0.0, poly=None) -> np.ndarray:
    """Remark in Section 2.2: V f(H_m + h_{m+1,m} x_hat e_m^T) ||b|| e_1 with
    x_hat = argmin ||S v_{m+1} - S V_m x||.  Needs ``extend=True`` Arnoldi."""
    if arn.v_next is None:
        raise ValueError("needs the extended basis (v_{m+1})")
    m = arn.m_used
    Hm = arn.H[:m, :m]
    hlast = arn.H[m, m - 1]
    Sv = _sketch_from(arn, arn.v_next)
    xhat = np.linalg.lstsq(arn.SV, Sv, rcond=None)[0]
    Hhat = Hm.copy()
    Hhat[:, m - 1] += hlast * xhat
    e1 = np.zeros(m)
    e1[0] = arn.beta
    return arn.V @ matfun_apply(Hhat, e1, f, fparam, poly)


def _sketch_from(arn: ArnoldiResult, v: np.ndarray) -> np.ndarray:
    if not hasattr(arn, "S") or arn.S is None:
        raise ValueError("attach the sketch as arn.S to use this form")
    return arn.S @ v


def fom(arn_full: ArnoldiResult, f: str, fparam: float = 0.0, poly=None) -> np.ndarray:
    """Standard FOM approximant (eq. FOM) ||b|| V_m f(H_m) e_1 from a fully
    orthogonalised basis."""
    m = arn_full.m_used
    e1 = np.zeros(m)
    e1[0] = arn_full.beta
    return arn_full.V @ matfun_apply(arn_full.H[:m, :m], e1, f, fparam, poly)


# ------------------------------------------------- monitoring (Section 4.3) ---
def embedding_eps_estimate(arn: ArnoldiResult) -> float:
    """max_j | ||S v_j||^2 - 1 |, the cheap epsilon monitor (Section 4.3)."""
    return float(np.max(np.abs(np.sum(arn.SV ** 2, axis=0) - 1.0)))


def sketched_difference(SV_big: np.ndarray, y_big: np.ndarray, y_small: np.ndarray) -> float:
    """|| S V_{m+d} (y_{m+d} - [y_m; 0]) ||, eq. (sketched_err_est2)."""
    d = np.zeros_like(y_big)
    d[: y_small.size] = y_small
    return float(np.linalg.norm(SV_big @ (y_big - d)))


def stopping_estimate(SV_big, y_big, y_small, eps: float) -> float:
    """Upper estimate of ||f_{m+d} - f_m||: the sketched difference / sqrt(1-eps)."""
    return sketched_difference(SV_big, y_big, y_small) / np.sqrt(1.0 - eps)


def solve(A, b, f: str, m: int, k: int, S, method: str = "sfom", fparam: float = 0.0,
          poly=None, tol: float = 1e-13, extend: bool = False):
    """Convenience driver: truncated Arnoldi + the chosen evaluation."""
    from .arnoldi import truncated_arnoldi
    arn = truncated_arnoldi(A, b, m, k, S, extend=extend)
    arn.S = S
    if method == "sfom":
        res = sfom_closed(arn, f, fparam, poly)
    elif method == "sfom_quad":
        res = sfom_quad(arn, f, tol)
    elif method == "sgmres":
        res = sgmres(arn, f, tol)
    else:
        raise ValueError(method)
    return res, arn


# ------------------------------------------------ adaptive m (Section 4.3) ---
def _prefix(arn: ArnoldiResult, m: int) -> ArnoldiResult:
    """The data of the first m steps of a longer run: the truncated recurrence is
    sequential, so these are exactly the arrays an m-step run produces."""
    return ArnoldiResult(arn.V[:, :m].copy(), arn.SV[:, :m].copy(), arn.SAV[:, :m].copy(),
                         arn.H[:m + 1, :m].copy(), arn.beta, m)


def relative_stopping_estimate(arn_m: ArnoldiResult, y_m: np.ndarray, y_prev: np.ndarray) -> float:
    """Relative form of the Section 4.3 estimate used by the adaptive loop:
    || S V_m (y_m - [y_prev; 0]) || / || S V_m y_m || * sqrt((1 + eps) / (1 - eps)),
    i.e. the upper estimate of ||f_m - f_prev|| over the lower estimate of ||f_m||
    (eps from the Section 4.3 monitor)."""
    eps = embedding_eps_estimate(arn_m)
    num = sketched_difference(arn_m.SV, y_m, y_prev)
    den = float(np.linalg.norm(arn_m.SV @ y_m))
    if den == 0.0:
        return 0.0 if num == 0.0 else np.inf
    return num / den * np.sqrt((1.0 + eps) / (1.0 - eps))


def adaptive_m(A, b, f: str, k: int, S, m0: int, d: int, m_max: int, tol: float,
               fparam: float = 0.0):
    """Plain adaptive-m sketched FOM: evaluate the closed form at m0, m0 + d, ...
    (<= m_max) on the nested truncated basis and stop at the first m whose
    relative stopping estimate against the previous checkpoint is <= tol.
    Returns (SolveResult, m_stop, estimate); the estimate is inf when no
    checkpoint pair passed (the result is then the one at the last checkpoint).
    A breakdown before a checkpoint ends the loop with the exact result."""
    from .arnoldi import truncated_arnoldi
    arn = truncated_arnoldi(A, b, m_max, k, S)
    prev = None
    est = np.inf
    res = None
    m = m0
    while m <= m_max:
        if arn.m_used < m:
            return sfom_closed(arn, f, fparam), arn.m_used, 0.0
        am = _prefix(arn, m)
        res = sfom_closed(am, f, fparam)
        if prev is not None:
            est = relative_stopping_estimate(am, res.y, prev.y)
            if est <= tol:
                return res, m, est
        prev = res
        m += d
    return res, m - d, est


# ------------------------------------------------- two passes (Section 4.2) ---
def two_pass(A, b, f: str, m: int, k: int, S, method: str = "sfom", fparam: float = 0.0, tol: float = 1e-13):
    """Section 4.2: the first pass runs the k-truncated recurrence and keeps only the
    sketches and coefficients (the basis vectors are not needed once the window has
    moved past them); the small problem gives the coefficient vector y; the second
    pass runs the recurrence again and accumulates x = sum_i y_i v_i, one vector at
    a time.  Returns the small problem's SolveResult with this x."""
    from .arnoldi import truncated_arnoldi, truncated_basis_vectors
    arn = truncated_arnoldi(A, b, m, k, S)
    # the first pass's data without the basis (a zero-height V: no N-sized work)
    first = ArnoldiResult(np.zeros((0, arn.m_used)), arn.SV, arn.SAV, arn.H, arn.beta, arn.m_used)
    if method == "sfom":
        res = sfom_closed(first, f, fparam)
    elif method == "sgmres":
        res = sgmres(first, f, tol)
    else:
        res = sfom_quad(first, f, tol)
    x = np.zeros(b.shape[0])
    for i, v in enumerate(truncated_basis_vectors(A, b, arn.m_used, k)):
        x += res.y[i] * v
    res.x = x
    return res


# ------------------------------------------------- s-adaptivity (Section 6)
EPS_MAX_DEFAULT = 0.5


def solve_reckless(A, b, f: str, m: int, k: int, s0: int, s_max: int, eps_max: float = EPS_MAX_DEFAULT,
                   zeta: int = 8, seed: int = 0, method: str = "sfom", fparam: float = 0.0, tol: float = 1e-13):
    """The 'responsibly reckless' choice of the sketch size that the conclusions
    propose: start with an optimistic s, monitor the computation, and redo it with
    a larger s when s turns out to be too small.  Reading: s is too small when the
    solve fails numerically (a sketched Ritz value on the branch cut, or a
    quadrature that does not converge) or when the Section 4.3 monitor
    max_j | ||S v_j||^2 - 1 | over the basis in use exceeds eps_max; the redo
    doubles s (capped at s_max; S is redrawn from the same seed).  Returns
    (SolveResult, s_used, trail) with trail = [(s, outcome, eps), ...]."""
    from . import arnoldi as oarn
    from . import sketch as osk
    N = A.shape[0]
    trail = []
    s = s0
    while True:
        S = osk.sparse_sign_matrix(N, s, zeta, seed)
        arn = oarn.truncated_arnoldi(A, b, m, k, S)
        used, mp = regularize(arn)
        eps = float(np.max(np.abs(np.sum(used.SV ** 2, axis=0) - 1.0))) if mp > 0 else 0.0
        res, outcome = None, "ok"
        try:
            if method == "sfom":
                res = sfom_closed(arn, f, fparam)
            elif method == "sfom_quad":
                res = sfom_quad(arn, f, tol=tol)
            else:
                res = sgmres(arn, f, tol=tol)
        except BranchError:
            outcome = "branch"
        except QuadratureError:
            outcome = "quad"
        if outcome == "ok" and eps > eps_max:
            outcome = "eps"
        trail.append((s, outcome, eps))
        if outcome == "ok" or s >= s_max:
            return res, s, trail
        s = min(2 * s, s_max)
