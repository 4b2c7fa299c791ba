"""Pins for the sketched FOM / GMRES approximants of the oracle.

Each test checks the oracle against something the paper (or mathematics) fixes,
not against a retyped copy of the oracle's own formula.
"""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import arnoldi as arn_mod
from oracle import methods, sketch
from oracle_helpers import (small_problem, identity_sketch, positive_real_matrix,
                            orthonormal_krylov, eps_on, dense_f, small_convdiff)
from workloads import gaussian_rhs

FUNCS = [("invsqrt", 0.0), ("exp", 1e-3), ("inv", 0.0)]


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("f,tau", FUNCS)
def test_identity_sketch_full_orth_equals_fom(f, tau):
    """Section 2, first remark: S = I reproduces FOM, ||b|| V_m f(H_m) e_1 (eq. FOM)."""
    A, b, _ = small_problem()
    m = 20
    S = identity_sketch(A.shape[0])
    arn = arn_mod.truncated_arnoldi(A, b, m, m, S)
    x = methods.sfom_closed(arn, f, tau).x
    full = arn_mod.full_arnoldi(A, b, m)
    assert rel(x, methods.fom(full, f, tau)) < 1e-11


@pytest.mark.parametrize("f,tau", FUNCS)
def test_closed_form_equals_gram_form_and_cortinovis(f, tau):
    """(sFOM''') = (sFOM') (Section 2.1) = the remark's H_hat form (Section 2.2)."""
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, 18, 2, S, extend=True)
    arn.S = S
    x = methods.sfom_closed(arn, f, tau).x
    assert rel(x, methods.sfom_gram_form(arn, f, tau)) < 1e-8
    assert rel(x, methods.cortinovis_form(arn, f, tau)) < 1e-8


def test_closed_form_equals_integral_form():
    """(sFOM) by quadrature of eq. (ym_hat) = closed form (Section 5.1: curves coincide)."""
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, 18, 2, S)
    xc = methods.sfom_closed(arn, "invsqrt").x
    xq = methods.sfom_quad(arn, "invsqrt", tol=1e-14).x
    assert rel(xq, xc) < 1e-12


def test_integral_form_unwhitened_definition():
    """eq. (sFOM) as printed, before whitening: V int [(SV)^H(tSV+SAV)]^-1 dmu (SV)^H S b,
    with the same Gauss-Chebyshev rule, equals the oracle's whitened evaluation."""
    from oracle import quadrature as quad
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, 12, 2, S)
    Sb = S @ b
    acc = np.zeros(arn.m_used)
    t, w = quad.gauss_chebyshev_invsqrt(400)
    sig = methods.spectral_scale(methods.whiten(arn).M)
    for ti, wi in zip(t, w):
        Kt = arn.SV.T @ (ti * sig * arn.SV + arn.SAV)
        acc += wi * sig * np.linalg.solve(Kt, arn.SV.T @ Sb) / np.sqrt(sig)
    assert rel(arn.V @ acc, methods.sfom_closed(arn, "invsqrt").x) < 1e-10


@pytest.mark.parametrize("method", ["sfom", "sgmres"])
def test_basis_independence_truncation(method):
    """Section 2.1: the approximants depend only on span(V_m): k = 2 vs k = m."""
    A, b, S = small_problem()
    m = 16
    a2 = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    am = arn_mod.truncated_arnoldi(A, b, m, m, S)
    f = methods.sfom_closed if method == "sfom" else methods.sgmres
    assert rel(f(a2, "invsqrt").x, f(am, "invsqrt").x) < 1e-9


def test_polynomial_exactness():
    """Corollary (interpolation): sFOM = q(A) b with q interpolating f at the
    eigenvalues of H_hat; for a polynomial of degree <= m-1 this is p(A) b."""
    A, b, S = small_problem()
    m = 8
    p = np.array([0.3, -2.0, 1e-4, 5e-9, -1e-12, 2e-17])   # degree 5 <= m-1
    arn = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    x = methods.sfom_closed(arn, "poly", poly=p).x
    ref = p[-1] * b
    for coef in p[-2::-1]:
        ref = A @ ref + coef * b
    assert rel(x, ref) < 1e-9


def test_invariant_subspace_exact():
    """b in an A-invariant subspace of dim <= m: Galerkin and sketched GMRES are exact."""
    rng = np.random.default_rng(3)
    blk = np.diag([2.0, 3.0, 5.0, 8.0]) + 0.3 * rng.standard_normal((4, 4))
    rest = sp.diags(np.linspace(1, 9, 60))
    A = sp.block_diag([blk, rest]).tocsr()
    b = np.zeros(64)
    b[:4] = rng.standard_normal(4)
    S = sketch.sparse_sign_matrix(64, 20, 8, 5)
    arn = arn_mod.truncated_arnoldi(A, b, 4, 4, S)
    truth = np.zeros(64)
    truth[:4] = np.real(np.linalg.solve(sla.sqrtm(blk), b[:4]))
    assert rel(methods.sfom_closed(arn, "invsqrt").x, truth) < 1e-10
    assert rel(methods.sgmres(arn, "invsqrt").x, truth) < 1e-10


def test_inverse_function_special_cases():
    """f = 1/z: eq. (ym_hat) at t = 0 gives (SV)^T(SAV) y = (SV)^T S b; eq. (sGMRES)
    with a point mass at 0 gives the sketched GMRES solution y = (SAV)^+ S b."""
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, 15, 2, S)
    Sb = S @ b
    y_fom = np.linalg.solve(arn.SV.T @ arn.SAV, arn.SV.T @ Sb)
    assert rel(methods.sfom_closed(arn, "inv").x, arn.V @ y_fom) < 1e-9
    y_gm = np.linalg.lstsq(arn.SAV, Sb, rcond=None)[0]
    assert rel(methods.sgmres(arn, "inv").x, arn.V @ y_gm) < 1e-9


@pytest.mark.parametrize("method", ["sfom", "sgmres"])
def test_full_dimension_exact(method):
    """Tiny N, m = N, s = N: both approximants equal f(A) b (dense Schur truth)."""
    A = small_convdiff(5, c=5.0)
    N = A.shape[0]
    b = gaussian_rhs(N, 1)
    S = sketch.sparse_sign_matrix(N, N, 8, 2)
    arn = arn_mod.truncated_arnoldi(A, b, N, N, S)
    truth = dense_f(A.toarray(), b, "invsqrt")
    x = (methods.sfom_closed if method == "sfom" else methods.sgmres)(arn, "invsqrt").x
    assert rel(x, truth) < 1e-8


def test_exp_full_dimension_exact():
    A = small_convdiff(5, c=5.0)
    N = A.shape[0]
    b = gaussian_rhs(N, 1)
    S = sketch.sparse_sign_matrix(N, N, 8, 2)
    arn = arn_mod.truncated_arnoldi(A, b, N, N, S)
    truth = dense_f(A.toarray(), b, "exp", 1e-3)
    assert rel(methods.sfom_closed(arn, "exp", 1e-3).x, truth) < 1e-8


def test_convergence_towards_dense_truth():
    A, b, S = small_problem(n=10, s=120)
    truth = dense_f(A.toarray(), b, "invsqrt")
    errs = [rel(methods.sgmres(arn_mod.truncated_arnoldi(A, b, m, 2, S), "invsqrt").x, truth)
            for m in (5, 15, 30)]
    assert errs[0] > errs[1] > errs[2]


def _whitened_basis(arn):
    w = methods.whiten(arn)
    return arn.V @ np.linalg.inv(w.R), w


@pytest.mark.parametrize("f,tau", [("invsqrt", 0.0), ("exp", 1e-4)])
def test_error_bound_sfom_vs_fom(f, tau):
    """Corollary (err): ||f_m - f_hat_m|| <= sqrt((1+e)/(1-e)) ||b|| ||f(V^+AV) - f(V^T S^T S A V)||
    with S V orthonormal and e the embedding constant on K_{m+1}."""
    A, b, S = small_problem(s=80)
    m = 12
    arn = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    Vw, w = _whitened_basis(arn)
    eps = eps_on(S, orthonormal_krylov(A, b, m + 1))
    assert eps < 1
    f_hat = methods.sfom_closed(arn, f, tau).x
    full = arn_mod.full_arnoldi(A, b, m)
    f_m = methods.fom(full, f, tau)
    Vp = np.linalg.pinv(Vw)
    F1 = _dense_fun(Vp @ (A @ Vw), f, tau)
    F2 = _dense_fun(w.M, f, tau)
    bound = np.sqrt((1 + eps) / (1 - eps)) * np.linalg.norm(b) * np.linalg.norm(F1 - F2, 2)
    assert np.linalg.norm(f_m - f_hat) <= bound * (1 + 1e-8)


def _dense_fun(M, f, tau):
    if f == "invsqrt":
        return np.real(np.linalg.inv(sla.sqrtm(M)))
    return sla.expm(-tau * M)


def test_sgmres_residual_bound():
    """eq. (resbnd): ||r_tilde(t)|| <= C_eps ||r(t)|| for the shifted systems."""
    A, b, S = small_problem(s=80)
    m = 12
    arn = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    eps = eps_on(S, orthonormal_krylov(A, b, m + 1))
    Ce = np.sqrt((1 + eps) / (1 - eps))
    Sb = S @ b
    V = arn.V
    AV = A @ V
    for t in [0.0, 1e2, 1e4, 1e6]:
        yt = np.linalg.lstsq(t * arn.SV + arn.SAV, Sb, rcond=None)[0]
        rt = b - (t * (V @ yt) + A @ (V @ yt))
        yf = np.linalg.lstsq(t * V + AV, b, rcond=None)[0]
        rf = b - (t * V + AV) @ yf
        assert np.linalg.norm(rt) <= Ce * np.linalg.norm(rf) * (1 + 1e-10)
        assert np.linalg.norm(rf) <= np.linalg.norm(rt) * (1 + 1e-10)


def test_theorem_sgmres_convergence_bound():
    """Theorem (conv): ||f(A)b - f_tilde_m||_{A^H A} <= C_1 C_eps ||b|| sin(beta_0)^m,
    C_1 = ||A|| f(rho ||A||^2), on a small positive real matrix."""
    Ad = positive_real_matrix(200, seed=0, skew=0.4)
    A = sp.csr_matrix(Ad)
    b = gaussian_rhs(200, 2)
    truth = dense_f(Ad, b, "invsqrt")
    nA = np.linalg.norm(Ad, 2)
    delta = np.linalg.eigvalsh((Ad + Ad.T) / 2).min()
    Ai = np.linalg.inv(Ad)
    rho = np.linalg.eigvalsh((Ai + Ai.T) / 2).min()
    C1 = nA * (rho * nA ** 2) ** -0.5
    sinb = np.sin(np.arccos(delta / nA))
    AtA = Ad.T @ Ad
    for m in (4, 8, 12):
        S = sketch.sparse_sign_matrix(200, 160, 8, m)
        eps = eps_on(S, orthonormal_krylov(Ad, b, m + 1))
        assert eps < 1
        Ce = np.sqrt((1 + eps) / (1 - eps))
        x = methods.sgmres(arn_mod.truncated_arnoldi(A, b, m, 2, S), "invsqrt").x
        e = truth - x
        assert np.sqrt(e @ AtA @ e) <= C1 * Ce * np.linalg.norm(b) * sinb ** m


def test_sketched_ritz_inclusion():
    """eq. (inclusion_sketched_ritz): Lambda(V^T S^T S A V) in W(A) + disc(eps ||A||)."""
    A, b, S = small_problem(s=80)
    m = 12
    arn = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    eps = eps_on(S, orthonormal_krylov(A, b, m + 1))
    Ad = A.toarray()
    nA = np.linalg.norm(Ad, 2)
    hs = np.linalg.eigvalsh((Ad + Ad.T) / 2)
    ks = np.linalg.norm((Ad - Ad.T) / 2, 2)
    theta = np.linalg.eigvals(methods.whiten(arn).M)
    assert np.all(theta.real >= hs.min() - eps * nA)
    assert np.all(theta.real <= hs.max() + eps * nA)
    assert np.all(np.abs(theta.imag) <= ks + eps * nA)


def test_stopping_estimate_bounds():
    """eqs. (sketched_err_est1/2): the sketched difference of two iterates brackets
    the true difference, evaluated from S V_{m+d} and coefficients only."""
    A, b, S = small_problem(s=80)
    m, d = 10, 5
    big = arn_mod.truncated_arnoldi(A, b, m + d, 2, S)
    small = arn_mod.truncated_arnoldi(A, b, m, 2, S)
    rb, rs = methods.sgmres(big, "invsqrt"), methods.sgmres(small, "invsqrt")
    eps = eps_on(S, orthonormal_krylov(A, b, m + d))
    true = np.linalg.norm(rb.x - rs.x)
    sk = methods.sketched_difference(big.SV, rb.y, rs.y)
    assert np.isclose(sk, np.linalg.norm(S @ (rb.x - rs.x)), rtol=1e-8)
    assert sk / np.sqrt(1 + eps) <= true * (1 + 1e-9)
    assert true <= methods.stopping_estimate(big.SV, rb.y, rs.y, eps) * (1 + 1e-9)


def test_eps_monitor_lower_bounds_true_eps():
    """Section 4.3 monitor: | ||S v_j||^2 - 1 | <= eps on the space (v_j unit, in K_m)."""
    A, b, S = small_problem(s=80)
    arn = arn_mod.truncated_arnoldi(A, b, 15, 2, S)
    assert methods.embedding_eps_estimate(arn) <= eps_on(S, orthonormal_krylov(A, b, 15)) + 1e-12


def test_branch_cut_detected():
    """A negative eigenvalue of the projected matrix: z^(-1/2) undefined -> BranchError."""
    Ad = np.diag([-3.0, 1.0, 2.0, 4.0, 5.0, 7.0])
    A = sp.csr_matrix(Ad)
    b = np.ones(6)
    S = identity_sketch(6)
    arn = arn_mod.truncated_arnoldi(A, b, 6, 6, S)
    with pytest.raises(methods.BranchError):
        methods.sfom_closed(arn, "invsqrt")


def test_zero_rhs_gives_zero():
    A, _, S = small_problem()
    res, _ = methods.solve(A, np.zeros(A.shape[0]), "invsqrt", 5, 2, S)
    assert np.all(res.x == 0)


def _sgmres_integrand_unwhitened(arn, Sb):
    """u -> (2/pi) (u^2 SV + SAV)^+ S b: the integrand of eq. (sGMRES) before any
    whitening, after t = u^2 (the measure t^(-1/2) dt / pi of z^(-1/2) becomes
    (2/pi) du on [0, inf))."""
    def g(u):
        t = u * u
        return (2.0 / np.pi) * np.linalg.lstsq(t * arn.SV + arn.SAV, Sb, rcond=None)[0]
    return g


@pytest.mark.parametrize("m,k", [(12, 2), (16, 3)])
def test_sgmres_equals_adaptive_integral_of_definition(m, k):
    """eq. (sGMRES) as printed, V_m int (t SV_m + SAV_m)^+ dmu(t) S b, integrated by
    a general-purpose adaptive integrator (SciPy quad_vec, no Gauss-Chebyshev rule,
    no whitening, no spectral scaling) equals the oracle's sGMRES.  A Galerkin
    rule in place of the least-squares one differs at the 1e-3 level here."""
    from scipy.integrate import quad_vec
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, m, k, S)
    Sb = S @ b
    val, err = quad_vec(_sgmres_integrand_unwhitened(arn, Sb), 0.0, np.inf, epsabs=0.0, epsrel=1e-13,
                        limit=2000)
    x_def = arn.V @ val
    x = methods.sgmres(arn, "invsqrt").x
    assert rel(x, x_def) < 1e-10
    # and it is not the sketched FOM approximant (the two differ on this problem)
    assert rel(methods.sfom_closed(arn, "invsqrt").x, x_def) > 1e-6


def test_sgmres_node_solutions_satisfy_normal_equations():
    """Section 3: at every shift t the sGMRES coefficients minimise ||S b - (t SV + SAV) y||,
    so the sketched residual is orthogonal to the columns of t SV + SAV.  The oracle's
    node solve (whitened: (t Q + B)^+ S b mapped back by R^-1) is checked on its own
    nodes against these normal equations in unwhitened coordinates."""
    from oracle import quadrature as quad
    A, b, S = small_problem()
    arn = arn_mod.truncated_arnoldi(A, b, 14, 2, S)
    w = methods.whiten(arn)
    sig = methods.spectral_scale(w.M)
    t, _ = quad.gauss_chebyshev_invsqrt(45)
    for ti in t * sig:
        u = np.linalg.lstsq(ti * w.Q + w.B, w.Sb, rcond=None)[0]
        y = sla.solve_triangular(w.R, u, lower=False)
        P = ti * arn.SV + arn.SAV
        r = w.Sb - P @ y
        assert np.linalg.norm(P.T @ r) <= 1e-9 * np.linalg.norm(P, 2) * np.linalg.norm(w.Sb)


@pytest.mark.parametrize("method", ["sfom", "sgmres", "sfom_quad"])
def test_two_pass_equals_one_pass(method):
    """Section 4.2: discarding the basis in the first pass and regenerating it in the
    second gives the one-pass approximant V_m y (to rounding)."""
    A, b, S = small_problem()
    m, k = 18, 2
    arn = arn_mod.truncated_arnoldi(A, b, m, k, S)
    one = {"sfom": lambda: methods.sfom_closed(arn, "invsqrt"),
           "sgmres": lambda: methods.sgmres(arn, "invsqrt"),
           "sfom_quad": lambda: methods.sfom_quad(arn, "invsqrt")}[method]().x
    two = methods.two_pass(A, b, "invsqrt", m, k, S, method).x
    assert rel(two, one) < 1e-13
    vs = list(arn_mod.truncated_basis_vectors(A, b, m, k))
    assert len(vs) == m
    assert max(np.max(np.abs(v - arn.V[:, i])) for i, v in enumerate(vs)) < 1e-13


def test_two_pass_breakdown_and_exp():
    """The second pass stops where the first broke down; closed-form exp as well."""
    rng = np.random.default_rng(4)
    blk = np.diag([2.0, 3.0, 5.0]) + 0.3 * rng.standard_normal((3, 3))
    A = sp.block_diag([blk, sp.diags(np.linspace(1, 9, 40))]).tocsr()
    b = np.zeros(43)
    b[:3] = rng.standard_normal(3)
    S = sketch.sparse_sign_matrix(43, 20, 8, 1)
    res = methods.two_pass(A, b, "exp", 8, 3, S, fparam=0.1)
    truth = np.zeros(43)
    truth[:3] = sla.expm(-0.1 * blk) @ b[:3]
    assert res.m_used == 3 and rel(res.x, truth) < 1e-10
