"""Planted mistakes in the oracle (CPU only): each must be caught by a pin.

Every test swaps one oracle function for a copy with a plausible mistake (a
transposed operand, a dropped factor, a wrong sign or index) and checks that
at least one pin test then fails.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import arnoldi as arn_mod
from oracle import methods, quadrature
import test_oracle_arnoldi as ta
import test_oracle_methods as tm
import test_oracle_quadrature as tq


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_transposed_projection_caught(monkeypatch):
    real = methods.whiten

    def bad(arn):
        w = real(arn)
        w.M = w.M.T.copy()
        return w
    monkeypatch.setattr(methods, "whiten", bad)
    _fails(tm.test_identity_sketch_full_orth_equals_fom, "invsqrt", 0.0)


def test_dropped_triangular_factor_caught(monkeypatch):
    real = sla.solve_triangular
    monkeypatch.setattr(methods.sla, "solve_triangular",
                        lambda R, g, lower=False, trans=0: g if np.ndim(g) == 1 else real(R, g, lower=lower, trans=trans))
    _fails(tm.test_polynomial_exactness)


def test_wrong_rhs_column_caught(monkeypatch):
    real = methods.whiten

    def bad(arn):
        w = real(arn)
        w.c = w.Q.T @ (arn.beta * arn.SV[:, 1])
        return w
    monkeypatch.setattr(methods, "whiten", bad)
    _fails(tm.test_polynomial_exactness)


def test_sign_of_shift_caught(monkeypatch):
    real = quadrature.gauss_chebyshev_invsqrt

    def bad(l):
        t, w = real(l)
        return -t, w
    monkeypatch.setattr(methods.quad, "gauss_chebyshev_invsqrt", bad)
    with pytest.raises((AssertionError, np.linalg.LinAlgError, methods.QuadratureError)):
        tm.test_closed_form_equals_integral_form()


def test_weight_formula_caught(monkeypatch):
    def bad(l):
        i = np.arange(1, l + 1, dtype=np.float64)
        x = np.cos((2.0 * i - 1.0) * np.pi / (2.0 * l))
        return (1.0 - x) / (1.0 + x), (2.0 / l) / (1.0 - x)
    monkeypatch.setattr(quadrature, "gauss_chebyshev_invsqrt", bad)
    _fails(tq.test_rule_reproduces_invsqrt, 45)


def test_window_off_by_one_caught(monkeypatch):
    def bad(A, b, m, k, S, extend=False):
        return real(A, b, m, k + 1, S, extend)
    real = arn_mod.truncated_arnoldi
    monkeypatch.setattr(arn_mod, "truncated_arnoldi", bad)
    _fails(ta.test_truncated_relation_band_and_local_orthogonality, 2)


def test_sketch_after_orthogonalisation_caught(monkeypatch):
    """Sketching w after the Gram-Schmidt updates breaks S A V consistency."""
    real = arn_mod.truncated_arnoldi

    def bad(A, b, m, k, S, extend=False):
        r = real(A, b, m, k, S, extend)
        r.SAV = r.SAV.copy()
        r.SAV[:, :-1] = r.SV[:, 1:] * np.diag(r.H, -1)[: r.m_used - 1]
        return r
    monkeypatch.setattr(arn_mod, "truncated_arnoldi", bad)
    _fails(tm.test_polynomial_exactness)


def test_galerkin_rule_in_sgmres_caught(monkeypatch):
    """sGMRES evaluated with the sketched Galerkin node solves (the sFOM integral)
    instead of the least-squares ones of eq. (sGMRES)."""
    def bad(arn, f="invsqrt", tol=1e-13, **kw):
        if f == "inv":
            return real(arn, f, tol, **kw)
        return methods.sfom_quad(arn, f, tol, **kw)
    real = methods.sgmres
    monkeypatch.setattr(methods, "sgmres", bad)
    _fails(tm.test_sgmres_equals_adaptive_integral_of_definition, 12, 2)


def test_remedy_dropped_caught(monkeypatch):
    """R^-1 taken literally for an extremely ill-conditioned R (no Section 2.1 remedy)."""
    import test_oracle_remedy as tr
    monkeypatch.setattr(methods, "regularize", lambda arn, cond_max=methods.COND_MAX: (arn, arn.m_used))
    data = tr.conv2d_m300.__wrapped__()
    _fails(tr.test_truncated_k2_equals_full_orthogonalisation, data, "exp", 0.01)


def test_remedy_keeps_ill_conditioned_columns_caught(monkeypatch):
    """A prefix rule that keeps far too many columns (threshold near 1/u)."""
    import test_oracle_remedy as tr
    real = methods.regularize
    monkeypatch.setattr(methods, "regularize", lambda arn, cond_max=methods.COND_MAX: real(arn, 1e17))
    data = tr.conv2d_m300.__wrapped__()
    _fails(tr.test_truncated_k2_equals_full_orthogonalisation, data, "exp", 0.01)
