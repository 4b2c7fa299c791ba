"""Reference values of f(A) b for the convergence tables (test infrastructure).

A^(-1/2) b for a sparse A with real positive spectrum (the convection-diffusion
operators here: each one-dimensional factor is similar to a symmetric tridiagonal
matrix) through the integral of Section 1 for the Stieltjes function z^(-1/2):
the Gauss-Chebyshev rule of oracle.quadrature at the scale sigma = sqrt(lambda_min
lambda_max), every node a sparse direct solve (t_i sigma I + A) x = b, orders
doubled until two consecutive results agree to tol.  No Krylov space and no sketch
is involved, so it is independent of the method it serves as the truth for.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import quadrature as quad


def extreme_eigenvalues(A):
    """(|lambda|_min, |lambda|_max): dense eigenvalues for small A, else ARPACK (largest
    magnitude directly, smallest by shift-and-invert at 0).  Only the quadrature's
    scale depends on them, not the value it converges to."""
    A = sp.csc_matrix(A)
    if A.shape[0] <= 2000:
        ev = np.abs(np.linalg.eigvals(A.toarray()))
        return float(ev.min()), float(ev.max())
    big = spla.eigs(A, k=1, which="LM", return_eigenvectors=False, tol=1e-8, ncv=40, maxiter=100000)
    small = spla.eigs(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-8, ncv=40)
    return float(np.abs(small).min()), float(np.abs(big).max())


def invsqrt_apply(A, b: np.ndarray, tol: float = 1e-14, l0: int = 64, lmax: int = 8192):
    A = sp.csc_matrix(A)
    N = A.shape[0]
    lo, hi = extreme_eigenvalues(A)
    sigma = np.sqrt(lo * hi)
    eye = sp.identity(N, format="csc")

    def rule(l):
        t, w = quad.gauss_chebyshev_invsqrt(l)
        acc = np.zeros(N)
        for ti, wi in zip(t, w):
            acc += wi * spla.spsolve(ti * sigma * eye + A, b)
        return acc * np.sqrt(sigma)   # sigma^(-1/2) sum w_i (t_i + A/sigma)^-1 b

    l = l0
    prev = rule(l)
    while True:
        l *= 2
        cur = rule(l)
        if np.linalg.norm(cur - prev) <= tol * np.linalg.norm(cur):
            return cur
        if l >= lmax:
            raise ArithmeticError(f"reference quadrature did not reach {tol} by l = {l}")
        prev = cur
