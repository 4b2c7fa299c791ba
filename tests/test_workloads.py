"""Pins for the synthetic input generators (no method arithmetic here)."""
import numpy as np
import pytest
import scipy.sparse as sp

from workloads import convdiff_csr, convdiff_spectrum_bounds, gaussian_rhs, batched_problem_params


def _csr(n, dim, D, c, **kw):
    rp, col, val = convdiff_csr(n, dim, D, c, **kw)
    N = rp.size - 1
    return sp.csr_matrix((val, col, rp), shape=(N, N))


def test_stencil_values_match_formula(golden):
    g = golden("conv_diff_stencils.txt")
    rp, col, val = convdiff_csr(100, 2, 1.0, 50.0)
    d, up, down, nnz = map(float, g["2d_n100"])
    assert rp[-1] == nnz
    assert set(np.unique(val)) == {d, up, down}
    rp, col, val = convdiff_csr(128, 3, 1.0, 100.0)
    d, up, down, nnz = map(float, g["3d_n128"])
    assert rp[-1] == nnz
    assert set(np.unique(val)) == {d, up, down}


@pytest.mark.parametrize("dim,n", [(2, 7), (3, 4)])
def test_matches_kronecker_definition(dim, n):
    """Kronecker construction of the same operator, built independently."""
    D, c = 1.3, 20.0
    h = 1.0 / (n + 1)
    I = sp.identity(n)
    L = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(n, n))
    C = sp.diags([-1, 1], [-1, 0], shape=(n, n))
    if dim == 2:
        K = (D / h**2) * (sp.kron(I, L) + sp.kron(L, I)) + (c / h) * (sp.kron(I, C) + sp.kron(C, I))
    else:
        K = (D / h**2) * (sp.kron(sp.kron(I, I), L) + sp.kron(sp.kron(I, L), I) + sp.kron(sp.kron(L, I), I)) \
            + (c / h) * (sp.kron(sp.kron(I, I), C) + sp.kron(sp.kron(I, C), I) + sp.kron(sp.kron(C, I), I))
    A = _csr(n, dim, D, c)
    assert abs(A - K).max() < 1e-9 * abs(K).max()


def test_paper_direction_is_kronecker_sum():
    """Section 5.1: (D/h^2)(I(x)L + L(x)I) + (1/h)(C (+) C^T) with x fastest."""
    n, D = 6, 1e-3
    h = 1.0 / (n + 1)
    I = sp.identity(n)
    L = sp.diags([-1, 2, -1], [-1, 0, 1], shape=(n, n))
    C = sp.diags([-1, 1], [-1, 0], shape=(n, n))
    K = (D / h**2) * (sp.kron(I, L) + sp.kron(L, I)) + (1 / h) * (sp.kron(I, C) + sp.kron(C.T, I))
    A = _csr(n, 2, D, 1.0, paper_direction=True)
    assert abs(A - K).max() < 1e-12 * abs(K).max()


def test_columns_sorted_and_in_range():
    rp, col, val = convdiff_csr(9, 3, 1.0, 5.0)
    N = rp.size - 1
    for r in range(N):
        cs = col[rp[r]:rp[r + 1]]
        assert np.all(np.diff(cs) > 0)
        assert cs.min() >= 0 and cs.max() < N


@pytest.mark.parametrize("dim,n,c", [(2, 10, 50.0), (3, 5, 100.0)])
def test_spectrum_closed_form(dim, n, c):
    """Derived closed form for the extreme eigenvalues (diagonally similar to a
    symmetric operator) against a dense eigensolver."""
    A = _csr(n, dim, 1.0, c).toarray()
    ev = np.linalg.eigvals(A)
    lo, hi = convdiff_spectrum_bounds(n, dim, 1.0, c)
    assert np.max(np.abs(ev.imag)) < 1e-6 * hi
    assert abs(ev.real.min() - lo) < 1e-7 * hi
    assert abs(ev.real.max() - hi) < 1e-7 * hi


def test_rhs_seeded():
    a = gaussian_rhs(1000, 0)
    b = gaussian_rhs(1000, 0)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, gaussian_rhs(1000, 1))
    B = gaussian_rhs(100, 3, nrhs=4)
    assert B.shape == (100, 4) and B.flags["F_CONTIGUOUS"]


def test_batched_params_ranges():
    ps = batched_problem_params()
    assert len(ps) == 64
    for p in ps:
        assert 256 <= p["n"] <= 1024 and 10 <= p["c"] <= 200 and 80 <= p["m"] <= 250
        assert p["s"] == 2 * p["m"]
