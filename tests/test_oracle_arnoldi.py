"""Pins for the k-truncated Arnoldi recurrence with sketches (Algorithm 2)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import arnoldi as arn_mod
from oracle_helpers import small_problem, identity_sketch


def test_full_arnoldi_relation_and_orthonormality():
    """eq. (arnoldi_relation): A V_m = V_m H_m + h_{m+1,m} v_{m+1} e_m^T, V orthonormal."""
    A, b, _ = small_problem()
    m = 25
    r = arn_mod.full_arnoldi(A, b, m)
    V1 = np.column_stack([r.V, r.v_next])
    # MGS without reorthogonalisation loses orthogonality like u * cond
    assert np.linalg.norm(V1.T @ V1 - np.eye(m + 1)) < 1e-9
    res = A @ r.V - V1 @ r.H
    assert np.linalg.norm(res) < 1e-12 * abs(A).max()
    assert np.allclose(np.tril(r.H, -2), 0)
    assert np.all(np.diag(r.H, -1) > 0)
    assert np.isclose(r.V[:, 0] @ b, np.linalg.norm(b))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_truncated_relation_band_and_local_orthogonality(k):
    A, b, S = small_problem()
    m = 30
    r = arn_mod.truncated_arnoldi(A, b, m, k, S, extend=True)
    V1 = np.column_stack([r.V, r.v_next])
    # the Arnoldi-like relation still holds with a banded H
    res = A @ r.V - V1 @ r.H
    assert np.linalg.norm(res) < 1e-11 * abs(A).max()
    for j in range(m):
        nz = np.nonzero(r.H[:, j])[0]
        assert nz.min() >= max(0, j - k + 1) and nz.max() == j + 1
    G = V1.T @ V1
    # unit vectors; each vector orthogonal to the k before it (derived: the
    # window of k+1 consecutive vectors is orthonormal)
    assert np.allclose(np.diag(G), 1, atol=1e-14)
    for d in range(1, k + 1):
        assert np.max(np.abs(np.diag(G, d))) < 1e-13
    # ... but not to the vector k+1 places back
    assert np.max(np.abs(np.diag(G, k + 1))) > 1e-3


def test_sketches_consistent_with_basis():
    A, b, S = small_problem()
    r = arn_mod.truncated_arnoldi(A, b, 20, 2, S)
    Sd = S.toarray()
    assert np.allclose(r.SV, Sd @ r.V, atol=1e-14)
    assert np.allclose(r.SAV, Sd @ (A @ r.V), rtol=1e-14, atol=1e-12 * abs(r.SAV).max())


def test_exactly_m_matvecs():
    """Reading of the loop bound: m products with A, no v_{m+1}."""
    A, b, S = small_problem()

    class Counting:
        def __init__(self, A):
            self.A, self.count = A, 0

        def __matmul__(self, x):
            self.count += 1
            return self.A @ x

    C = Counting(A)
    r = arn_mod.truncated_arnoldi(C, b, 17, 2, S)
    assert C.count == 17 and r.m_used == 17 and r.v_next is None


def _invariant_block_problem():
    rng = np.random.default_rng(0)
    blk = np.diag([2.0, 5.0, 9.0]) + 0.5 * rng.standard_normal((3, 3))
    rest = sp.random(40, 40, density=0.2, random_state=1) + 5 * sp.identity(40)
    A = sp.block_diag([blk, rest]).tocsr()
    b = np.zeros(43)
    b[:3] = rng.standard_normal(3)
    return A, b


def test_lucky_breakdown_invariant_subspace():
    """b in an invariant subspace of dimension 3 and k >= 3 -> m_used = 3."""
    A, b = _invariant_block_problem()
    r = arn_mod.truncated_arnoldi(A, b, 10, 3, identity_sketch(43))
    assert r.breakdown and r.m_used == 3


def test_truncation_shorter_than_invariant_subspace_cycles():
    """With k = 2 < 3 the new vector is never orthogonalised against the whole
    invariant subspace, so no breakdown occurs; the basis repeats with period 3
    (derived), i.e. V_m is rank deficient."""
    A, b = _invariant_block_problem()
    r = arn_mod.truncated_arnoldi(A, b, 10, 2, identity_sketch(43))
    assert not r.breakdown
    assert np.linalg.matrix_rank(r.V, tol=1e-10) == 3


def test_zero_rhs():
    A, _, S = small_problem()
    r = arn_mod.truncated_arnoldi(A, np.zeros(A.shape[0]), 5, 2, S)
    assert r.m_used == 0 and r.beta == 0.0
