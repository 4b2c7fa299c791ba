"""k-truncated modified Gram-Schmidt Arnoldi with on-the-fly sketches.

Follows Algorithm 2 of the paper (Section 4) for the basis part, with the
truncation rule of Section 2.2: the new vector is orthogonalised, in order,
against the previous k basis vectors only (indices below 1 are ignored), by
modified Gram-Schmidt without reorthogonalisation.

Readings of the algorithm (also listed in the design notes):

* Exactly m products with A are formed: v_1..v_m and A v_1..A v_m.  The
  vector v_{m+1} is formed only when ``extend=True`` (needed by the
  Cortinovis-Kressner form of Section 2.2's remark and by the stopping
  estimate pins).
* The sketch of A v_j is taken before orthogonalisation (the algorithm
  sketches w right after w <- A v).
* Breakdown: if h_{j+1,j} <= 1e-14 * ||A v_j|| the Krylov space is invariant;
  the iteration stops with m_used = j (exact on that space).

Indices are 0-based in code: column j holds the paper's v_{j+1}.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BREAKDOWN_TOL = 1e-14


@dataclass
class ArnoldiResult:
    V: np.ndarray        # N x m_used basis (column j = v_{j+1})
    SV: np.ndarray       # s x m_used
    SAV: np.ndarray      # s x m_used
    H: np.ndarray        # (m_used+1) x m_used truncated Hessenberg entries
    beta: float          # ||b||_2
    m_used: int
    v_next: np.ndarray | None = None   # v_{m+1} when extend=True
    breakdown: bool = False


def truncated_arnoldi(A, b: np.ndarray, m: int, k: int, S, extend: bool = False
                      ) -> ArnoldiResult:
    """Run m steps of k-truncated MGS Arnoldi, sketching v_j and A v_j.

    A: anything supporting ``A @ x`` (scipy sparse or dense), b: (N,) float64,
    S: s x N sketch (sparse or dense).
    """
    if k < 1:
        raise ValueError("truncation length k must be >= 1")
    N = b.shape[0]
    s = S.shape[0]
    beta = float(np.linalg.norm(b))
    V = np.zeros((N, m))
    SV = np.zeros((s, m))
    SAV = np.zeros((s, m))
    H = np.zeros((m + 1, m))
    if beta == 0.0:
        return ArnoldiResult(V[:, :0], SV[:, :0], SAV[:, :0], H[:1, :0], 0.0, 0)
    v = b / beta
    m_used = m
    v_next = None
    breakdown = False
    for j in range(m):
        V[:, j] = v
        SV[:, j] = S @ v
        w = A @ v
        SAV[:, j] = S @ w
        if j == m - 1 and not extend:
            break
        norm_av = np.linalg.norm(w)
        for i in range(max(0, j - k + 1), j + 1):
            hij = float(V[:, i] @ w)
            w = w - hij * V[:, i]
            H[i, j] = hij
        hnext = float(np.linalg.norm(w))
        H[j + 1, j] = hnext
        if hnext <= BREAKDOWN_TOL * norm_av:
            m_used = j + 1
            breakdown = True
            break
        v = w / hnext
        if j == m - 1:
            v_next = v
    return ArnoldiResult(V[:, :m_used].copy(), SV[:, :m_used].copy(),
                         SAV[:, :m_used].copy(), H[:m_used + 1, :m_used].copy(),
                         beta, m_used, v_next, breakdown)


def full_arnoldi(A, b: np.ndarray, m: int) -> ArnoldiResult:
    """Standard Arnoldi with full MGS orthogonalisation (k = m), no sketch.

    Used for the FOM approximant of eq. (FOM) and the Arnoldi relation
    eq. (arnoldi_relation).  Returns v_{m+1} as ``v_next``.
    """
    N = b.shape[0]
    eye_sketch = _IdentityOp(N)
    return truncated_arnoldi(A, b, m, m, eye_sketch, extend=True)


class _IdentityOp:
    """S = I (s = N) without forming a matrix."""

    def __init__(self, N: int):
        self.shape = (N, N)

    def __matmul__(self, v):
        return np.array(v, dtype=np.float64, copy=True)


def truncated_basis_vectors(A, b: np.ndarray, m: int, k: int):
    """The basis vectors v_1, v_2, ... of the k-truncated recurrence, one at a time,
    holding only the last k of them (the second pass of Section 4.2).  The same
    operations in the same order as truncated_arnoldi; the vectors agree with the
    first pass's to rounding (NumPy may sum the dot products of a strided column in
    another order).  Stops early at a breakdown."""
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return
    window = []
    v = b / beta
    for j in range(m):
        yield v
        if j == m - 1:
            return
        window.append(v)
        if len(window) > k:
            window.pop(0)
        w = A @ v
        norm_av = np.linalg.norm(w)
        for vi in window[max(0, len(window) - k):]:
            hij = float(vi @ w)
            w = w - hij * vi
        hnext = float(np.linalg.norm(w))
        if hnext <= BREAKDOWN_TOL * norm_av:
            return
        v = w / hnext
