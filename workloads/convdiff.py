"""Finite-difference convection-diffusion operators in CSR form.

The operator follows the model problem of the paper's convection-diffusion
experiment (Section 5.1): second-order central differences for diffusion and
first-order upwind differences for convection on the unit square (or cube),
h = 1/(n+1), homogeneous Dirichlet boundary, lexicographic ordering with the
x index fastest (row = i + n*j [+ n*n*l]).

In one dimension the diffusion factor is L = tridiag(-1, 2, -1) and the upwind
convection factor is C = tridiag(-1, 1, 0) (diagonal 1, sub-diagonal -1), so

    A = (D/h^2) * sum_d L_d  +  (1/h) * sum_d c_d * C_d

where L_d, C_d act along axis d (Kronecker products with identities).  With
``paper_direction=True`` (2D only) the y factor uses C^T instead of C, i.e. the
paper's convection field pointing in direction [1, -1] (its Kronecker sum
C (+) C^T).

Rows are emitted with strictly increasing column indices; indices are int32
and values float64.
"""
from __future__ import annotations

import numpy as np


def grid_coefficients(n: int, dim: int, diffusion: float, convection):
    """Return (h, diag, lower[d], upper[d]) stencil weights.

    lower[d] multiplies the neighbour at index-1 along axis d, upper[d] the one
    at index+1.  With upwind convection c_d >= 0 the lower neighbour carries
    the convective term.
    """
    conv = np.broadcast_to(np.asarray(convection, dtype=np.float64), (dim,))
    h = 1.0 / (n + 1)
    dh2 = diffusion / (h * h)
    diag = 2.0 * dim * dh2 + float(np.sum(conv)) / h
    lower = [-dh2 - conv[d] / h for d in range(dim)]
    upper = [-dh2 for _ in range(dim)]
    return h, diag, lower, upper


def convdiff_csr(n: int, dim: int = 2, diffusion: float = 1.0, convection=50.0,
                 paper_direction: bool = False):
    """Build the n^dim x n^dim convection-diffusion matrix as CSR arrays.

    Returns (rowptr int32[N+1], col int32[nnz], val float64[nnz]).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if paper_direction and dim != 2:
        raise ValueError("paper_direction applies to the 2D operator only")
    h, diag, lower, upper = grid_coefficients(n, dim, diffusion, convection)
    if paper_direction:
        # y factor is C^T: the convective weight sits on the upper neighbour
        conv = np.broadcast_to(np.asarray(convection, dtype=np.float64), (dim,))
        dh2 = diffusion / (h * h)
        lower[1] = -dh2
        upper[1] = -dh2 - conv[1] / h
    N = n ** dim
    idx = np.arange(N, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for _ in range(dim):
        coords.append(rem % n)
        rem //= n
    strides = [n ** d for d in range(dim)]
    # neighbour offsets in increasing column order: axes from slowest to fastest below
    # the diagonal, then fastest to slowest above it
    entries = []  # (offset, weight, mask)
    for d in reversed(range(dim)):
        entries.append((-strides[d], lower[d], coords[d] > 0))
    entries.append((0, diag, np.ones(N, dtype=bool)))
    for d in range(dim):
        entries.append((strides[d], upper[d], coords[d] < n - 1))
    counts = np.zeros(N, dtype=np.int64)
    for _, _, mask in entries:
        counts += mask
    rowptr = np.zeros(N + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    pos = rowptr[:-1].copy()
    for off, w, mask in entries:
        rows = idx[mask]
        p = pos[mask]
        col[p] = (rows + off).astype(np.int32)
        val[p] = w
        pos[mask] += 1
    return rowptr.astype(np.int32), col, val


def convdiff_spectrum_bounds(n: int, dim: int, diffusion: float, convection):
    """Closed-form extreme eigenvalues of the (non-paper-direction) operator.

    Each 1D factor a0*I + a_lo*S_down + a_up*S_up with a_lo*a_up > 0 is similar
    (by a diagonal scaling) to a symmetric tridiagonal matrix with off-diagonal
    sqrt(a_lo*a_up), whose eigenvalues are a0 - 2 sqrt(a_lo a_up) cos(p pi/(n+1)),
    p = 1..n.  The Kronecker sum adds one such eigenvalue per axis.
    """
    conv = np.broadcast_to(np.asarray(convection, dtype=np.float64), (dim,))
    h = 1.0 / (n + 1)
    dh2 = diffusion / (h * h)
    lo, hi = 0.0, 0.0
    for d in range(dim):
        a0 = 2.0 * dh2 + conv[d] / h
        alo = dh2 + conv[d] / h
        aup = dh2
        r = 2.0 * np.sqrt(alo * aup)
        lo += a0 - r * np.cos(np.pi / (n + 1))
        hi += a0 - r * np.cos(n * np.pi / (n + 1))
    return lo, hi
