"""Storage forms of A in the step kernel: the SELL-64 copy keeps 16-bit column
offsets (col - row) when every offset of A fits [-32768, 32767], and 32-bit
columns otherwise.  Each case checks the form reported in skfab_info.a_format and
the sketched FOM result against the FP64 oracle (same sketch, m, k): matrices
with couplings at the offsets just inside and just outside the 16-bit range, and
a matrix whose far couplings force the 32-bit form on every slice.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_common import gpu_solve, log, oracle_run, rel
from oracle import methods as ometh
from workloads import convdiff_csr, gaussian_rhs

pytestmark = pytest.mark.gpu

N_GRID = 200  # 2D grid: N = 40,000 > 32,768, so offsets beyond the int16 range exist


def with_couplings(offsets, every=97):
    """2D convection-diffusion operator plus weak couplings A[r, r + o] for each
    offset o (every `every`-th row where r + o is a valid column); the couplings
    are 2 % of the mean diagonal and the same amount is added to the diagonal of
    their rows, so the row dominance of the operator (Gershgorin discs in the
    closed right half-plane) is kept."""
    rp, col, val = convdiff_csr(N_GRID, 2, 1.0, 50.0)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    dmean = float(A.diagonal().mean())
    rows, cols = [np.zeros(0, dtype=np.int64)], [np.zeros(0, dtype=np.int64)]
    for o in offsets:
        r = np.arange(0, N, every)
        c = r + o
        keep = (c >= 0) & (c < N)
        rows.append(r[keep])
        cols.append(c[keep])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    E = sp.csr_matrix((np.full(rows.size, -0.02 * dmean), (rows, cols)), shape=(N, N))
    D = sp.csr_matrix((np.full(rows.size, 0.02 * dmean), (rows, rows)), shape=(N, N))
    A = (A + E + D).tocsr()
    A.sort_indices()
    return A, (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


@pytest.mark.parametrize("offsets,form", [
    ((), 2),                    # stencil only: offsets +-1, +-200
    ((32767, -32768), 2),       # the extreme offsets of the 16-bit form
    ((32768,), 1),              # one step beyond: 32-bit columns
    ((-32769, 35000), 1),
])
def test_matrix_form_and_parity(offsets, form):
    A, arrs = with_couplings(offsets)
    b = gaussian_rhs(A.shape[0], 3)
    m, k, s = 40, 2, 160
    x, info = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, seed=5)
    assert info.status == 0 and info.m_used == m
    assert info.a_format == form, (offsets, info.a_format)
    arn, _ = oracle_run(A, b, m, k, s, seed=5)
    e = rel(x, ometh.sfom_closed(arn, "invsqrt").x)
    log(f"offsets {offsets}: storage form {info.a_format}, rel. err vs oracle {e:.2e}")
    assert e < 1e-10


def test_forms_agree_on_one_operator():
    """The same operator once with a zero-valued far coupling stored explicitly
    (forcing the 32-bit form) and once without it: the two results agree to
    rounding (the zero entries add nothing)."""
    A, arrs = with_couplings(())
    rp, col, val = arrs
    N = rp.size - 1
    b = gaussian_rhs(N, 4)
    x16, i16 = gpu_solve(arrs, b, f="invsqrt", m=30, k=2, s=120, seed=1)
    # explicit zero at (0, N - 1): offset N - 1 = 39,999 > 32,767 (last entry of row 0)
    e1 = int(rp[1])
    arrs32 = (np.concatenate([rp[:1], rp[1:] + 1]).astype(np.int32),
              np.insert(col, e1, N - 1).astype(np.int32),
              np.insert(val, e1, 0.0))
    x32, i32 = gpu_solve(arrs32, b, f="invsqrt", m=30, k=2, s=120, seed=1)
    assert (i16.a_format, i32.a_format) == (2, 1)
    d = rel(x32, x16)
    log(f"int16 vs int32 column forms on one operator: rel. diff {d:.2e}")
    assert d < 1e-13
