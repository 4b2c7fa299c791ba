"""Storage forms of A in the step kernel: the SELL-64 copy keeps 16-bit column
offsets (col - row) when every offset of A fits [-32768, 32767], and 32-bit
columns otherwise; its values are uint8 indices into a table of A's distinct
values when there are at most 256 of them (0.0, the padding value, counted).
Each column-form case checks the form reported in skfab_info.a_format (bits 0-1)
and the sketched FOM result against the FP64 oracle (same sketch, m, k): matrices
with couplings at the offsets just inside and just outside the 16-bit range, and
a matrix whose far couplings force the 32-bit form on every slice.  The value
table cases check bit 2 of a_format at the 256-value limit and that the table form
gives bitwise the results of the plain form (skfab_set_value_table off), single
and batched.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_common import ctx, device_csr, gpu_solve, log, oracle_run, rel
from oracle import methods as ometh
from paper_2208_11447_amd import skfab as sk
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
    assert info.a_format & 3 == form, (offsets, info.a_format)
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
    assert (i16.a_format & 3, i32.a_format & 3) == (2, 1)
    d = rel(x32, x16)
    log(f"int16 vs int32 column forms on one operator: rel. diff {d:.2e}")
    assert d < 1e-13


def with_diagonal_values(n_grid, ndiag):
    """2D convection-diffusion operator whose diagonal takes ndiag distinct values
    (d + 1e-3 j, j = i mod ndiag): the matrix has ndiag + (off-diagonal values)
    distinct values."""
    rp, col, val = convdiff_csr(n_grid, 2, 1.0, 50.0)
    N = rp.size - 1
    A = sp.csr_matrix((val.copy(), col, rp), shape=(N, N))
    d = A.diagonal()
    A.setdiag(d + 1e-3 * (np.arange(N) % ndiag))
    A = A.tocsr()
    A.sort_indices()
    return A, (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64))


def distinct_with_padding(arrs):
    vals = np.unique(arrs[2])
    return vals.size + (0 if np.any(vals == 0.0) else 1)


def solve_both_forms(arrs, b, **kw):
    """The same solve with the value table allowed and with the plain form forced."""
    x_t, i_t = gpu_solve(arrs, b, **kw)
    sk.skfab_set_value_table(ctx(), False)
    try:
        x_p, i_p = gpu_solve(arrs, b, **kw)
    finally:
        sk.skfab_set_value_table(ctx(), True)
    return x_t, i_t, x_p, i_p


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_value_table_bitwise(prec):
    """Constant-coefficient stencil (a handful of distinct values): the FP64 form
    chooses the table and its result equals the plain form's bit for bit; the FP32
    forms keep their 4-byte values."""
    rp, col, val = convdiff_csr(120, 2, 1.0, 60.0)
    b = gaussian_rhs(rp.size - 1, 2)
    x_t, i_t, x_p, i_p = solve_both_forms((rp, col, val), b, f="invsqrt", m=40, k=2, s=160, prec=prec)
    log(f"value table {prec}: a_format {i_t.a_format} / {i_p.a_format}, "
        f"{distinct_with_padding((rp, col, val))} distinct values")
    assert i_t.status == 0 and i_p.status == 0
    assert i_t.a_format == (6 if prec == "fp64" else 2) and i_p.a_format == 2
    assert np.array_equal(x_t, x_p)


@pytest.mark.parametrize("extra,table", [(0, True), (1, False)])
def test_value_table_limit(extra, table):
    """At most 256 distinct values (0.0 counted) use the table, one more does not;
    both results agree with the oracle and, at the limit, with the plain form."""
    rp, col, val = convdiff_csr(60, 2, 1.0, 50.0)
    base = distinct_with_padding((rp, col, val))  # off-diagonal values, diagonal, 0.0
    ndiag = 256 - (base - 1) + extra
    A, arrs = with_diagonal_values(60, ndiag)
    nd = distinct_with_padding(arrs)
    assert nd == 256 + extra
    b = gaussian_rhs(A.shape[0], 6)
    m, k, s = 30, 2, 120
    x_t, i_t, x_p, i_p = solve_both_forms(arrs, b, f="invsqrt", m=m, k=k, s=s, seed=2)
    log(f"{nd} distinct values: a_format {i_t.a_format}")
    assert bool(i_t.a_format & 4) == table and not (i_p.a_format & 4)
    assert np.array_equal(x_t, x_p)
    arn, _ = oracle_run(A, b, m, k, s, seed=2)
    assert rel(x_t, ometh.sfom_closed(arn, "invsqrt").x) < 1e-10


def test_value_table_batched_bitwise():
    """Batched solve with one problem in each value form: every pair's result equals
    the plain form's bit for bit."""
    rp1, col1, val1 = convdiff_csr(80, 2, 1.0, 40.0)
    _, arrs2 = with_diagonal_values(70, 400)
    mats = [(rp1, col1, val1), arrs2]
    R = 2

    def run():
        probs = []
        for i, (rp, col, val) in enumerate(mats):
            A = sk.CSR.from_numpy(rp, col, val)
            B = torch.as_tensor(np.random.default_rng(10 + i).standard_normal((R, rp.size - 1)), device="cuda")
            probs.append(sk.BatchProblem(A, B, torch.empty_like(B), m=30, s=120, seed=i))
        p = sk.make_params(f="invsqrt", k=2, zeta=8, method="sfom", quad_tol=1e-13)
        ws = sk.alloc_workspace(sk.skfab_batch_workspace_bytes(probs, p))
        info = sk.skfab_solve_batched(ctx(), probs, p, ws)
        torch.cuda.synchronize()
        return [pr.X.cpu().numpy() for pr in probs], info

    x_t, info_t = run()
    sk.skfab_set_value_table(ctx(), False)
    try:
        x_p, info_p = run()
    finally:
        sk.skfab_set_value_table(ctx(), True)
    forms = [[info_t[i][r].a_format for r in range(R)] for i in range(2)]
    log(f"batched value forms: {forms}")
    assert all(f & 4 for f in forms[0]) and not any(f & 4 for f in forms[1])
    for i in range(2):
        assert all(info_t[i][r].status == 0 for r in range(R))
        assert np.array_equal(x_t[i], x_p[i])
