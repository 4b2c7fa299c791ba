"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances: bit-exact for the sketch pattern (integer work); relative 2-norm
1e-10 for FP64 solves (stated per config); basis vectors compared column by
column with a tolerance that grows with the step index, since two correct
implementations of the recurrence round differently and the truncated basis
amplifies the difference (the approximant itself depends only on the span).
"""
import numpy as np
import pytest
import torch

from gpu_common import (ctx, problem, device_csr, dev, gpu_solve, gpu_arnoldi, oracle_run, rel, log)
from oracle import methods as ometh
from oracle import sketch as osk
from paper_2208_11447_amd import _native as N
from paper_2208_11447_amd import skfab as sk

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


@pytest.mark.parametrize("N,s,zeta,seed,col0", [
    (5000, 200, 8, 0, 0), (3000, 37, 8, 5, 0), (4000, 400, 16, 1, 0), (2000, 9, 4, 2, 0),
    (1000, 600, 8, 7, (1 << 31) - 500),   # counters beyond 32 bits
])
def test_sketch_pattern_bit_exact(N, s, zeta, seed, col0):
    log(f"sketch pattern N={N} s={s} zeta={zeta} seed={seed} col0={col0}")
    rows = torch.empty(N * zeta, dtype=torch.int32, device="cuda")
    signs = torch.empty(N * zeta, dtype=torch.int8, device="cuda")
    sk.skfab_sketch_pattern(ctx(), col0, N, s, zeta, seed, rows, signs)
    r_or, s_or = osk.sparse_sign_pattern(col0 + N, s, zeta, seed, cols=np.arange(col0, col0 + N))
    assert np.array_equal(rows.cpu().numpy().reshape(N, zeta), r_or.astype(np.int32))
    assert np.array_equal(signs.cpu().numpy().reshape(N, zeta), s_or)


@pytest.mark.parametrize("N,s", [(1000, 50), (123457, 400), (10000, 1024)])
def test_sketch_apply(N, s):
    log(f"sketch apply N={N} s={s}")
    v = np.random.default_rng(N).standard_normal(N)
    S = osk.sparse_sign_matrix(N, s, 8, 3)
    ws = sk.alloc_workspace(sk.skfab_sketch_ws_bytes(N, s))
    out = torch.empty(s, dtype=torch.float64, device="cuda")
    sk.skfab_sketch_apply(ctx(), N, s, 8, 3, dev(v), out, ws)
    assert rel(out.cpu().numpy(), S @ v) < 1e-14


@pytest.mark.parametrize("n,m,k,s", [(30, 20, 2, 80), (37, 25, 3, 100), (40, 16, 1, 64), (33, 12, 4, 60),
                                     (31, 20, 6, 80), (29, 18, 8, 72)])
def test_arnoldi_state_parity(n, m, k, s):
    """V, SV, S A V and the truncated Hessenberg entries against the oracle; ragged N."""
    log(f"arnoldi parity n={n} m={m} k={k} s={s}")
    A, b, arrs = problem(n)
    V, SV, SAV, H, info = gpu_arnoldi(arrs, b, m, k, s)
    arn, _ = oracle_run(A, b, m, k, s, extend=True)
    assert info.m_used == m
    assert abs(info.beta - np.linalg.norm(b)) <= 1e-14 * np.linalg.norm(b)
    for j in range(m):
        tol = 1e-13 * 4.0 ** j
        tol = min(tol, 1e-6)
        assert rel(V[:, j], arn.V[:, j]) < tol, j
        assert rel(SV[:, j], arn.SV[:, j]) < tol, j
        assert rel(SAV[:, j], arn.SAV[:, j]) < tol, j
    Ho = arn.H[:m + 1, :m]
    assert np.max(np.abs(H - Ho)) < 1e-8 * np.max(np.abs(Ho))
    assert np.allclose(np.tril(H, -2), 0)
    # first columns must agree to rounding
    assert rel(V[:, :3], arn.V[:, :3]) < 1e-13


CASES_C1 = [
    ("sfom", "invsqrt"), ("sgmres", "invsqrt"), ("sfom_quad", "invsqrt"),
    ("sfom", "inv"), ("sgmres", "inv"),
]


@pytest.mark.parametrize("k", [1, 3, 4, 6])
def test_solve_parity_window_lengths(k):
    """Square-case node solves: the band elimination (k <= 4) and the dense one
    (beyond), each against the oracle on a 2D problem, m = 30."""
    A, b, arrs = problem(40, c=60.0, seed=k)
    m, s = 30, 120
    x, info = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, method="sfom", quad_tol=1e-13)
    assert info.status == 0 and info.m_used == m
    arn, _ = oracle_run(A, b, m, k, s)
    e = rel(x, ometh.sfom_closed(arn, "invsqrt").x)
    log(f"window k={k}: rel. err vs oracle {e:.2e}")
    assert e < 1e-10


def test_high_quadrature_orders_match():
    """Orders 987 and 1395 from the start: groups of more than 1024 nodes (one lane per
    node in the band elimination, each node's U rows in its own slots)."""
    A, b, arrs = problem(40, c=60.0, seed=11)
    m, k, s = 30, 2, 120
    x_hi, info = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, method="sfom", l1=987, l2=1395, lmax=1395)
    assert info.status == 0 and info.l_used in (1395,)
    x_lo, _ = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, method="sfom")
    arn, _ = oracle_run(A, b, m, k, s)
    xr = ometh.sfom_closed(arn, "invsqrt").x
    log(f"orders 987/1395: rel. err vs oracle {rel(x_hi, xr):.2e}, vs default orders {rel(x_hi, x_lo):.2e}")
    assert rel(x_hi, xr) < 1e-10 and rel(x_hi, x_lo) < 1e-10


@pytest.mark.parametrize("method", ["sfom", "sfom_quad", "sgmres"])
def test_solve_parity_m300(method):
    """Krylov dimension above 256: the small-problem kernels in their wider
    register form (up to 512 rows: QR panels, H_hat rows, node solves, pencil),
    2D 200x200 grid, convection 200, m=300, k=2, s=600, f = z^(-1/2).  The
    sketched basis stays well conditioned here (no truncation); the numerically
    dependent case is test_ill_conditioned_basis_remedy."""
    A, b, arrs = problem(200, c=200.0, seed=7)
    m, k, s = 300, 2, 600
    x, info = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, method=method, quad_tol=1e-13)
    assert info.status == 0 and info.m_used == m
    arn, _ = oracle_run(A, b, m, k, s)
    ref = {"sfom": ometh.sfom_closed, "sgmres": ometh.sgmres, "sfom_quad": ometh.sfom_quad}[method]
    xr = (ref(arn, "invsqrt") if method == "sfom" else ref(arn, "invsqrt", tol=1e-13)).x
    err = rel(x, xr)
    log(f"m=300 {method}: rel err vs oracle {err:.3e}  l_used={info.l_used} rcond={info.rcond_R:.3e}")
    assert err < FP64_TOL


@pytest.mark.parametrize("method,f", CASES_C1)
def test_solve_parity_convdiff2d_n100(method, f):
    """2D convection-diffusion, 100x100 grid, m=50, k=2, s=200, zeta=8."""
    log(f"solve parity 2D n=100 method={method} f={f}")
    A, b, arrs = problem(100)
    sk.skfab_set_arnoldi_check(ctx(), True)  # S A V_m sketched too; relres reported
    try:
        x, info = gpu_solve(arrs, b, f=f, m=50, k=2, s=200, method=method, quad_tol=1e-13)
    finally:
        sk.skfab_set_arnoldi_check(ctx(), False)
    assert info.status == 0 and info.m_used == 50
    arn, _ = oracle_run(A, b, 50, 2, 200)
    ref = {"sfom": ometh.sfom_closed, "sgmres": ometh.sgmres, "sfom_quad": ometh.sfom_quad}[method]
    xr = (ref(arn, f) if method == "sfom" else ref(arn, f, tol=1e-13)).x
    err = rel(x, xr)
    log(f"  rel err {err:.3e}  l_used={info.l_used} sigma={info.sigma:.4g} rcond={info.rcond_R:.3e} "
        f"relres={info.arnoldi_relres:.2e}")
    assert err < FP64_TOL
    assert info.arnoldi_relres < 1e-12


@pytest.mark.parametrize("tau", [1e-3, 1e-2])
def test_solve_parity_exp_convdiff2d_n100(tau):
    """f(z) = exp(-tau z), closed form, 2D 100x100 grid, m=50, k=2, s=200."""
    log(f"solve parity exp tau={tau}")
    A, b, arrs = problem(100)
    x, info = gpu_solve(arrs, b, f="exp", fparam=tau, m=50, k=2, s=200, method="sfom")
    arn, _ = oracle_run(A, b, 50, 2, 200)
    xr = ometh.sfom_closed(arn, "exp", tau).x
    err = rel(x, xr)
    log(f"  rel err {err:.3e} |x|={np.linalg.norm(xr):.3e}")
    assert info.status == 0
    assert err < FP64_TOL


def test_polynomial_exactness_gpu():
    """Interpolation corollary on the GPU: deg p <= m-1 gives p(A) b exactly."""
    log("polynomial exactness n=60")
    A, b, arrs = problem(60)
    p = [0.5, -1e-4, 3e-9, -2e-14]
    x, info = gpu_solve(arrs, b, f="poly", poly=p, m=10, k=2, s=40)
    ref = p[-1] * b
    for c in p[-2::-1]:
        ref = A @ ref + c * b
    assert rel(x, ref) < 1e-10


def test_small_problem_hook_parity():
    """The small problem alone, fed the oracle's Arnoldi data."""
    log("small problem hook")
    A, b, arrs = problem(50)
    m, k, s = 30, 2, 120
    arn, S = oracle_run(A, b, m, k, s, extend=True)
    hlast = arn.H[m, m - 1]
    SVext = np.column_stack([arn.SV, hlast * (S @ arn.v_next)])
    for method in ("sfom", "sgmres"):
        p = sk.make_params(f="invsqrt", m=m, k=k, s=s, method=method, quad_tol=1e-13)
        ws = sk.alloc_workspace(sk.skfab_small_workspace_bytes(p))
        y = torch.empty(m, dtype=torch.float64, device="cuda")
        info = sk.skfab_small_problem(ctx(), dev(SVext.T.copy()), dev(arn.H[:m + 1, :m].T.copy()),
                                      arn.beta, p, y, ws)
        ref = (ometh.sfom_closed(arn, "invsqrt") if method == "sfom" else ometh.sgmres(arn, "invsqrt", tol=1e-13))
        assert info.status == 0
        assert rel(arn.V @ y.cpu().numpy(), ref.x) < 1e-11


def test_zero_rhs_gives_zero():
    log("zero rhs")
    _, b, arrs = problem(20)
    x, info = gpu_solve(arrs, np.zeros_like(b), m=10, k=2, s=40)
    assert info.m_used == 0 and np.all(x == 0)


def test_lucky_breakdown():
    """b in an A-invariant subspace of dimension 3 with k = 3: m_used = 3, exact result."""
    log("breakdown")
    import scipy.sparse as sp
    rng = np.random.default_rng(0)
    blk = np.diag([2.0, 5.0, 9.0]) + 0.5 * rng.standard_normal((3, 3))
    rest = sp.diags(np.linspace(1.0, 9.0, 197))
    A = sp.block_diag([blk, rest]).tocsr()
    A.sort_indices()
    b = np.zeros(200)
    b[:3] = rng.standard_normal(3)
    arrs = (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    x, info = gpu_solve(arrs, b, f="invsqrt", m=8, k=3, s=40)
    import scipy.linalg as sla
    truth = np.zeros(200)
    truth[:3] = np.real(np.linalg.solve(sla.sqrtm(blk), b[:3]))
    assert info.m_used == 3
    assert rel(x, truth) < 1e-10


def test_run_to_run_bitwise_identical():
    log("determinism")
    _, b, arrs = problem(64)
    x1, _ = gpu_solve(arrs, b, m=30, k=2, s=100)
    x2, _ = gpu_solve(arrs, b, m=30, k=2, s=100)
    assert np.array_equal(x1, x2)


def test_seed_matters_and_zeta():
    log("seed/zeta")
    A, b, arrs = problem(40)
    for zeta, seed in ((4, 3), (16, 1)):
        x, info = gpu_solve(arrs, b, m=20, k=2, s=80, zeta=zeta, seed=seed)
        arn, _ = oracle_run(A, b, 20, 2, 80, zeta=zeta, seed=seed)
        assert rel(x, ometh.sfom_closed(arn, "invsqrt").x) < FP64_TOL


def test_timing_stride_counts_launches():
    """Event timing: the recurrence of a solve (step launches j = 0 .. m-1) is one
    timed run whose launches all count, whatever the stride; launches timed one by
    one (here the second pass of the two-pass form) follow skfab_timing_enable(n):
    every n-th.  A negative n is refused; timing leaves x unchanged."""
    A, b, arrs = problem(30)
    m = 20
    Ad = device_csr(arrs)
    bd = dev(b)
    c = ctx()
    for two_pass in (False, True):
        p = sk.make_params(m=m, k=2, s=80, two_pass=two_pass)
        ws = sk.alloc_workspace(sk.skfab_workspace_bytes(Ad, p))
        x0 = torch.empty_like(bd)
        x1 = torch.empty_like(bd)
        sk.skfab_solve(c, Ad, bd, x0, p, ws, want_info=False)
        for stride, solves in ((1, 2), (3, 3)):
            sk.skfab_timing_enable(c, True, stride=stride)
            sk.skfab_timing_read(c, 0)
            for _ in range(solves):
                sk.skfab_solve(c, Ad, bd, x1, p, ws, want_info=False)
            ms, n = sk.skfab_timing_read(c, 0)
            sk.skfab_timing_enable(c, False)
            want = solves * m  # the runs (the extension pass j = m is not timed)
            if two_pass:  # second-pass launches j = 0 .. m-1, one by one
                want += (solves * m + stride - 1) // stride
            log(f"two_pass={two_pass} stride={stride} solves={solves}: {n} launches, {ms:.3f} ms")
            assert n == want, (two_pass, stride, n, want)
            assert ms > 0.0
        torch.cuda.synchronize()
        assert torch.equal(x0, x1)
    with pytest.raises(RuntimeError):
        sk.skfab_timing_enable(c, True, stride=-2)


@pytest.mark.parametrize("method", ["sfom", "sfom_quad", "sgmres"])
def test_ill_conditioned_basis_remedy(method):
    """2D 100x100 grid, convection 60, m = 300, k = 2, s = 600: the truncated basis
    is numerically dependent (cond(SV_m) ~ 1e16).  Section 2.1's remedy on both
    sides (longest prefix with kappa_F(R_j) <= 1e10): every method agrees with the
    oracle, and the result with the fully orthogonalised oracle run (k = m)."""
    A, b, arrs = problem(100, c=60.0, seed=3)
    m, k, s = 300, 2, 600
    log(f"ill-conditioned basis m={m} method={method}")
    x, info = gpu_solve(arrs, b, f="invsqrt", m=m, k=k, s=s, method=method, quad_tol=1e-13)
    arn, _ = oracle_run(A, b, m, k, s)
    ref = {"sfom": ometh.sfom_closed, "sgmres": ometh.sgmres, "sfom_quad": ometh.sfom_quad}[method]
    r = ref(arn, "invsqrt") if method == "sfom" else ref(arn, "invsqrt", tol=1e-13)
    err = rel(x, r.x) if info.status == 0 else float("nan")
    log(f"  status={info.status} m_used={info.m_used}/{info.m_basis} (oracle {r.m_used}) flags={info.flags} "
        f"rcond={info.rcond_R:.2e} l_used={info.l_used} quad_diff={info.quad_diff:.2e} err={err:.3e}")
    assert np.linalg.cond(arn.SV) > 1e14
    assert info.status == 0
    assert info.flags & N.SKFAB_FLAG_TRUNCATED and info.m_used < m and info.m_basis == m
    assert 1.0 / info.rcond_R <= 1e10
    assert err < FP64_TOL


@pytest.mark.parametrize("f,tau,nrhs", [("invsqrt", 0.0, 3), ("inv", 0.0, 4), ("exp", 1e-3, 2)])
def test_multi_rhs_solve(f, tau, nrhs):
    """skfab_solve with nrhs columns (ld = N): each column equals the single-column
    solve (the batched form for z^(-1/2) and 1/z, to rounding; the column loop for
    exp, bitwise) and the oracle."""
    A, b0, arrs = problem(60, seed=1)
    Nn = A.shape[0]
    m, k, s = 30, 2, 120
    B = np.stack([np.random.default_rng(10 + r).standard_normal(Nn) for r in range(nrhs)])
    Ad = device_csr(arrs)
    p = sk.make_params(f=f, fparam=tau, m=m, k=k, s=s, method="sfom")
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(Ad, p, nrhs))
    Bd = dev(B)
    X = torch.zeros_like(Bd)
    log(f"multi-rhs f={f} nrhs={nrhs}")
    infos = sk.skfab_solve(ctx(), Ad, Bd, X, p, ws)
    torch.cuda.synchronize()
    Xh = X.cpu().numpy()
    for r in range(nrhs):
        assert infos[r].status == 0 and infos[r].m_used == m
        x1, _ = gpu_solve(arrs, B[r], f=f, fparam=tau, m=m, k=k, s=s, method="sfom")
        arn, _ = oracle_run(A, B[r], m, k, s)
        e_or = rel(Xh[r], ometh.sfom_closed(arn, f, tau).x)
        e_1 = rel(Xh[r], x1)
        log(f"  column {r}: vs single solve {e_1:.2e}, vs oracle {e_or:.2e}")
        assert e_or < FP64_TOL
        if f == "exp":
            assert np.array_equal(Xh[r], x1)
        else:
            assert e_1 < 1e-12


def test_quadrature_reporting():
    """info.quad_diff is the accepted relative difference: at most tol unless the
    rounding-floor flag is set, and then at most the floor (1e-10)."""
    A, b, arrs = problem(80, c=40.0, seed=5)
    for method, tol in (("sfom_quad", 1e-8), ("sgmres", 1e-8), ("sfom", 1e-13)):
        x, info = gpu_solve(arrs, b, f="invsqrt", m=40, k=2, s=160, method=method, quad_tol=tol)
        log(f"quad reporting {method}: l_used={info.l_used} quad_diff={info.quad_diff:.2e} flags={info.flags}")
        assert info.status == 0 and info.l_used >= 45
        if info.flags & N.SKFAB_FLAG_QUAD_FLOOR:
            assert tol < info.quad_diff <= 1e-10
        else:
            assert 0.0 <= info.quad_diff <= tol


@pytest.mark.parametrize("method,f,tau", [("sfom", "invsqrt", 0.0), ("sgmres", "invsqrt", 0.0),
                                          ("sfom", "exp", 1e-3)])
def test_two_pass_form(method, f, tau):
    """Section 4.2 two-pass form: the first pass keeps k + 1 basis vectors, the second
    regenerates them (bitwise, fixed-order sums) and accumulates x.  Its x equals the
    one-pass x to rounding and the oracle's two-pass result to the FP64 tolerance; its
    workspace holds k + 1 instead of m basis vectors."""
    A, b, arrs = problem(100, seed=2)
    m, k, s = 50, 2, 200
    Ad = device_csr(arrs)
    p1 = sk.make_params(f=f, fparam=tau, m=m, k=k, s=s, method=method)
    p2 = sk.make_params(f=f, fparam=tau, m=m, k=k, s=s, method=method, two_pass=True)
    ws1, ws2 = sk.skfab_workspace_bytes(Ad, p1), sk.skfab_workspace_bytes(Ad, p2)
    assert ws1 - ws2 >= (m - k - 1) * A.shape[0] * 8
    log(f"two-pass {method} {f}: workspace {ws2 / 2**20:.1f} MiB vs one-pass {ws1 / 2**20:.1f} MiB")
    x1, i1 = gpu_solve(arrs, b, f=f, fparam=tau, m=m, k=k, s=s, method=method)
    x2, i2 = gpu_solve(arrs, b, f=f, fparam=tau, m=m, k=k, s=s, method=method, two_pass=True)
    assert i1.status == 0 and i2.status == 0 and i2.m_used == m
    S = osk.sparse_sign_matrix(A.shape[0], s, 8, 0)
    ref = ometh.two_pass(A, b, f, m, k, S, method, fparam=tau).x
    e12, eor = rel(x2, x1), rel(x2, ref)
    log(f"  two-pass vs one-pass {e12:.2e}, vs oracle {eor:.2e}")
    assert e12 <= 1e-14 and eor < FP64_TOL


@pytest.mark.parametrize("method", ["sfom", "sgmres"])
def test_arnoldi_check_switch(method):
    """The Arnoldi relation check (skfab_set_arnoldi_check) only adds the sketch of
    A u_j and the residual: x is bitwise the same with it on and off, relres is
    below 1e-12 with it and -1 without."""
    _, b, arrs = problem(60)
    kw = dict(f="invsqrt", m=40, k=2, s=160, method=method, quad_tol=1e-13)
    x0, i0 = gpu_solve(arrs, b, **kw)
    sk.skfab_set_arnoldi_check(ctx(), True)
    try:
        x1, i1 = gpu_solve(arrs, b, **kw)
    finally:
        sk.skfab_set_arnoldi_check(ctx(), False)
    log(f"relres off {i0.arnoldi_relres}, on {i1.arnoldi_relres:.2e}")
    assert i0.status == 0 and i1.status == 0
    assert np.array_equal(x0, x1)
    assert i0.arnoldi_relres == -1.0 and 0.0 <= i1.arnoldi_relres < 1e-12
