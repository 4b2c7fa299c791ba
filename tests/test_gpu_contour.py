"""Sketched GMRES for exp(-tau A) b by the contour rule (Sections 4.1, 5.2) through
the C ABI, against the oracle (oracle/contour.py) on the same sketch, m and k.

The device finds the sketched Ritz values with its own Hessenberg QR iteration and
chooses the parabola from them by the same reading as the oracle (which takes
LAPACK's eigenvalues), so the two rules differ only by the rounding of the
eigenvalues: both results lie within the rule's tolerance of the sketched GMRES
approximant.  The oracle's sketched FOM by the same rule is pinned against the
closed form on the CPU; here the device's sGMRES is also checked to approach the
device's closed-form sketched FOM as m grows, and the accepted order and the
contour are reported.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from gpu_common import gpu_solve, log, oracle_run, problem
from oracle import contour as C
from oracle import methods as ometh

pytestmark = pytest.mark.gpu


def rel(x, y):
    return float(np.linalg.norm(x - y) / np.linalg.norm(y))


@pytest.mark.parametrize("n,conv,m,tau", [(30, 50.0, 40, 1e-3), (30, 50.0, 60, 1e-2), (40, 100.0, 50, 5e-3),
                                          (60, 50.0, 80, 1e-3)])
def test_sgmres_exp_contour_parity(n, conv, m, tau):
    A, b, arrs = problem(n, 2, conv, seed=3)
    k, s = 2, 2 * m
    log(f"contour sGMRES exp: n={n} conv={conv} m={m} tau={tau}")
    x, info = gpu_solve(arrs, b, f="exp", fparam=tau, m=m, k=k, s=s, method="sgmres", quad_tol=1e-12, seed=1)
    arn, _ = oracle_run(A, b, m, k, s, seed=1)
    r = C.sgmres_contour(arn, tau, tol=1e-12)
    e = rel(x, r.x)
    truth = sla.expm(-tau * A.toarray()) @ b if A.shape[0] <= 3600 else None
    et = rel(x, truth) if truth is not None else float("nan")
    log(f"  status={info.status} m_used={info.m_used} nodes={info.l_used} (oracle {r.l_used}) "
        f"quad_diff={info.quad_diff:.1e}; vs oracle {e:.2e}; vs expm {et:.2e}")
    assert info.status == 0
    assert info.m_used == r.m_used
    assert e < 1e-9


def test_sgmres_exp_contour_approaches_sfom():
    """As m grows both sketched approximants converge to exp(-tau A) b: at m = 80
    the device's sGMRES (contour) and sFOM (closed form) agree with the dense
    truth and with each other to the accuracy the oracle reaches at that m."""
    A, b, arrs = problem(30, 2, 50.0, seed=2)
    tau, m = 1e-3, 80
    truth = sla.expm(-tau * A.toarray()) @ b
    xg, ig = gpu_solve(arrs, b, f="exp", fparam=tau, m=m, k=2, s=2 * m, method="sgmres", quad_tol=1e-12, seed=4)
    xf, inf_ = gpu_solve(arrs, b, f="exp", fparam=tau, m=m, k=2, s=2 * m, method="sfom", seed=4)
    arn, _ = oracle_run(A, b, m, 2, 2 * m, seed=4)
    eg_or = rel(C.sgmres_contour(arn, tau, tol=1e-12).x, truth)
    eg, ef = rel(xg, truth), rel(xf, truth)
    log(f"m={m}: sGMRES contour vs expm {eg:.2e} (oracle {eg_or:.2e}); sFOM closed vs expm {ef:.2e}")
    assert ig.status == 0 and inf_.status == 0
    assert eg <= 2 * eg_or + 1e-10


def test_sgmres_exp_contour_refusals():
    """The contour form needs tau > 0 and m <= 200; other (f, method) pairs that
    have no evaluation are refused before anything runs."""
    from paper_2208_11447_amd import skfab as sk
    _, b, arrs = problem(20, 2, 50.0)
    for kw in (dict(fparam=0.0, m=30, s=60, method="sgmres"), dict(fparam=1e-2, m=201, s=402, method="sgmres"),
               dict(fparam=1e-2, m=30, s=60, method="sfom_quad")):
        with pytest.raises(sk.SkfabError):
            gpu_solve(arrs, b, f="exp", k=2, **kw)


def test_sgmres_exp_contour_lucky_breakdown():
    """b in an A-invariant subspace of dimension 3 (k = 3): the recurrence stops at
    m_used = 3, the sketched GMRES problem is solved exactly at every node, and the
    contour rule reproduces exp(-tau A) b (dense expm of the 3 x 3 block)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(0)
    blk = np.diag([2.0, 5.0, 9.0]) + 0.5 * rng.standard_normal((3, 3))
    rest = sp.diags(np.linspace(1.0, 9.0, 197))
    A = sp.block_diag([blk, rest]).tocsr()
    A.sort_indices()
    b = np.zeros(200)
    b[:3] = rng.standard_normal(3)
    arrs = (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    tau = 0.3
    x, info = gpu_solve(arrs, b, f="exp", fparam=tau, m=8, k=3, s=40, method="sgmres", quad_tol=1e-12)
    truth = np.zeros(200)
    truth[:3] = sla.expm(-tau * blk) @ b[:3]
    log(f"breakdown: m_used={info.m_used} nodes={info.l_used} rel err {rel(x, truth):.2e}")
    assert info.status == 0 and info.m_used == 3
    assert rel(x, truth) < 1e-10


def test_sgmres_exp_contour_strong_convection():
    """m = 200 on a 100 x 100 grid with strong convection (the largest m of the
    contour form): the device agrees with the oracle."""
    A, b, arrs = problem(100, 2, 60.0, seed=7)
    tau, m, k, s = 2e-3, 200, 2, 400
    x, info = gpu_solve(arrs, b, f="exp", fparam=tau, m=m, k=k, s=s, method="sgmres", quad_tol=1e-12, seed=2)
    arn, _ = oracle_run(A, b, m, k, s, seed=2)
    r = C.sgmres_contour(arn, tau, tol=1e-12)
    e = rel(x, r.x)
    log(f"strong convection: m_used={info.m_used} nodes={info.l_used} (oracle {r.l_used}) vs oracle {e:.2e}")
    assert info.status == 0 and info.m_used == r.m_used
    assert e < 1e-9


def test_sgmres_exp_contour_conditioned_prefix():
    """The Section 2.1 remedy ahead of the contour rule: with cond_max = 300 the
    basis of the previous case is truncated to its conditioned prefix, to the same
    length on both sides, and the contour rule on that prefix agrees with the
    oracle's."""
    A, b, arrs = problem(100, 2, 60.0, seed=7)
    tau, m, k, s = 2e-3, 200, 2, 400
    x, info = gpu_solve(arrs, b, f="exp", fparam=tau, m=m, k=k, s=s, method="sgmres", quad_tol=1e-12, seed=2,
                        cond_max=300.0)
    arn, _ = oracle_run(A, b, m, k, s, seed=2)
    r = C.sgmres_contour(arn, tau, tol=1e-12, cond_max=300.0)
    e = rel(x, r.x)
    log(f"prefix: m_used={info.m_used} (oracle {r.m_used}) of {info.m_basis}, flags={info.flags} "
        f"nodes={info.l_used} (oracle {r.l_used}) vs oracle {e:.2e}")
    assert info.status == 0 and info.flags & 1 and info.m_used == r.m_used < m
    assert e < 1e-9
