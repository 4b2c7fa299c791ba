"""Batched form through the C ABI: several 2D convection-diffusion problems of
uneven size, Krylov dimension and convection, each with several right-hand
sides, in one skfab_solve_batched call; every (problem, right-hand side) pair is
checked against the FP64 oracle run on that pair alone (same sketch, m, k), and
against the single-problem GPU path.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_common import ctx, gpu_solve, log, oracle_run, rel
from oracle import methods as ometh
from paper_2208_11447_amd import skfab as sk
from workloads import convdiff_csr, gaussian_rhs

pytestmark = pytest.mark.gpu

# (grid n, convection, m) per problem: N from 1600 to 4096, m from 18 to 44
SPECS = [(40, 10.0, 30), (64, 150.0, 44), (48, 80.0, 18), (56, 40.0, 36)]
NRHS = 3


def build_batch(specs=SPECS, nrhs=NRHS, seed0=100):
    hosts, probs = [], []
    for i, (n, c, m) in enumerate(specs):
        rp, col, val = convdiff_csr(n, 2, 1.0, c)
        N_ = rp.size - 1
        B = gaussian_rhs(N_, seed0 + i, nrhs)  # N x nrhs
        if nrhs == 1:
            B = B[:, None]
        A = sk.CSR.from_numpy(rp, col, val)
        Bt = torch.as_tensor(np.ascontiguousarray(B.T), device="cuda")
        Xt = torch.full_like(Bt, np.nan)
        probs.append(sk.BatchProblem(A, Bt, Xt, m=m, s=2 * m, seed=i))
        hosts.append((sp.csr_matrix((val, col, rp), shape=(N_, N_)), np.asarray(B), (rp, col, val)))
    return hosts, probs


def run_batch(probs, **pkw):
    p = sk.make_params(**pkw)
    ws = sk.alloc_workspace(sk.skfab_batch_workspace_bytes(probs, p))
    info = sk.skfab_solve_batched(ctx(), probs, p, ws)
    torch.cuda.synchronize()
    return [q.X.cpu().numpy() for q in probs], info


@pytest.fixture(scope="module")
def batch():
    return build_batch()


@pytest.mark.parametrize("method", ["sfom", "sgmres"])
def test_batched_matches_oracle(batch, method):
    hosts, probs = batch
    X, info = run_batch(probs, f="invsqrt", k=2, method=method)
    worst = 0.0
    for i, ((A, B, _), q) in enumerate(zip(hosts, probs)):
        for r in range(NRHS):
            assert info[i][r].status == 0, (i, r, info[i][r].status)
            assert info[i][r].m_used == q.m
            arn, _ = oracle_run(A, B[:, r], q.m, 2, q.s, seed=q.seed)
            xr = ometh.sfom_closed(arn, "invsqrt").x if method == "sfom" else ometh.sgmres(arn, "invsqrt",
                                                                                           tol=1e-13).x
            e = rel(X[i][r], xr)
            worst = max(worst, e)
            assert e < 1e-10, (i, r, e)
    log(f"batched {method}: {len(probs)} problems x {NRHS} rhs, worst rel. err vs oracle {worst:.2e}")


def test_batched_equals_single_problem_path(batch):
    hosts, probs = batch
    X, _ = run_batch(probs, f="invsqrt", k=2)
    worst = 0.0
    for i, ((A, B, arrs), q) in enumerate(zip(hosts, probs)):
        for r in range(NRHS):
            xs, inf = gpu_solve(arrs, B[:, r], f="invsqrt", m=q.m, k=2, s=q.s, seed=q.seed)
            assert inf.status == 0
            worst = max(worst, rel(X[i][r], xs))
    log(f"batched vs single-problem GPU path: worst rel. diff {worst:.2e}")
    assert worst < 1e-12


def test_batched_inverse_and_determinism(batch):
    hosts, probs = batch
    X1, info = run_batch(probs, f="inv", k=2)
    X2, _ = run_batch(probs, f="inv", k=2)
    for i, ((A, B, _), q) in enumerate(zip(hosts, probs)):
        assert np.array_equal(X1[i], X2[i]), "batched solve is not bitwise reproducible"
        for r in range(NRHS):
            assert info[i][r].status == 0
            arn, _ = oracle_run(A, B[:, r], q.m, 2, q.s, seed=q.seed)
            assert rel(X1[i][r], ometh.sfom_closed(arn, "inv").x) < 1e-10


def test_batched_breakdown_and_single_rhs():
    """A problem whose right-hand side lies in a 3-dimensional invariant subspace
    (lucky breakdown at m_used = 3) batched with a regular one, one rhs each."""
    hosts, probs = build_batch(specs=[(48, 40.0, 30)], nrhs=1)
    Nb = 1500
    rng = np.random.default_rng(7)
    blk = np.diag(rng.uniform(2.0, 5.0, 3)) + np.triu(rng.uniform(-0.3, 0.3, (3, 3)), 1)
    diag = rng.uniform(1.0, 9.0, Nb)
    A = sp.lil_matrix((Nb, Nb))
    A.setdiag(diag)
    A[:3, :3] = blk
    A = sp.csr_matrix(A)
    A.sort_indices()
    b = np.zeros(Nb)
    b[:3] = rng.standard_normal(3)
    Ad = sk.CSR.from_numpy(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    Bt = torch.as_tensor(b[None, :].copy(), device="cuda")
    probs.append(sk.BatchProblem(Ad, Bt, torch.zeros_like(Bt), m=12, s=40, seed=9))
    X, info = run_batch(probs, f="invsqrt", k=3)
    assert info[1][0].status == 0 and info[1][0].m_used == 3
    import scipy.linalg as sla
    truth = np.zeros(Nb)
    truth[:3] = np.linalg.solve(sla.sqrtm(blk).real, b[:3])
    assert rel(X[1][0], truth) < 1e-10
    assert info[0][0].status == 0 and info[0][0].m_used == 30
    arn, _ = oracle_run(hosts[0][0], hosts[0][1][:, 0], 30, 3, 60, seed=0)
    assert rel(X[0][0], ometh.sfom_closed(arn, "invsqrt").x) < 1e-10


def test_batched_autotune_keeps_results(batch):
    hosts, probs = batch
    p = sk.make_params(f="invsqrt", k=2)
    ws = sk.alloc_workspace(sk.skfab_batch_workspace_bytes(probs, p))
    c = ctx()
    saved = sk.skfab_batch_get_tuning(c)
    try:
        X0, _ = run_batch(probs, f="invsqrt", k=2)
        block, spw, packed = sk.skfab_batch_autotune(c, probs, p, ws, steps=3)
        assert block in (256, 512, 1024) and spw in (1, 2, 4, 8, 16, 32, 64)
        assert not packed or block == 512
        assert sk.skfab_batch_get_tuning(c) == (block, spw, packed)
        log(f"autotuned launch shape on the test batch: block {block}, {spw} slices per wavefront, packed {packed}")
        for blk, s, pk in ((256, 2, True), (512, 8, False), (512, 8, True), (block, spw, packed)):
            sk.skfab_batch_set_tuning(c, blk, s, pk)
            X1, info = run_batch(probs, f="invsqrt", k=2)
            for i in range(len(probs)):
                assert all(info[i][r].status == 0 for r in range(NRHS))
                assert rel(X1[i], X0[i]) < 1e-12
    finally:
        sk.skfab_batch_set_tuning(c, *saved)


def test_batched_timing_counts_step_launches(batch):
    """Event timing of a batched solve: its step launches j = 0 .. max m form one
    timed run, every launch counted, and the assembly one timed launch; the
    result is bitwise the untimed one."""
    _, probs = batch
    c = ctx()
    saved = sk.skfab_batch_get_tuning(c)
    sk.skfab_batch_set_tuning(c, saved[0], saved[1], False)  # one launch per step
    try:
        _timed_batch(probs, c)
    finally:
        sk.skfab_batch_set_tuning(c, *saved)


def _timed_batch(probs, c):
    X0, _ = run_batch(probs, f="invsqrt", k=2)
    p = sk.make_params(f="invsqrt", k=2)
    ws = sk.alloc_workspace(sk.skfab_batch_workspace_bytes(probs, p))
    sk.skfab_timing_enable(c, True, stride=1)
    sk.skfab_timing_read(c, 0)
    sk.skfab_timing_read(c, 1)
    sk.skfab_solve_batched(c, probs, p, ws, want_info=False)
    ms0, n0 = sk.skfab_timing_read(c, 0)
    ms1, n1 = sk.skfab_timing_read(c, 1)
    sk.skfab_timing_enable(c, False)
    torch.cuda.synchronize()
    X1 = [q.X.cpu().numpy() for q in probs]
    mmax = max(q.m for q in probs)
    log(f"batched timing: {n0} step launches in {ms0:.3f} ms, {n1} assembly launch in {ms1:.3f} ms")
    assert n0 == mmax + 1 and ms0 > 0.0
    assert n1 == 1 and ms1 > 0.0
    for a, b in zip(X0, X1):
        assert np.array_equal(a, b)


def _with_tuning(c, block, spw, packed, fn):
    saved = sk.skfab_batch_get_tuning(c)
    sk.skfab_batch_set_tuning(c, block, spw, packed)
    try:
        return fn()
    finally:
        sk.skfab_batch_set_tuning(c, *saved)


@pytest.mark.parametrize("nrhs,prec", [(3, "fp64"), (4, "fp64"), (1, "fp64"), (4, "fp32")])
def test_batched_packed_form_is_bitwise_per_unit_form(nrhs, prec):
    """The packed form of the batched step (one block per chunk for all of a
    problem's right-hand sides, steps 2 <= j < m, 512-thread blocks) gives X bit
    for bit equal to the per-unit form at the same launch shape, and the oracle's
    result per pair."""
    hosts, probs = build_batch(nrhs=nrhs, seed0=300)
    c = ctx()
    X = {}
    for packed in (False, True):
        X[packed], info = _with_tuning(c, 512, 4, packed, lambda: run_batch(probs, f="invsqrt", k=2, prec=prec))
        for i, q in enumerate(probs):
            assert all(info[i][r].status == 0 and info[i][r].m_used == q.m for r in range(nrhs))
    for i in range(len(probs)):
        assert np.array_equal(X[True][i], X[False][i]), i
    if prec == "fp64":
        worst = 0.0
        for i, ((A, B, _), q) in enumerate(zip(hosts, probs)):
            for r in range(nrhs):
                arn, _ = oracle_run(A, B[:, r], q.m, 2, q.s, seed=q.seed)
                worst = max(worst, rel(X[True][i][r], ometh.sfom_closed(arn, "invsqrt").x))
        log(f"packed form, {nrhs} rhs: bitwise the per-unit form; worst rel. err vs oracle {worst:.2e}")
        assert worst < 1e-10


def test_batched_packed_form_with_a_breakdown():
    """Right-hand side 1 of the second problem lies in a 3-dimensional invariant
    subspace (lucky breakdown at m_used = 3, inside the packed form's steps) while
    its other right-hand sides run to m = 12: packed and per-unit forms agree bit
    for bit, the broken-down pair is exact and the others match the oracle."""
    hosts, probs = build_batch(specs=[(48, 40.0, 30)], nrhs=3)
    Nb = 1500
    rng = np.random.default_rng(11)
    blk = np.diag(rng.uniform(2.0, 5.0, 3)) + np.triu(rng.uniform(-0.3, 0.3, (3, 3)), 1)
    A = sp.lil_matrix((Nb, Nb))
    A.setdiag(rng.uniform(1.0, 9.0, Nb))
    A[:3, :3] = blk
    A = sp.csr_matrix(A)
    A.sort_indices()
    B = rng.standard_normal((3, Nb))
    B[1, 3:] = 0.0
    Ad = sk.CSR.from_numpy(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    Bt = torch.as_tensor(B, device="cuda")
    probs.append(sk.BatchProblem(Ad, Bt, torch.zeros_like(Bt), m=12, s=40, seed=9))
    c = ctx()
    X, infos = {}, {}
    for packed in (False, True):
        X[packed], infos[packed] = _with_tuning(c, 512, 2, packed, lambda: run_batch(probs, f="invsqrt", k=2))
    for i in range(len(probs)):
        assert np.array_equal(X[True][i], X[False][i]), i
    info = infos[True]
    assert info[1][1].status == 0 and info[1][1].m_used == 3
    import scipy.linalg as sla
    truth = np.zeros(Nb)
    truth[:3] = np.linalg.solve(sla.sqrtm(blk).real, B[1, :3])
    assert rel(X[True][1][1], truth) < 1e-10
    for r in (0, 2):
        assert info[1][r].status == 0 and info[1][r].m_used == 12
        arn, _ = oracle_run(A, B[r], 12, 2, 40, seed=9)
        assert rel(X[True][1][r], ometh.sfom_closed(arn, "invsqrt").x) < 1e-10
    for r in range(3):
        assert info[0][r].status == 0 and info[0][r].m_used == 30
