"""s-adaptive solve (skfab_solve_reckless) through the C ABI against the oracle's
loop (methods.solve_reckless): the same sequence of sketch sizes and the same
final approximant.

* A batched-workload pair (problem 7, right-hand side 1: N = 101,124, m = 180)
  whose sketched Ritz values reach the branch cut at s = 2m = 360: both sides
  refuse s = 360 and accept s = 720; x agrees to 1e-10.
* A problem that is fine at the first s returns at that s, bitwise equal to
  skfab_solve there.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_common import ctx, dev, device_csr, gpu_solve, log, problem
from oracle import methods as ometh
from paper_2208_11447_amd import skfab as sk
from workloads import batched_problem_params, convdiff_csr

pytestmark = pytest.mark.gpu


def reckless(arrs, b, s0, s_max, eps_max=0.5, **kw):
    A = device_csr(arrs)
    p = sk.make_params(s=s_max, **kw)
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(A, p))
    p.s = s0
    bd = dev(b)
    x = torch.empty_like(bd)
    info, s_used = sk.skfab_solve_reckless(ctx(), A, bd, x, p, s_max, eps_max, ws)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info, s_used


def test_reckless_recovers_branch_failure():
    q = batched_problem_params(64)[7]
    rp, col, val = convdiff_csr(q["n"], 2, 1.0, q["c"])
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = np.random.default_rng(q["rhs_seedseq"]).standard_normal((4, N))[1]
    log(f"reckless s: N={N} m={q['m']} s0={q['s']}")
    s_max = min(4 * q["s"], 1024)  # (the library's largest sketch)
    x, info, s_used = reckless((rp, col, val), b, q["s"], s_max, f="invsqrt", m=q["m"], k=2,
                               seed=q["sketch_seed"])
    res, s_or, trail = ometh.solve_reckless(A, b, "invsqrt", q["m"], 2, q["s"], s_max, seed=q["sketch_seed"])
    e = float(np.linalg.norm(x - res.x) / np.linalg.norm(res.x))
    log(f"  device s_used={s_used} status={info.status} eps={info.eps_est:.3f}; oracle trail {trail}; rel err {e:.2e}")
    assert info.status == 0 and s_used == s_or == 2 * q["s"]
    assert e < 1e-10


def test_reckless_keeps_good_s():
    _, b, arrs = problem(40, 2, 50.0, seed=6)
    kw = dict(f="invsqrt", m=50, k=2, seed=3)
    x, info, s_used = reckless(arrs, b, 150, 600, **kw)
    x1, info1 = gpu_solve(arrs, b, s=150, **kw)
    assert info.status == 0 and s_used == 150
    assert np.array_equal(x, x1)
