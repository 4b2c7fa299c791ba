"""Precision form of the 2D 100x100 convection-diffusion problem (m = 200, 300,
s = 2m, k = 2): basis and SpMV in FP32 (and a bfloat16-basis variant) against the
FP64 oracle, with the small problem and the assembly in FP64.

The FP32 and BF16 errors are measured properties of the mixed-precision form, not
parity claims; the bounds below sit above the measured values with margin and
are printed by each test.  The FP64 path is held to the FP64 parity tolerance.

At m = 300 the k = 2 truncated basis of this operator is numerically dependent:
the oracle's sketched basis SV_m has a 2-norm condition number near 1e16, so the
whitened matrix Q^T SAV R^-1 (Section 2.1) is not determined by FP64 arithmetic
and both sides produce sketched Ritz values far to the left of the field of
values (the oracle's exp(-0.01 z) result has norm ~1e10).  There the error
against the oracle is recorded, not bounded; the test checks that the case is
genuinely in that regime and that the library returns a result or one of its
documented numerical statuses rather than an argument or HIP failure.
"""
import numpy as np
import pytest

from gpu_common import problem, gpu_solve, oracle_run, rel, log
from oracle import methods as ometh
from paper_2208_11447_amd import _native as N

pytestmark = pytest.mark.gpu

CASES = [(200, "invsqrt", 0.0), (200, "exp", 0.01), (300, "invsqrt", 0.0), (300, "exp", 0.01)]
BOUND = {"fp64": 1e-10, "fp32": 1e-5, "bf16basis": 1e-1}
U = np.finfo(np.float64).eps / 2
ILL_POSED = 1e-3          # u * cond(SV_m) above this: FP64 does not fix the result


@pytest.fixture(scope="module")
def setup():
    A, b, arrs = problem(100)
    refs = {}
    for m in (200, 300):
        arn, _ = oracle_run(A, b, m, 2, 2 * m)
        refs[m] = (arn, np.linalg.cond(arn.SV))
    return A, b, arrs, refs


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16basis"])
@pytest.mark.parametrize("m,f,tau", CASES)
def test_precision_form(setup, prec, m, f, tau):
    A, b, arrs, refs = setup
    arn, cond_sv = refs[m]
    x, info = gpu_solve(arrs, b, f=f, fparam=tau, m=m, k=2, s=2 * m, method="sfom", prec=prec)
    if info.status == 0:
        xr = ometh.sfom_closed(arn, f, tau).x
        err = rel(x, xr)
    else:
        err = float("nan")
    log(f"precision {prec} m={m} f={f}: rel. err vs FP64 oracle {err:.3e} status={info.status} "
        f"({N.lib().skfab_status_string(info.status).decode()}) cond(SV_m)={cond_sv:.2e} "
        f"rcond={info.rcond_R:.2e} relres={info.arnoldi_relres:.2e}")
    if U * cond_sv > ILL_POSED:
        assert m == 300, "only the m = 300 cases are expected to leave the FP64-determined regime"
        assert info.status in (N.SKFAB_OK, N.SKFAB_ERR_BRANCH, N.SKFAB_ERR_QUAD, N.SKFAB_ERR_RANK)
        return
    assert info.status == 0
    assert err < BOUND[prec]
