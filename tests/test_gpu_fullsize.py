"""GPU checks at the benchmark's full size (3D convection-diffusion, 128^3 grid,
N = 2,097,152, m = 200, k = 2, s = 400), in the launch configuration the
benchmark times: the first Arnoldi steps against the oracle, properties that
hold at any size (polynomial exactness, exactness on an invariant subspace),
and the whole solve for f(z) = exp(-0.01 z) against the oracle's full run
(about 15 s on the host; z^(-1/2) is checked the same way by the benchmark)."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

from gpu_common import ctx, dev, gpu_arnoldi, gpu_solve, oracle_run, rel, log
from oracle import methods as ometh
from workloads import convdiff_csr, gaussian_rhs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    rp, col, val = convdiff_csr(128, 3, 1.0, 100.0)
    N = rp.size - 1
    return sp.csr_matrix((val, col, rp), shape=(N, N)), gaussian_rhs(N, 0), (rp, col, val)


def test_fullsize_first_steps(c2):
    A, b, arrs = c2
    m = 4
    log(f"full-size first {m} Arnoldi steps, N={A.shape[0]}")
    V, SV, SAV, H, info = gpu_arnoldi(arrs, b, m, 2, 400)
    arn, _ = oracle_run(A, b, m, 2, 400, extend=True)
    for j in range(m):
        assert rel(V[:, j], arn.V[:, j]) < 1e-12, j
        assert rel(SV[:, j], arn.SV[:, j]) < 1e-12, j
        assert rel(SAV[:, j], arn.SAV[:, j]) < 1e-12, j
    assert np.max(np.abs(H - arn.H[:m + 1, :m])) < 1e-10 * np.max(np.abs(arn.H))


def test_fullsize_polynomial_exact(c2):
    """Interpolation corollary at full size: deg p <= m-1 gives p(A) b."""
    A, b, arrs = c2
    p = [1.0, 2e-6, -3e-12, 5e-18, 1e-24]
    log("full-size polynomial exactness, m=200")
    x, info = gpu_solve(arrs, b, f="poly", poly=p, m=200, k=2, s=400)
    ref = p[-1] * b
    for c in p[-2::-1]:
        ref = A @ ref + c * b
    assert info.status == 0 and info.m_used == 200
    assert rel(x, ref) < 1e-9


def test_fullsize_invariant_block_exact():
    """A = blockdiag(B, D) of size 2^21 with b supported on the 6x6 block B:
    with k = 6 the recurrence breaks down at m_used = 6 and sketched FOM and
    sketched GMRES both return f(A) b exactly."""
    import scipy.linalg as sla
    N = 1 << 21
    rng = np.random.default_rng(7)
    B = np.diag([3.0, 5.0, 8.0, 13.0, 21.0, 34.0]) + 0.4 * rng.standard_normal((6, 6))
    D = sp.diags(np.linspace(1.0, 100.0, N - 6))
    A = sp.block_diag([sp.csr_matrix(B), D]).tocsr()
    A.sort_indices()
    arrs = (A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data)
    b = np.zeros(N)
    b[:6] = rng.standard_normal(6)
    truth = np.zeros(N)
    truth[:6] = np.real(np.linalg.solve(sla.sqrtm(B), b[:6]))
    for method in ("sfom", "sgmres"):
        log(f"full-size invariant block {method}")
        x, info = gpu_solve(arrs, b, f="invsqrt", m=12, k=6, s=400, method=method)
        assert info.m_used == 6 and info.status == 0
        assert rel(x, truth) < 1e-10


def test_fullsize_exp_matches_oracle(c2):
    """f(z) = exp(-0.01 z), the benchmark's second function: sketched FOM (Pade on
    H_hat) at full size against the FP64 oracle on the same sketch."""
    A, b, arrs = c2
    log("full-size exp(-0.01 z) against the oracle")
    x, info = gpu_solve(arrs, b, f="exp", fparam=0.01, m=200, k=2, s=400, method="sfom")
    assert info.status == 0 and info.m_used == 200
    arn, _ = oracle_run(A, b, 200, 2, 400)
    xr = ometh.sfom_closed(arn, "exp", 0.01).x
    e = rel(x, xr)
    log(f"  rel. err vs oracle {e:.2e}, |x| = {np.linalg.norm(xr):.3e}")
    assert e < 1e-10
