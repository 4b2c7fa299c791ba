"""skfab_solve_noalloc (the entry point that allocates nothing) against skfab_solve,
through the C ABI: two calls in a row, the second on a smaller problem, each equal
to the ordinary entry point's result on the same input and within the FP64 parity
tolerance of the oracle; a problem beyond the static workspace is refused before
any device work."""
import numpy as np
import pytest
import torch

from gpu_common import ctx, problem, device_csr, dev, oracle_run, rel, log
from oracle import methods as ometh
from paper_2208_11447_amd import _native as N
from paper_2208_11447_amd import skfab as sk

pytestmark = pytest.mark.gpu


def _pair(n, m, s, method, seed):
    A, b, arrs = problem(n, seed=seed)
    Ad = device_csr(arrs)
    p = sk.make_params(f="invsqrt", m=m, k=2, s=s, method=method)
    bd = dev(b)
    x_na = torch.full_like(bd, np.nan)
    log(f"noalloc n={n} m={m} s={s} {method}: solving")
    info = sk.skfab_solve_noalloc(ctx(), Ad, bd, x_na, p)
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(Ad, p))
    x_ref = torch.full_like(bd, np.nan)
    sk.skfab_solve(ctx(), Ad, bd, x_ref, p, ws)
    torch.cuda.synchronize()
    return A, b, info, x_na.cpu().numpy(), x_ref.cpu().numpy()


def test_noalloc_two_calls_then_smaller():
    # first call: the 2D 100 x 100 problem at m = 50 (26 MiB of the 64 MiB array)
    A, b, info, x_na, x_ref = _pair(100, 50, 200, "sfom", 0)
    assert info.status == 0 and info.m_used == 50
    arn, _ = oracle_run(A, b, 50, 2, 200)
    e_or = rel(x_na, ometh.sfom_closed(arn, "invsqrt").x)
    log(f"  call 1: vs skfab_solve {rel(x_na, x_ref):.2e} (bitwise {np.array_equal(x_na, x_ref)}), vs oracle {e_or:.2e}")
    assert rel(x_na, x_ref) <= 1e-13 and e_or < 1e-10
    # second call: smaller problem, other method; the array still holds call 1's data
    A, b, info, x_na, x_ref = _pair(40, 20, 80, "sgmres", 1)
    assert info.status == 0 and info.m_used == 20
    arn, _ = oracle_run(A, b, 20, 2, 80)
    e_or = rel(x_na, ometh.sgmres(arn, "invsqrt", tol=1e-13).x)
    log(f"  call 2: vs skfab_solve {rel(x_na, x_ref):.2e} (bitwise {np.array_equal(x_na, x_ref)}), vs oracle {e_or:.2e}")
    assert rel(x_na, x_ref) <= 1e-13 and e_or < 1e-10


def test_noalloc_refuses_too_large():
    _, b, arrs = problem(100)
    Ad = device_csr(arrs)
    p = sk.make_params(f="invsqrt", m=150, k=2, s=300)
    assert sk.skfab_workspace_bytes(Ad, p) > N.SKFAB_NOALLOC_WS_BYTES
    bd = dev(b)
    x = torch.zeros_like(bd)
    with pytest.raises(sk.SkfabError) as e:
        sk.skfab_solve_noalloc(ctx(), Ad, bd, x, p)
    assert e.value.status == N.SKFAB_ERR_TOO_LARGE
    torch.cuda.synchronize()
    assert torch.count_nonzero(x).item() == 0
