"""Shared setup for the GPU parity tests (the HIP library through its C ABI)."""
import sys

import numpy as np
import scipy.sparse as sp
import torch

from oracle import arnoldi as oarn
from oracle import methods as ometh
from oracle import sketch as osk
from paper_2208_11447_amd import skfab as sk
from workloads import convdiff_csr, gaussian_rhs


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


_CTX = None


def ctx():
    global _CTX
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a HIP device")
    if _CTX is None:
        _CTX = sk.Context(0)
    return _CTX


def problem(n=30, dim=2, c=50.0, seed=0):
    rp, col, val = convdiff_csr(n, dim, 1.0, c)
    N = rp.size - 1
    A = sp.csr_matrix((val, col, rp), shape=(N, N))
    b = gaussian_rhs(N, seed)
    return A, b, (rp, col, val)


def device_csr(arrs):
    rp, col, val = arrs
    return sk.CSR.from_numpy(rp, col, val)


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def gpu_solve(arrs, b, **pkw):
    A = device_csr(arrs)
    p = sk.make_params(**pkw)
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(A, p))
    bd = dev(b)
    x = torch.empty_like(bd)
    info = sk.skfab_solve(ctx(), A, bd, x, p, ws)
    torch.cuda.synchronize()
    return x.cpu().numpy(), info


def gpu_arnoldi(arrs, b, m, k, s, zeta=8, seed=0):
    A = device_csr(arrs)
    N = A.n
    p = sk.make_params(m=m, k=k, s=s, zeta=zeta, seed=seed)
    ws = sk.alloc_workspace(sk.skfab_workspace_bytes(A, p))
    V = torch.zeros((m, N), dtype=torch.float64, device="cuda")   # column-major N x m
    SV = torch.zeros((m, s), dtype=torch.float64, device="cuda")
    SAV = torch.zeros((m, s), dtype=torch.float64, device="cuda")
    H = torch.zeros((m, m + 1), dtype=torch.float64, device="cuda")
    info = sk.skfab_arnoldi(ctx(), A, dev(b), p, V, SV, SAV, H, ws)
    torch.cuda.synchronize()
    return (V.cpu().numpy().T, SV.cpu().numpy().T, SAV.cpu().numpy().T, H.cpu().numpy().T, info)


def oracle_run(A, b, m, k, s, zeta=8, seed=0, extend=False):
    S = osk.sparse_sign_matrix(A.shape[0], s, zeta, seed)
    arn = oarn.truncated_arnoldi(A, b, m, k, S, extend=extend)
    arn.S = S
    return arn, S


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
