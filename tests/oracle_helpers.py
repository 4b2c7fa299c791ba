"""Small problems shared by the oracle pin tests."""
import numpy as np
import scipy.sparse as sp

from oracle import sketch
from workloads import convdiff_csr, gaussian_rhs


def small_convdiff(n=12, dim=2, D=1.0, c=50.0):
    rp, col, val = convdiff_csr(n, dim, D, c)
    N = rp.size - 1
    return sp.csr_matrix((val, col, rp), shape=(N, N))


def small_problem(n=12, s=64, seed=0, c=50.0):
    A = small_convdiff(n, c=c)
    N = A.shape[0]
    b = gaussian_rhs(N, seed)
    S = sketch.sparse_sign_matrix(N, s, 8, seed)
    return A, b, S


def identity_sketch(N):
    return sp.identity(N, format="csc")


def positive_real_matrix(N=40, seed=0, skew=0.4):
    """A = diag(1..3) + skew * K with K skew-symmetric: Re v^T A v >= 1."""
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((N, N))
    K = (K - K.T) / np.sqrt(N)
    return np.diag(np.linspace(1.0, 3.0, N)) + skew * K


def orthonormal_krylov(A, b, m):
    """Orthonormal basis of K_m(A, b) by Householder QR of the power basis,
    with normalised columns (independent of the Arnoldi code)."""
    N = b.size
    K = np.zeros((N, m))
    v = b / np.linalg.norm(b)
    for j in range(m):
        K[:, j] = v
        v = A @ v
        v = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    return Q


def eps_on(S, U):
    sv = np.linalg.svd(S @ U, compute_uv=False)
    return float(np.max(np.abs(sv ** 2 - 1)))


def dense_f(Ad, b, f, fparam=0.0):
    import scipy.linalg as sla
    if f == "invsqrt":
        return np.real(np.linalg.solve(sla.sqrtm(Ad), b))
    if f == "exp":
        return sla.expm(-fparam * Ad) @ b
    if f == "inv":
        return np.linalg.solve(Ad, b)
    raise ValueError(f)
