"""Sparse-sign subspace embedding S (s x N) from a counter-based generator.

The paper requires an epsilon-subspace embedding for K_{m+1}(A, b)
(Section 1, eqs. (sketch) and (sketch_innerproduct)) and uses a subsampled DCT
in its experiments (Section 5.1).  This implementation uses the sparse sign
embedding instead: every column of S has exactly ``zeta`` nonzeros, placed in
distinct rows chosen uniformly at random, each equal to +-1/sqrt(zeta) with an
independent fair sign.

Definition of the random stream (shared as a document with the GPU code, which
implements it independently):

* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): with gamma =
  0x9E3779B97F4A7C15, the n-th output (n >= 1) of the generator seeded with x
  is mix(x + n*gamma mod 2^64), where
      mix(z): z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
              z = (z ^ (z >> 27)) * 0x94D049BB133111EB
              return z ^ (z >> 31)          (all mod 2^64)
* Column i uses outputs n = 4*i + 1, ..., 4*i + 4 of the generator seeded with
  ``seed``: o_t = mix(seed + (4*i + t + 1)*gamma), t = 0..3.  They give eight
  32-bit words, w_q = (o_{q//2} >> (32*(q % 2))) & 0xFFFFFFFF, q = 0..7
  (zeta <= 8; larger zeta continues the same pattern with 4*ceil(zeta/8)
  outputs per column).
* Rows by Robert Floyd's sampling algorithm (a uniform zeta-subset of
  {0..s-1} with exactly zeta draws): for q = 0..zeta-1 let j = s - zeta + q
  and r = floor((w_q >> 1) * (j + 1) / 2^31), a draw in [0, j]; if r was
  already chosen for this column the row is j, otherwise it is r.  (The
  multiply-shift draw deviates from uniform by at most (j+1)/2^31 relative.)
* Sign of entry q: +1 if bit 0 of w_q is 0, else -1.

``zeta`` words per column are consumed, so the general layout uses
``4*ceil(zeta/8)`` SplitMix64 outputs per column; the outputs used by column i
start at n = 4*ceil(zeta/8)*i + 1.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

GAMMA = 0x9E3779B97F4A7C15
MIX1 = 0xBF58476D1CE4E5B9
MIX2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1


def splitmix64_mix_int(z: int) -> int:
    """SplitMix64 output function on a Python int (reference, scalar)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * MIX1) & MASK64
    z = ((z ^ (z >> 27)) * MIX2) & MASK64
    return z ^ (z >> 31)


def splitmix64_outputs_int(seed: int, count: int, start: int = 1):
    """Outputs start..start+count-1 of SplitMix64 seeded with ``seed``."""
    return [splitmix64_mix_int(seed + (start + t) * GAMMA) for t in range(count)]


def _mix_u64(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(MIX1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(MIX2)
        z ^= z >> np.uint64(31)
    return z


def words_per_column(zeta: int) -> int:
    return 8 * ((zeta + 7) // 8)


def column_words(seed: int, cols: np.ndarray, zeta: int) -> np.ndarray:
    """The 32-bit words w_q (uint64 array, shape (len(cols), zeta))."""
    cols = np.asarray(cols, dtype=np.uint64)
    outs_per_col = words_per_column(zeta) // 2
    t = np.arange(outs_per_col, dtype=np.uint64)
    with np.errstate(over="ignore"):
        n = cols[:, None] * np.uint64(outs_per_col) + t[None, :] + np.uint64(1)
        z = np.uint64(seed & MASK64) + n * np.uint64(GAMMA)
    o = _mix_u64(z)
    lo = o & np.uint64(0xFFFFFFFF)
    hi = o >> np.uint64(32)
    w = np.empty((cols.size, 2 * outs_per_col), dtype=np.uint64)
    w[:, 0::2] = lo
    w[:, 1::2] = hi
    return w[:, :zeta]


def sparse_sign_pattern(N: int, s: int, zeta: int = 8, seed: int = 0,
                        cols: np.ndarray | None = None):
    """Rows (int64, shape (ncols, zeta)) and signs (+-1 int8) of the columns.

    Entry q of column i is S[rows[i, q], i] = signs[i, q] / sqrt(zeta).
    """
    if not (1 <= zeta <= s):
        raise ValueError("need 1 <= zeta <= s")
    if cols is None:
        cols = np.arange(N, dtype=np.int64)
    w = column_words(seed, cols, zeta)
    ncols = w.shape[0]
    rows = np.empty((ncols, zeta), dtype=np.int64)
    for q in range(zeta):
        j = s - zeta + q
        r = ((w[:, q] >> np.uint64(1)) * np.uint64(j + 1)) >> np.uint64(31)
        r = r.astype(np.int64)
        if q > 0:
            dup = np.any(rows[:, :q] == r[:, None], axis=1)
            r = np.where(dup, j, r)
        rows[:, q] = r
    signs = np.where((w & np.uint64(1)) == 0, 1, -1).astype(np.int8)
    return rows, signs


def sparse_sign_matrix(N: int, s: int, zeta: int = 8, seed: int = 0) -> sp.csc_matrix:
    """S as a scipy CSC matrix with entries +-1/sqrt(zeta)."""
    rows, signs = sparse_sign_pattern(N, s, zeta, seed)
    data = signs.astype(np.float64).ravel() * (1.0 / np.sqrt(zeta))
    indices = rows.ravel()
    indptr = np.arange(0, N * zeta + 1, zeta, dtype=np.int64)
    return sp.csc_matrix((data, indices, indptr), shape=(s, N))


def apply_sketch(S, v: np.ndarray) -> np.ndarray:
    """S @ v (plain sparse product)."""
    return S @ v


# ------------------------------------------------------------ SRDCT (Section 5.1)
def dct_matrix(N: int, rows=None) -> np.ndarray:
    """Rows of the orthonormal DCT-II matrix F (N x N): F[k, i] = c_k cos(pi k (2i + 1)
    / (2N)), c_0 = sqrt(1/N), c_k = sqrt(2/N) for k >= 1.  The angle is reduced
    exactly in integers: k (2i + 1) mod 4N."""
    k = np.arange(N, dtype=np.int64) if rows is None else np.asarray(rows, dtype=np.int64)
    i = np.arange(N, dtype=np.int64)
    q = (k[:, None] * (2 * i[None, :] + 1)) % (4 * N)
    c = np.where(k == 0, np.sqrt(1.0 / N), np.sqrt(2.0 / N))
    return c[:, None] * np.cos(np.pi * q / (2.0 * N))


def srdct_matrix(N: int, signs: np.ndarray, rows: np.ndarray) -> np.ndarray:
    """S = sqrt(N/s) P F E as a dense s x N matrix (E = diag(signs), P selects
    `rows` of F E).  The factor sqrt(N/s) makes E ||S v||^2 = ||v||^2 over the
    uniform choice of the s rows."""
    s = len(rows)
    return np.sqrt(N / s) * dct_matrix(N, rows) * np.asarray(signs, dtype=np.float64)[None, :]
