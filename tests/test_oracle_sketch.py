"""Pins for the sparse-sign sketch of the oracle (embedding of Section 1)."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import sketch


def test_splitmix64_reference_outputs(golden):
    g = golden("splitmix64_seed0.txt")
    expect = [int(g[k][0], 16) for k in ("out1", "out2", "out3")]
    assert sketch.splitmix64_outputs_int(0, 3) == expect
    # the vectorised stream used by the sketch: column 0 words come from outputs 1..4
    w = sketch.column_words(0, np.array([0]), 8)[0]
    assert int(w[0]) == expect[0] & 0xFFFFFFFF and int(w[1]) == expect[0] >> 32
    assert int(w[2]) == expect[1] & 0xFFFFFFFF and int(w[5]) == expect[2] >> 32


def test_column_stream_offsets():
    """Column i consumes SplitMix64 outputs 4i+1..4i+4."""
    seed = 12345
    outs = sketch.splitmix64_outputs_int(seed, 40)
    w = sketch.column_words(seed, np.arange(10), 8)
    for i in range(10):
        for q in range(8):
            o = outs[4 * i + q // 2]
            assert int(w[i, q]) == (o >> (32 * (q % 2))) & 0xFFFFFFFF


@pytest.mark.parametrize("s,zeta", [(8, 8), (20, 8), (200, 8), (400, 8), (37, 3), (600, 16)])
def test_columns_distinct_rows_unit_norm(s, zeta):
    N = 5000
    rows, signs = sketch.sparse_sign_pattern(N, s, zeta, seed=7)
    assert rows.min() >= 0 and rows.max() < s
    srt = np.sort(rows, axis=1)
    assert np.all(np.diff(srt, axis=1) > 0)
    assert set(np.unique(signs)) <= {-1, 1}
    S = sketch.sparse_sign_matrix(N, s, zeta, seed=7)
    norms = np.sqrt(np.asarray(S.multiply(S).sum(axis=0))).ravel()
    assert np.allclose(norms, 1.0, rtol=0, atol=4e-16)


def test_floyd_subsets_uniform():
    """Brute force: every zeta-subset of a tiny row range is equally likely."""
    s, zeta, N = 6, 3, 120000
    rows, _ = sketch.sparse_sign_pattern(N, s, zeta, seed=3)
    keys = {c: i for i, c in enumerate(itertools.combinations(range(s), zeta))}
    counts = np.zeros(len(keys))
    for r in np.sort(rows, axis=1):
        counts[keys[tuple(r)]] += 1
    chi2 = stats.chisquare(counts)
    assert chi2.pvalue > 1e-4


def test_rows_and_signs_balanced():
    s, N = 200, 200000
    rows, signs = sketch.sparse_sign_pattern(N, s, 8, seed=11)
    counts = np.bincount(rows.ravel(), minlength=s)
    assert stats.chisquare(counts).pvalue > 1e-4
    frac = np.mean(signs == 1)
    assert abs(frac - 0.5) < 4 * 0.5 / np.sqrt(signs.size)


def test_isometry_in_expectation():
    """E ||S v||^2 = ||v||^2 (entries independent, mean-zero signs)."""
    rng = np.random.default_rng(0)
    N, s = 3000, 100
    v = rng.standard_normal(N)
    vals = [np.sum((sketch.sparse_sign_matrix(N, s, 8, seed) @ v) ** 2) for seed in range(300)]
    mean, sd = np.mean(vals), np.std(vals) / np.sqrt(len(vals))
    assert abs(mean - v @ v) < 4 * sd


def test_embedding_distortion_random_subspaces():
    """epsilon of eq. (sketch) on random d-dimensional subspaces, s = 10 d,
    against the textbook Gaussian embedding on the same subspaces: the
    Marchenko-Pastur edge puts its distortion near (1 + sqrt(d/s))^2 - 1."""
    rng = np.random.default_rng(1)
    N, d, s = 4000, 20, 200
    eps, eps_gauss = [], []
    for seed in range(100):
        U, _ = np.linalg.qr(rng.standard_normal((N, d)))
        S = sketch.sparse_sign_matrix(N, s, 8, seed)
        sv = np.linalg.svd(S @ U, compute_uv=False)
        eps.append(np.max(np.abs(sv ** 2 - 1)))
        G = rng.standard_normal((s, N)) / np.sqrt(s)
        svg = np.linalg.svd(G @ U, compute_uv=False)
        eps_gauss.append(np.max(np.abs(svg ** 2 - 1)))
    eps, eps_gauss = np.array(eps), np.array(eps_gauss)
    mp_edge = (1 + np.sqrt(d / s)) ** 2 - 1
    assert eps.max() < 1.0                      # an embedding for every draw
    assert abs(np.median(eps) - np.median(eps_gauss)) < 0.15 * mp_edge
    assert abs(np.median(eps) - mp_edge) < 0.25 * mp_edge


def test_seed_changes_pattern():
    r0, _ = sketch.sparse_sign_pattern(100, 50, 8, seed=0)
    r1, _ = sketch.sparse_sign_pattern(100, 50, 8, seed=1)
    assert not np.array_equal(r0, r1)
    r0b, _ = sketch.sparse_sign_pattern(100, 50, 8, seed=0, cols=np.arange(40, 60))
    assert np.array_equal(r0[40:60], r0b)


# ------------------------------------------------------------------ SRDCT
def test_dct_matrix_matches_library_and_is_orthogonal():
    """F of the SRDCT sketch is the orthonormal DCT-II: SciPy's transform of the unit
    vectors, and F F^T = I."""
    import scipy.fft
    N = 37
    F = sketch.dct_matrix(N)
    ref = scipy.fft.dct(np.eye(N), type=2, norm="ortho", axis=0)
    assert np.max(np.abs(F - ref)) < 1e-14
    assert np.max(np.abs(F @ F.T - np.eye(N))) < 1e-13


def test_srdct_expected_norm_and_rows():
    """E ||S v||^2 = ||v||^2 over the choice of rows: the average over all N rows of
    (N/s) s (F E v)_k^2 / N is ||v||^2 exactly (Parseval); S picks the drawn rows."""
    from workloads import srdct_draws
    N, s = 200, 40
    signs, rows = srdct_draws(N, s, 3)
    v = np.random.default_rng(1).standard_normal(N)
    S = sketch.srdct_matrix(N, signs, rows)
    z = sketch.dct_matrix(N) @ (signs * v)
    assert np.isclose(np.sum(z ** 2), v @ v, rtol=1e-13)           # Parseval
    assert np.allclose(S @ v, np.sqrt(N / s) * z[rows], rtol=1e-12, atol=1e-14)
    mc = np.mean([np.sum((sketch.srdct_matrix(N, *srdct_draws(N, s, t)) @ v) ** 2) for t in range(300)])
    assert abs(mc / (v @ v) - 1) < 0.05


def test_srdct_embedding_distortion():
    """Distortion of the SRDCT embedding on a random 10-dimensional subspace with
    s = 200, N = 2000: well below 1 (an epsilon-subspace embedding, eq. sketch)."""
    from workloads import srdct_draws
    N, s, d = 2000, 200, 10
    U, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((N, d)))
    signs, rows = srdct_draws(N, s, 5)
    sv = np.linalg.svd(sketch.srdct_matrix(N, signs, rows) @ U, compute_uv=False)
    assert np.max(np.abs(sv ** 2 - 1)) < 0.7
