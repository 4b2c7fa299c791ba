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
