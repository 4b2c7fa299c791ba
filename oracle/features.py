"""Cheap features of a matrix for the learned controller (test infrastructure).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gershgorin_bounds(A) -> tuple[float, float]:
    """min_i (a_ii - sum_{j != i} |a_ij|) and max_i (a_ii + sum_{j != i} |a_ij|):
    the real extent of the union of Gershgorin discs (Gershgorin's theorem)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    r = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    return float(np.min(d - r)), float(np.max(d + r))
