"""Seeded right-hand sides."""
from __future__ import annotations

import numpy as np


def gaussian_rhs(N: int, seed: int = 0, nrhs: int = 1) -> np.ndarray:
    """b ~ N(0, 1) from numpy's default_rng(seed); shape (N,) or (N, nrhs) column-major."""
    rng = np.random.default_rng(seed)
    if nrhs == 1:
        return rng.standard_normal(N)
    return np.asfortranarray(rng.standard_normal((nrhs, N)).T)


def ones_rhs(N: int) -> np.ndarray:
    """The normalised all-ones vector of the paper's convection-diffusion test."""
    return np.full(N, 1.0 / np.sqrt(N))
