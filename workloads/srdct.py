"""Random draws of the subsampled randomized DCT sketch S = P F E.

The paper's convection-diffusion experiment sketches with S = P F E (Section
5.1): E a diagonal of random signs, F a DCT, P a random selection of s of its
rows.  The draws are inputs of both the oracle and the device library; this
module only draws them (numpy default_rng(seed)), with none of the sketch's
arithmetic.
"""
from __future__ import annotations

import numpy as np


def srdct_draws(N: int, s: int, seed: int = 0):
    """(signs int8[N] of E, each +-1 with probability 1/2; rows int32[s] of P,
    distinct indices in [0, N) drawn uniformly without replacement)."""
    if not 1 <= s <= N:
        raise ValueError("need 1 <= s <= N")
    rng = np.random.default_rng(seed)
    signs = np.where(rng.integers(0, 2, size=N) == 0, 1, -1).astype(np.int8)
    rows = rng.choice(N, size=s, replace=False).astype(np.int32)
    return signs, rows
