"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds problem generators only (matrices, right-hand sides, the
parameter draws of the batched workload). It contains none of the arithmetic
of the sketched Krylov method itself.
"""
from .convdiff import convdiff_csr, convdiff_spectrum_bounds, grid_coefficients
from .rhs import gaussian_rhs, ones_rhs
from .configs import CONFIGS, config, batched_problem_params
from .srdct import srdct_draws

__all__ = [
    "convdiff_csr",
    "convdiff_spectrum_bounds",
    "grid_coefficients",
    "gaussian_rhs",
    "ones_rhs",
    "CONFIGS",
    "config",
    "batched_problem_params",
    "srdct_draws",
]
