"""The benchmark workloads, named by what they are.

Each entry fixes the synthetic operator, the right-hand side recipe and the
method parameters (m, k, s, zeta, f).  The matrices are generated on demand by
``convdiff_csr``; nothing here performs any of the method's arithmetic.
"""
from __future__ import annotations

import numpy as np

CONFIGS = {
    # 2D, 100x100 grid, diffusion 1, convection (50,50), 5-point upwind stencil
    "convdiff2d_n100_m50": dict(
        n=100, dim=2, diffusion=1.0, convection=50.0, rhs_seed=0, sketch_seed=0,
        m=50, k=2, s=200, zeta=8, funcs=("invsqrt",), methods=("sfom", "sgmres")),
    # 3D, 128^3 grid, convection (100,100,100), 7-point upwind stencil
    "convdiff3d_n128_m200": dict(
        n=128, dim=3, diffusion=1.0, convection=100.0, rhs_seed=0, sketch_seed=0,
        m=200, k=2, s=400, zeta=8, funcs=("invsqrt", "exp"), methods=("sfom",)),
    # precision form of the 2D problem at larger Krylov dimensions
    "convdiff2d_n100_m200_fp32": dict(
        n=100, dim=2, diffusion=1.0, convection=50.0, rhs_seed=0, sketch_seed=0,
        m=200, k=2, s=400, zeta=8, funcs=("invsqrt", "exp"), methods=("sfom",)),
    # the paper's convection-diffusion experiment (Section 5.1): 100x100 grid, diffusion
    # 1e-3, unit convection in direction [1, -1] (C (+) C^T), b = ones / ||ones||, k = 4,
    # s = 2 m_max = 400, Krylov dimensions up to 200; sketch: SRDCT or sparse sign
    "paper51_convdiff2d_n100": dict(
        n=100, dim=2, diffusion=1e-3, convection=1.0, paper_direction=True, rhs="ones", sketch_seed=0,
        m=200, k=4, s=400, zeta=8, funcs=("invsqrt",), methods=("sfom", "sfom_quad", "sgmres")),
    "convdiff2d_n100_m300_fp32": dict(
        n=100, dim=2, diffusion=1.0, convection=50.0, rhs_seed=0, sketch_seed=0,
        m=300, k=2, s=600, zeta=8, funcs=("invsqrt", "exp"), methods=("sfom",)),
}

EXP_TAU = 0.01  # f(z) = exp(-tau z)


def config(name: str) -> dict:
    return dict(CONFIGS[name])


def batched_problem_params(nprob: int = 64, seed: int = 4):
    """Parameters of the batched 2D workload: per problem grid n, convection c,
    Krylov dimension m and sketch size s = 2m, all from default_rng(seed).

    Grids are drawn uniformly in 256..1024 per side, convection magnitude
    uniformly in [10, 200] (used for both axes), m uniformly in 80..250.
    Right-hand sides use numpy SeedSequence(0).spawn(nprob), four per problem.
    """
    rng = np.random.default_rng(seed)
    n = rng.integers(256, 1025, size=nprob)
    c = rng.uniform(10.0, 200.0, size=nprob)
    m = rng.integers(80, 251, size=nprob)
    s = 2 * m
    children = np.random.SeedSequence(0).spawn(nprob)
    return [dict(n=int(n[p]), c=float(c[p]), m=int(m[p]), s=int(s[p]), k=2,
                 zeta=8, nrhs=4, rhs_seedseq=children[p], sketch_seed=p)
            for p in range(nprob)]
