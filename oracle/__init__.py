"""Plain FP64 CPU oracle for sketched FOM / sketched GMRES approximations of f(A)b.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or link
this package: only the test-suite, the smoke check and the CPU-baseline leg of
the benchmark use it.  It shares no code with the HIP implementation; the only
common dependency is the input generator package ``workloads``.

The oracle follows Guettel & Schweitzer, "Randomized sketching for Krylov
approximations of large-scale matrix functions" (arXiv 2208.11447) step by
step, in NumPy/SciPy double precision:

* ``sketch``     - the sparse-sign embedding S (Section 1, eq. (sketch)), drawn
                   from a counter-based SplitMix64 stream (definition in that
                   module's docstring),
* ``arnoldi``    - k-truncated modified Gram-Schmidt Arnoldi with on-the-fly
                   sketches SV_m, SAV_m (Algorithm 2, Section 2.2),
* ``quadrature`` - Gauss-Chebyshev rule for z^(-1/2) after t=(1-x)/(1+x) and
                   the adaptive order sequence (Section 4.1, Section 5.1),
* ``methods``    - whitening QR, the closed form (sFOM'''), the integral forms
                   (sFOM) and (sGMRES), the equivalent forms used as pins, and
                   the sketched stopping estimate and the adaptive-m loop
                   (Section 4.3),
* ``contour``    - the parabolic contour rule for exp(-tau z): sketched GMRES
                   and sketched FOM by Cauchy's integral (Sections 4.1, 5.2),
* ``features``   - Gershgorin bounds (controller features),
* ``mlp``        - the controller network, its loss gradient and Adam step.

Parity status: every function here is pinned by a CPU test against values the
paper prints or against mathematics it fixes (closed forms, invariants,
special cases); see tests/test_oracle_*.py.
"""
from . import sketch, arnoldi, quadrature, methods, contour, features, mlp  # noqa: F401
