"""Quadrature for the Stieltjes function f(z) = z^(-1/2).

Integral representation (Section 1): for a Stieltjes function
f(z) = int_0^inf (t + z)^(-1) dmu(t); for z^(-1/2) the measure is
dmu(t) = t^(-1/2) dt / pi.

Gauss-Chebyshev rule after the change of variables t = (1 - x)/(1 + x), which
maps x in (-1, 1] onto t in [0, inf) (Section 5.1): substituting gives

    z^(-1/2) = (2/pi) int_{-1}^{1} [(1 - x) + z (1 + x)]^(-1) (1 - x^2)^(-1/2) dx,

so the l-point first-kind Gauss-Chebyshev rule, nodes
x_i = cos((2i - 1) pi / (2 l)), reads

    z^(-1/2) ~= sum_i w_i (t_i + z)^(-1),  t_i = (1 - x_i)/(1 + x_i),
                                          w_i = (2/l) / (1 + x_i).

Spectral scaling: z^(-1/2) = sigma^(-1/2) (z/sigma)^(-1/2) for any sigma > 0;
evaluating the rule at z/sigma changes only the quadrature error.

Adaptive order (Section 4.1): start with l1 < l2, accept q_{l2} when
||q_{l1} - q_{l2}|| < tol, else l1 <- l2, l2 <- floor(sqrt(2) l2).  With
l1 = 32, l2 = 45 the sequence 45, 63, 89, 125, 176, ... contains both orders the
paper reports (l = 45 in Section 5.1, l = 176 in Section 5.3).
"""
from __future__ import annotations

import math

import numpy as np

L1_DEFAULT = 32
L2_DEFAULT = 45
# Largest order tried: 1395 is the twelfth order of the sequence from (32, 45);
# the next one, 1972, would double the cost of the last level again.
LMAX_DEFAULT = 1395


def next_order(l2: int) -> int:
    """floor(sqrt(2) * l2), computed exactly with integers."""
    return math.isqrt(2 * l2 * l2)


def order_sequence(l1: int = L1_DEFAULT, l2: int = L2_DEFAULT, lmax: int = LMAX_DEFAULT):
    seq = [l1, l2]
    while True:
        nxt = next_order(seq[-1])
        if nxt > lmax:
            break
        seq.append(nxt)
    return seq


def gauss_chebyshev_invsqrt(l: int):
    """Shifts t_i and weights w_i of the l-point rule for z^(-1/2)."""
    i = np.arange(1, l + 1, dtype=np.float64)
    x = np.cos((2.0 * i - 1.0) * np.pi / (2.0 * l))
    t = (1.0 - x) / (1.0 + x)
    w = (2.0 / l) / (1.0 + x)
    return t, w


def scalar_invsqrt_rule(z, l: int, sigma: float = 1.0):
    """sum_i w_i (t_i + z/sigma)^(-1) * sigma^(-1/2) for scalar/array z."""
    t, w = gauss_chebyshev_invsqrt(l)
    z = np.asarray(z, dtype=np.complex128 if np.iscomplexobj(z) else np.float64)
    acc = np.zeros_like(z)
    for ti, wi in zip(t, w):
        acc = acc + wi / (ti + z / sigma)
    return acc / np.sqrt(sigma)
