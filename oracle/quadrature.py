"""Quadrature rules (oracle). TEST INFRASTRUCTURE ONLY.

The paper does not give the quadrature for the singular stiffness entries
(Section 3.2 defers to Lemma 4 of Mao and Shen); the rules here are the
standard Gauss-Legendre and Gauss-Jacobi rules from SciPy.

Pinned by tests/test_oracle_quadrature.py against closed-form Jacobi moments.
"""
from functools import lru_cache

import numpy as np
from scipy.special import roots_jacobi, roots_legendre


@lru_cache(maxsize=None)
def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1]."""
    x, w = roots_legendre(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


@lru_cache(maxsize=None)
def gauss_jacobi(n: int, a: float, b: float):
    """n-point Gauss rule on [-1, 1] for the weight (1 - x)^a (1 + x)^b."""
    x, w = roots_jacobi(n, a, b)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gauss_legendre_on(n: int, lo: float, hi: float):
    x, w = gauss_legendre(n)
    return 0.5 * (hi - lo) * x + 0.5 * (hi + lo), 0.5 * (hi - lo) * w


def jacobi_unit_weight(n: int, beta: float):
    """Rule for int_0^1 y^beta g(y) dy:  nodes y_k, weights (scaled)."""
    x, w = gauss_jacobi(n, 0.0, beta)
    return 0.5 * (1.0 + x), w * 2.0 ** (-beta - 1.0)


def graded_panels(length: float, gap: float):
    """Geometric panels [p_j, p_{j+1}] of [0, length] graded toward 0.

    Panel j spans [gap (2^j - 1), gap (2^{j+1} - 1)] (clipped), so each panel is
    no longer than its distance to a singular point at -gap.
    """
    if gap >= length:
        return [(0.0, length)]
    out = []
    j = 0
    while True:
        lo = gap * (2.0 ** j - 1.0)
        hi = gap * (2.0 ** (j + 1) - 1.0)
        if hi >= length:
            out.append((lo, length))
            break
        out.append((lo, hi))
        j += 1
    return out
