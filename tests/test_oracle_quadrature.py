"""Pins for the oracle's quadrature and basis (no GPU)."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

from oracle.quadrature import gauss_jacobi, gauss_legendre, graded_panels, jacobi_unit_weight
from oracle.sem import legendre_table, psi_table


def jacobi_moment(beta, k):
    """int_{-1}^{1} (1+x)^beta x^k dx from x = (1+x) - 1 and the binomial theorem
    (evaluated in 40-digit arithmetic: the alternating sum cancels)."""
    import mpmath
    with mpmath.workdps(40):
        b = mpmath.mpf(beta)
        s = sum(math.comb(k, j) * (-1) ** (k - j) * mpmath.power(2, b + j + 1) / (b + j + 1)
                for j in range(k + 1))
        return float(s)


@pytest.mark.parametrize("beta", [-0.9, -0.5, 0.0, 0.3, 0.8, 1.5])
def test_gauss_jacobi_exact_on_closed_form_moments(beta):
    n = 8
    x, w = gauss_jacobi(n, 0.0, beta)
    for k in range(2 * n):
        ref = jacobi_moment(beta, k)
        assert abs(np.sum(w * x ** k) - ref) <= 1e-13 * max(1.0, abs(ref))


def test_unit_weight_rule():
    y, w = jacobi_unit_weight(6, 0.4)
    for k in range(10):
        assert abs(np.sum(w * y ** k) - 1.0 / (1.4 + k)) < 1e-14


def test_gauss_legendre_exact():
    x, w = gauss_legendre(10)
    for k in range(20):
        ref = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.sum(w * x ** k) - ref) < 1e-14


def test_legendre_recurrence_matches_numpy_and_orthogonality():
    x = np.linspace(-1, 1, 7)
    L = legendre_table(9, x)
    for p in range(9):
        c = np.zeros(p + 1); c[p] = 1
        assert np.allclose(L[p], npleg.legval(x, c), atol=1e-14)
    xq, wq = gauss_legendre(12)
    Lq = legendre_table(9, xq)
    G = (Lq * wq) @ Lq.T
    assert np.allclose(G, np.diag(2.0 / (2 * np.arange(9) + 1)), atol=1e-14)
    assert np.allclose(legendre_table(9, np.array([1.0]))[:, 0], 1.0)
    assert np.allclose(legendre_table(9, np.array([-1.0]))[:, 0], (-1.0) ** np.arange(9))


def test_bubble_derivative_identity():
    """psi_p' = -(2p+1) L_p, which makes every basis derivative a Legendre series."""
    for p in range(1, 10):
        c = np.zeros(p + 2); c[p - 1] = 1.0; c[p + 1] = -1.0     # psi_p in Legendre coefficients
        d = npleg.legder(c)
        ref = np.zeros(len(d)); ref[p] = -(2 * p + 1)
        assert np.allclose(d, ref[:len(d)], atol=1e-12)
    x = np.array([-1.0, 1.0])
    assert np.allclose(psi_table(6, x), 0.0, atol=1e-14)


def test_graded_panels_cover_and_are_graded():
    pan = graded_panels(1.0, 0.01)
    assert pan[0][0] == 0.0 and pan[-1][1] == 1.0
    for (a, b), (c, d) in zip(pan[:-1], pan[1:]):
        assert b == c
    for a, b in pan:
        assert (b - a) <= (a + 0.01) * (1 + 1e-12)
