"""Pins of the oracle's reference-element operators (section 2.1)."""
import math

import numpy as np
import pytest


@pytest.mark.parametrize("n", range(1, 11))
def test_gauss_legendre_matches_numpy(oracle_lib, n):
    x, w = oracle_lib.gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.abs(x - xr).max() < 1e-15
    assert np.abs(w - wr).max() < 4e-15


def test_p1_closed_form(oracle_lib):
    xs, ws, xf, L, M = oracle_lib.operators(1)
    r3 = math.sqrt(3.0)
    assert np.allclose(xs, [-1 / r3, 1 / r3], atol=2e-16, rtol=0)
    assert np.allclose(xf, [-1.0, 0.0, 1.0], atol=1e-16, rtol=0)
    # l_1(x) = (1 - sqrt3 x)/2, l_2(x) = (1 + sqrt3 x)/2 at -1, 0, 1
    Lref = np.array([[(1 + r3) / 2, (1 - r3) / 2], [0.5, 0.5], [(1 - r3) / 2, (1 + r3) / 2]])
    assert np.abs(L - Lref).max() < 1e-15
    # flux basis on {-1, 0, 1}: x(x-1)/2, 1-x^2, x(x+1)/2; derivatives at +-1/sqrt3
    Mref = np.array([[(2 * x - 1) / 2, -2 * x, (2 * x + 1) / 2] for x in (-1 / r3, 1 / r3)])
    assert np.abs(M - Mref).max() < 1e-15


@pytest.mark.parametrize("p", range(1, 9))
def test_operator_exactness(oracle_lib, p):
    xs, ws, xf, L, M = oracle_lib.operators(p)
    n = p + 1
    assert xf[0] == -1.0 and xf[-1] == 1.0
    assert np.all(np.diff(xs) > 0) and np.all(np.diff(xf) > 0)
    # interior flux points are the (n-1)-point Gauss-Legendre rule
    assert np.abs(xf[1:-1] - np.polynomial.legendre.leggauss(n - 1)[0]).max() < 1e-15
    cond = 10.0 ** (p / 2.0)
    assert np.abs(L.sum(axis=1) - 1.0).max() < 1e-14 * cond
    assert np.abs(M.sum(axis=1)).max() < 1e-13 * cond * n
    for k in range(p + 1):              # L is exact on degree <= p
        assert np.abs(L @ xs ** k - xf ** k).max() < 1e-13 * cond
    for k in range(p + 2):              # M is exact on degree <= p + 1
        dk = k * xs ** (k - 1) if k > 0 else 0.0 * xs
        assert np.abs(M @ xf ** k - dk).max() < 1e-12 * cond * n


@pytest.mark.parametrize("p", range(1, 9))
def test_LM_is_flux_point_differentiation(oracle_lib, p):
    """L M equals the differentiation matrix on the flux points, built here
    from an independent Vandermonde construction."""
    xs, ws, xf, L, M = oracle_lib.operators(p)
    n = p + 1
    V = np.vander(xf, n + 1, increasing=True)
    dV = np.zeros_like(V)
    for k in range(1, n + 1):
        dV[:, k] = k * xf ** (k - 1)
    DF = dV @ np.linalg.inv(V)
    assert np.abs(L @ M - DF).max() < 1e-11 * 10 ** (p / 2)


@pytest.mark.parametrize("p", range(1, 9))
def test_compact_correction_constant(oracle_lib, p):
    """c_L^T L M c_R = l'_{n+1/2}(-1) = (-1)^p / 2 and c_R^T L M c_L = -(-1)^p / 2."""
    xs, ws, xf, L, M = oracle_lib.operators(p)
    n = p + 1
    LM = L @ M
    assert abs(LM[0, n] - (-1) ** p / 2) < 1e-12
    assert abs(LM[n, 0] + (-1) ** p / 2) < 1e-12
