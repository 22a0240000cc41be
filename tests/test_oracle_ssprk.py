"""Pins of the SSP-RK(5,4) reference (section 4.4's integrator): the
Butcher tableau of its Shu-Osher coefficients satisfies every order
condition up to order 4 and misses one of order 5; the SSP coefficient is
the published 1.508; the linear stability function matches exp(z) to
O(z^5); observed temporal order 4 on the 1-D diffusion reference."""
import math

import numpy as np
import pytest

from oracle import ssprk


def test_order_conditions_and_ssp_coefficient():
    A, b, c = ssprk.butcher()
    conds = [b.sum() - 1, b @ c - 1 / 2, b @ c ** 2 - 1 / 3, b @ (A @ c) - 1 / 6,
             b @ c ** 3 - 1 / 4, b @ (c * (A @ c)) - 1 / 8, b @ (A @ c ** 2) - 1 / 12,
             b @ (A @ (A @ c)) - 1 / 24]
    assert max(abs(x) for x in conds) < 1e-14
    # not order 5 (one of the order-5 conditions fails clearly)
    assert abs(b @ c ** 4 - 1 / 5) > 1e-6 or abs(b @ (A @ (A @ (A @ c))) - 1 / 120) > 1e-6
    a, be = ssprk.shu_osher()
    assert np.all(a >= 0) and np.all(be >= 0)
    assert np.allclose(a[1:].sum(axis=1), 1.0, atol=1e-14)
    ssp = min(a[i, j] / be[i, j] for i in range(1, 6) for j in range(i) if be[i, j] > 0)
    assert 1.508 < ssp < 1.5082


def test_stability_function_matches_exp():
    for z in (0.05, -0.1, 0.2j, -0.3 + 0.1j):
        R = ssprk.step(lambda u: z * u, np.array([1.0 + 0j]), 1.0)[0]
        assert abs(R - np.exp(z)) < 0.2 * abs(z) ** 5


def test_temporal_order_four_on_diffusion(oracle_lib):
    p, N = 3, 8
    xs = oracle_lib.operators(p)[0]
    h = 2 * math.pi / N
    x = np.array([[e * h + (s + 1) * h / 2 for s in xs] for e in range(N)])
    u0 = np.sin(x) + 0.5 * np.sin(3 * x)
    rhs = lambda u: oracle_lib.rhs_1d(u, p, 0.0, 2 * math.pi, scheme="compact")
    T = 0.2
    ref = ssprk.integrate(rhs, u0, T / 400, 400)
    errs = [np.abs(ssprk.integrate(rhs, u0, T / k, k) - ref).max() for k in (20, 40)]
    order = math.log2(errs[0] / errs[1])
    assert 3.7 < order < 4.5, order
