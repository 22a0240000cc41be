"""Pins of the oracle's Navier-Stokes pointwise laws (section 4.4)."""
import math

import numpy as np
import pytest


def cons(rho, u, p, gamma=1.4):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (gamma - 1) + 0.5 * rho * u @ u])


def test_convective_flux_closed_form(oracle_lib):
    prm = oracle_lib.make_params("ns")
    rho, u, p = 1.3, np.array([0.4, -0.7, 0.2]), 65.0
    U = cons(rho, u, p)
    for d in range(3):
        F = oracle_lib.ns_flux_conv(prm, U, d)
        E = U[4] / rho
        ref = np.array([rho * u[d], *(rho * u * u[d] + p * np.eye(3)[d]), (rho * E + p) * u[d]])
        assert np.abs(F - ref).max() < 1e-13 * np.abs(ref).max()


def test_roe_consistency_and_supersonic_upwinding(oracle_lib):
    prm = oracle_lib.make_params("ns")
    U = cons(1.1, [0.3, 0.2, -0.5], 70.0)
    for d in range(3):
        assert np.abs(oracle_lib.ns_roe(prm, U, U, d) - oracle_lib.ns_flux_conv(prm, U, d)).max() < 1e-12
    # every wave speed positive and above the entropy-fix threshold: pure upwind
    c = math.sqrt(1.4 * 1.0 / 1.0)
    UL = cons(1.0, [4 * c, 0.1, 0.0], 1.0)
    UR = cons(0.9, [3.8 * c, -0.2, 0.1], 0.95)
    F = oracle_lib.ns_roe(prm, UL, UR, 0)
    assert np.abs(F - oracle_lib.ns_flux_conv(prm, UL, 0)).max() < 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_property(oracle_lib, d):
    """The signed wave sum equals F(UR) - F(UL) (Roe linearisation)."""
    prm = oracle_lib.make_params("ns")
    rng = np.random.Generator(np.random.PCG64(d))
    for _ in range(20):
        UL = cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(50, 90))
        UR = cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(50, 90))
        D = oracle_lib.ns_roe_signed_waves(prm, UL, UR, d)
        jump = oracle_lib.ns_flux_conv(prm, UR, d) - oracle_lib.ns_flux_conv(prm, UL, d)
        assert np.abs(D - jump).max() < 1e-11 * np.abs(jump).max()


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_mirror_symmetry(oracle_lib, d):
    """Reflecting x_d swaps the two states and flips every flux component
    except the normal-momentum one."""
    prm = oracle_lib.make_params("ns")
    rng = np.random.Generator(np.random.PCG64(10 + d))
    P = -np.ones(5)
    P[1 + d] = 1.0
    Q = np.ones(5)
    Q[1 + d] = -1.0                      # state mirror: flip u_d
    for _ in range(10):
        UL = cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(50, 90))
        UR = cons(rng.uniform(0.5, 2), rng.uniform(-1, 1, 3), rng.uniform(50, 90))
        F = oracle_lib.ns_roe(prm, UL, UR, d)
        Fm = oracle_lib.ns_roe(prm, Q * UR, Q * UL, d)
        assert np.abs(Fm - P * F).max() < 1e-12 * np.abs(F).max()


def test_viscous_flux_shear_and_heat(oracle_lib):
    prm = oracle_lib.make_params("ns", Re=200.0, sutherland_s=-1.0)
    mu = 1.0 / 200.0
    g = 1.4
    # linear shear u = a y at uniform rho, p: T uniform, tau_xy = mu a
    rho, a, y, p = 1.0, 0.3, 0.5, 70.0
    u = np.array([a * y, 0.0, 0.0])
    U = cons(rho, u, p)
    G = np.zeros((5, 3))
    G[1, 1] = rho * a
    G[4, 1] = rho * u[0] * a
    Fy = oracle_lib.ns_flux_visc(prm, U, G, 1)
    Fx = oracle_lib.ns_flux_visc(prm, U, G, 0)
    assert np.abs(Fy - [0, mu * a, 0, 0, u[0] * mu * a]).max() < 1e-14
    assert np.abs(Fx - [0, 0, mu * a, 0, 0]).max() < 1e-14
    # fluid at rest with dT/dx = b (T = p / rho, rho uniform): q = kappa b
    b = 2.0
    U = cons(1.0, [0, 0, 0], 70.0)
    G = np.zeros((5, 3))
    G[4, 0] = b / (g - 1.0)              # d(rho E)/dx = rho dT/dx / (gamma - 1)
    Fx = oracle_lib.ns_flux_visc(prm, U, G, 0)
    kappa = mu * g / (g - 1.0) / 0.71
    assert np.abs(Fx - [0, 0, 0, 0, kappa * b]).max() < 1e-13


def test_sutherland_law(oracle_lib):
    """mu(T0) = mu0 and mu(2 T0) from the closed form of Sutherland's law."""
    S = 110.4 / 300.0
    prm = oracle_lib.make_params("ns", Re=1000.0, sutherland_s=S)
    p0 = 1.0 / 1.4 / 0.01
    for fac in (1.0, 2.0):
        U = cons(1.0, [0, 0, 0], p0 * fac)
        G = np.zeros((5, 3))
        G[1, 1] = 1.0                    # du/dy = 1 -> F_v,y momentum-x = mu
        F = oracle_lib.ns_flux_visc(prm, U, G, 1)
        mu = 1e-3 * fac ** 1.5 * (1 + S) / (fac + S)
        assert abs(F[1] - mu) < 1e-15
