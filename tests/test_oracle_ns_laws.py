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


# --- Harten's entropy fix of the interface Roe flux (section 4.4; reading:
# |lambda| -> (lambda^2 + delta^2) / (2 delta) on the two acoustic waves when
# |lambda| < delta, delta = 0.1 (|u~_n| + c~) at the Roe state) -------------

def _euler_flux(U, d, gamma=1.4):
    """Convective flux along e_d; works on complex states (complex step)."""
    rho = U[0]
    u = U[1:4] / rho
    p = (gamma - 1.0) * (U[4] - 0.5 * rho * (u @ u))
    F = np.empty(5, dtype=U.dtype)
    F[0] = U[1 + d]
    F[1:4] = U[1:4] * u[d]
    F[1 + d] += p
    F[4] = (U[4] + p) * u[d]
    return F


def _jacobian(U, d):
    """dF_d/dU by complex-step differentiation (exact to rounding)."""
    h = 1e-30
    A = np.empty((5, 5))
    for k in range(5):
        Z = U.astype(complex)
        Z[k] += 1j * h
        A[:, k] = _euler_flux(Z, d).imag / h
    return A


def _roe_state(UL, UR, gamma=1.4):
    """Conservative state whose u and H are the square-root-density averages
    (the Euler Jacobian depends on u and H only)."""
    def uh(U):
        u = U[1:4] / U[0]
        p = (gamma - 1.0) * (U[4] - 0.5 * U[0] * (u @ u))
        return u, (U[4] + p) / U[0]
    (uL, HL), (uR, HR) = uh(UL), uh(UR)
    sL, sR = math.sqrt(UL[0]), math.sqrt(UR[0])
    u = (sL * uL + sR * uR) / (sL + sR)
    H = (sL * HL + sR * HR) / (sL + sR)
    E = (H + 0.5 * (gamma - 1.0) * (u @ u)) / gamma
    return np.array([1.0, *u, E])


def _fixed_abs(lam, delta):
    a = abs(lam)
    return (a * a + delta * delta) / (2.0 * delta) if a < delta else a


def _roe_flux_spectral(UL, UR, d, efix=0.1, fix_waves=(0, 2), delta_scale=1.0):
    """(F(UL) + F(UR))/2 - f(A~)(UR - UL)/2 with f(A~) evaluated as a matrix
    function of the Roe-averaged Jacobian: A~ is diagonalisable with the three
    distinct eigenvalues u_n - c, u_n, u_n + c, so f(A~) is the quadratic
    Lagrange interpolant of f on them, evaluated at A~ (no eigenvectors)."""
    A = _jacobian(_roe_state(UL, UR), d)
    ev = np.sort(np.linalg.eigvals(A).real)
    lam = [ev[0], ev[2], ev[4]]                 # u_n - c, u_n, u_n + c
    un, c = lam[1], 0.5 * (lam[2] - lam[0])
    delta = delta_scale * efix * (abs(un) + c)
    f = [_fixed_abs(l, delta) if k in fix_waves else abs(l) for k, l in enumerate(lam)]
    I = np.eye(5)
    fA = np.zeros((5, 5))
    for k in range(3):
        P = I.copy()
        for j in range(3):
            if j != k:
                P = P @ (A - lam[j] * I) / (lam[k] - lam[j])
        fA += f[k] * P
    dU = UR - UL
    return 0.5 * (_euler_flux(UL, d) + _euler_flux(UR, d)) - 0.5 * fA @ dU, A, lam, delta


def _near_sonic_pairs():
    """Face state pairs whose Roe-averaged u_n -+ c lies inside (-delta, delta):
    transonic jets along +d (u_n ~ c) and along -d (u_n ~ -c)."""
    rng = np.random.Generator(np.random.PCG64(2024))
    pairs = []
    for sgn in (1.0, -1.0):
        for _ in range(6):
            rho_l, rho_r = rng.uniform(0.8, 1.2, 2)
            p_l, p_r = rng.uniform(0.6, 0.8, 2)
            c_l = math.sqrt(1.4 * p_l / rho_l)
            ul = rng.uniform(-0.2, 0.2, 3)
            ur = rng.uniform(-0.2, 0.2, 3)
            pairs.append((sgn, cons(rho_l, ul, p_l), cons(rho_r, ur, p_r), c_l, rng.uniform(0.97, 1.05)))
    return pairs


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_entropy_fix_against_matrix_function(oracle_lib, d):
    """Near-sonic faces: the oracle's Roe flux equals the flux built from the
    Roe-averaged Jacobian with Harten's fix on the acoustic eigenvalues; the
    Jacobian satisfies the Roe property A~ (UR - UL) = F(UR) - F(UL)."""
    prm = oracle_lib.make_params("ns")
    active = 0
    for sgn, UL, UR, c_l, mach in _near_sonic_pairs():
        # put the normal velocity of both states near sgn * c
        for U in (UL, UR):
            rho = U[0]
            u = U[1:4] / rho
            p = 0.4 * (U[4] - 0.5 * rho * (u @ u))
            u[d] = sgn * mach * c_l
            U[:] = cons(rho, u, p)
        Fs, A, lam, delta = _roe_flux_spectral(UL, UR, d)
        jump = _euler_flux(UR, d) - _euler_flux(UL, d)
        assert np.abs(A @ (UR - UL) - jump).max() < 1e-12 * np.abs(jump).max()
        acoustic = lam[0] if sgn > 0 else lam[2]
        assert abs(acoustic) < delta              # the fixed branch is the one taken
        active += 1
        F = oracle_lib.ns_roe(prm, UL, UR, d)
        scale = np.abs(F).max()
        assert np.abs(F - Fs).max() < 2e-13 * scale, (d, sgn)
    assert active == 12


def _low_mach_pairs(d):
    """Face state pairs of the Ma = 0.1 Taylor-Green regime: |u_n| < delta, so
    a fix wrongly applied to the contact wave would act."""
    rng = np.random.Generator(np.random.PCG64(77 + d))
    out = []
    for _ in range(8):
        UL = cons(rng.uniform(0.9, 1.1), rng.uniform(-1, 1, 3), rng.uniform(70, 73))
        UR = cons(rng.uniform(0.9, 1.1), rng.uniform(-1, 1, 3), rng.uniform(70, 73))
        out.append((UL, UR))
    return out


@pytest.mark.parametrize("d", [0, 1, 2])
def test_roe_low_mach_against_matrix_function(oracle_lib, d):
    """Low-Mach faces (the Taylor-Green regime): acoustic waves far above
    delta, contact wave below it and left unfixed."""
    prm = oracle_lib.make_params("ns")
    for UL, UR in _low_mach_pairs(d):
        Fs, A, lam, delta = _roe_flux_spectral(UL, UR, d)
        assert abs(lam[1]) < delta < min(abs(lam[0]), abs(lam[2]))
        F = oracle_lib.ns_roe(prm, UL, UR, d)
        assert np.abs(F - Fs).max() < 2e-13 * np.abs(F).max()


def test_roe_entropy_fix_detects_planted_slips(oracle_lib):
    """The matrix-function construction tells the fix apart from plausible
    slips: delta doubled or no fix (near-sonic faces), the fix also applied
    to the contact wave u_n (low-Mach faces).  Each slip moves the flux far
    beyond the parity tolerance."""
    prm = oracle_lib.make_params("ns")
    d = 0
    worst = {"delta x2": np.inf, "no fix": np.inf, "fix on u_n": np.inf}
    for sgn, UL, UR, c_l, mach in _near_sonic_pairs():
        for U in (UL, UR):
            rho = U[0]
            u = U[1:4] / rho
            p = 0.4 * (U[4] - 0.5 * rho * (u @ u))
            u[d] = sgn * mach * c_l
            U[:] = cons(rho, u, p)
        F = oracle_lib.ns_roe(prm, UL, UR, d)
        scale = np.abs(F).max()
        for k, kw in (("delta x2", dict(delta_scale=2.0)), ("no fix", dict(fix_waves=()))):
            worst[k] = min(worst[k], np.abs(F - _roe_flux_spectral(UL, UR, d, **kw)[0]).max() / scale)
    for UL, UR in _low_mach_pairs(d):
        F = oracle_lib.ns_roe(prm, UL, UR, d)
        Fk = _roe_flux_spectral(UL, UR, d, fix_waves=(0, 1, 2))[0]
        worst["fix on u_n"] = min(worst["fix on u_n"], np.abs(F - Fk).max() / np.abs(F).max())
    for k, v in worst.items():
        assert v > 1e-6, (k, v)


def test_entropy_fix_is_continuous_at_delta():
    """The fixed eigenvalue meets |lambda| at |lambda| = delta and stays at or
    above delta / 2 (its value at lambda = 0)."""
    for delta in (0.05, 0.3, 2.0):
        assert abs(_fixed_abs(delta * (1 - 1e-12), delta) - delta) < 1e-11 * delta
        assert _fixed_abs(0.0, delta) == pytest.approx(0.5 * delta, rel=1e-15)
        for l in np.linspace(-delta, delta, 11):
            assert _fixed_abs(l, delta) >= abs(l)
