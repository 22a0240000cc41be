"""Pins of the curvilinear Navier-Stokes reference (section 2.3, eqs.
ns:mapped and adj:f, with the fluxes of section 4.4): the pointwise laws
along a direction vector equal the C oracle's axis laws (an independent
code) and are linear in the direction (Roe: invariant under rotations);
affine node sets reproduce the Cartesian C oracle; a rigidly rotated mesh
with the velocity rotated alike rotates the momentum residual; a uniform
flow is preserved on curved meshes where the metric identities hold; the
scheme conserves mass, momentum and energy on a curved periodic mesh."""
import math

import numpy as np
import pytest

from oracle import curvilinear as C
from paper_2608_09615_amd import workloads as W

TWO_PI = 2 * math.pi
BOX = ((0.0, 0.0, 0.0), (TWO_PI, TWO_PI, TWO_PI))


def rotation(a, b, c):
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    Ry = np.array([[math.cos(c), 0, math.sin(c)], [0, 1, 0], [-math.sin(c), 0, math.cos(c)]])
    return Rz @ Rx @ Ry


def cons(rho, u, p, gamma=1.4):
    u = np.asarray(u, dtype=float)
    return np.array([rho, *(rho * u), p / (gamma - 1) + 0.5 * rho * u @ u])


def random_states(rng, k, sonic=False):
    out = []
    for _ in range(k):
        rho, p = rng.uniform(0.7, 1.3), rng.uniform(60, 80)
        u = rng.uniform(-2, 2, 3)
        if sonic:
            u[0] = math.sqrt(1.4 * p / rho) * rng.uniform(0.95, 1.05)
        out.append(cons(rho, u, p))
    return np.array(out)


def test_pointwise_laws_along_axes_equal_the_c_oracle(oracle_lib):
    prm = oracle_lib.make_params("ns", Re=300.0)
    rng = np.random.Generator(np.random.PCG64(5))
    U = random_states(rng, 12)
    G = rng.normal(size=(12, 5, 3))
    for d in range(3):
        e = np.zeros((12, 3))
        e[:, d] = 1.0
        Fc = C.ns_conv_dir(prm, U, e)
        Fv = C.ns_visc_dir(prm, U, G, e)
        for k in range(12):
            rc = oracle_lib.ns_flux_conv(prm, U[k], d)
            rv = oracle_lib.ns_flux_visc(prm, U[k], G[k].reshape(-1), d)
            assert np.abs(Fc[k] - rc).max() < 1e-14 * np.abs(rc).max()
            assert np.abs(Fv[k] - rv).max() < 1e-14 * np.abs(rv).max() + 1e-18
    # Roe along the axes, including near-sonic faces where Harten's fix acts
    for sonic in (False, True):
        UL, UR = random_states(rng, 10, sonic), random_states(rng, 10, sonic)
        for d in range(3):
            n = np.zeros((10, 3))
            n[:, d] = 1.0
            Fr = C.ns_roe_normal(prm, UL, UR, n)
            for k in range(10):
                ref = oracle_lib.ns_roe(prm, UL[k], UR[k], d)
                assert np.abs(Fr[k] - ref).max() < 1e-13 * np.abs(ref).max()


def test_pointwise_laws_linear_in_direction_and_roe_rotation_invariant(oracle_lib):
    prm = oracle_lib.make_params("ns", Re=300.0)
    rng = np.random.Generator(np.random.PCG64(6))
    U = random_states(rng, 8)
    G = rng.normal(size=(8, 5, 3))
    s1, s2 = rng.normal(size=(8, 3)), rng.normal(size=(8, 3))
    a, b = 0.7, -1.3
    for f in (lambda s: C.ns_conv_dir(prm, U, s), lambda s: C.ns_visc_dir(prm, U, G, s)):
        lhs = f(a * s1 + b * s2)
        rhs = a * f(s1) + b * f(s2)
        assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
    # Roe: rotating both states (momentum) and the normal rotates the flux
    Q = rotation(0.4, -0.9, 1.7)
    UL, UR = random_states(rng, 8, sonic=True), random_states(rng, 8)
    n = rng.normal(size=(8, 3))
    n /= np.linalg.norm(n, axis=1)[:, None]
    rot = lambda X: np.concatenate([X[:, :1], X[:, 1:4] @ Q.T, X[:, 4:]], axis=1)
    F = C.ns_roe_normal(prm, UL, UR, n)
    Fq = C.ns_roe_normal(prm, rot(UL), rot(UR), n @ Q.T)
    assert np.abs(Fq - rot(F)).max() < 1e-12 * np.abs(F).max()
    # consistency F(U, U; n) = F_c(U) . n
    assert np.abs(C.ns_roe_normal(prm, UL, UL, n) - C.ns_conv_dir(prm, UL, n)).max() < 1e-12 * np.abs(F).max()


def _sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm):
    """Per-variable change of the C oracle's RHS when its input moves by
    about one ulp, relative to the variable's largest value."""
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    U2 = U * (1.0 + 2.2e-16 * np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, U.shape))
    R2 = oracle_lib.rhs_3d(U2, nel, lo, hi, p, scheme, prm)
    return Ro, [np.abs(R2[:, v] - Ro[:, v]).max() / np.abs(Ro[:, v]).max() for v in range(5)]


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_affine_nodes_reproduce_the_cartesian_oracle(oracle_lib, scheme, p):
    """Straight, axis-aligned elements of three different sizes (q = 1, and
    q = 2 with midpoint nodes): S is diagonal, J^-1 S_dd = 2 / h_d, and the
    curvilinear steps reduce to the Cartesian ones of the C oracle."""
    prm = oracle_lib.make_params("ns", Re=400.0)
    nel = (3, 2, 4)
    lo, hi = (0.0, 0.0, 0.0), (TWO_PI, 0.8 * TWO_PI, 1.2 * TWO_PI)
    U = W.perturbed_tgv_state(nel, p, seed=3 + p, noise=1e-2)
    Ro, sens = _sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm)
    for q in (1, 2):
        R = C.rhs_ns(U, nel, W.mesh_nodes(nel, lo, hi, q=q), p, scheme, prm)
        for v in range(5):
            err = np.abs(R[:, v] - Ro[:, v]).max() / np.abs(Ro[:, v]).max()
            assert err < max(1e-12, 8 * sens[v]), (q, v, err, sens[v])


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_rigid_rotation_rotates_the_momentum_residual(oracle_lib, scheme):
    """Rotating the mesh by Q (S becomes a full matrix: every transverse
    metric term of the gradient, the fluxes and the Roe normal is active) and
    the velocity by Q leaves the mass and energy residuals unchanged and
    rotates the momentum residual."""
    prm = oracle_lib.make_params("ns", Re=400.0)
    nel, p = (3, 2, 3), 2
    lo, hi = (0.0, 0.0, 0.0), (TWO_PI, TWO_PI, TWO_PI)
    U = W.perturbed_tgv_state(nel, p, seed=9, noise=1e-2)
    Q = rotation(0.7, 0.4, -1.1)
    R = C.rhs_ns(U, nel, W.mesh_nodes(nel, lo, hi, q=1), p, scheme, prm)
    Ur = U.copy()
    Ur[:, 1:4] = np.einsum("ij,ej...->ei...", Q, U[:, 1:4])
    Rr = C.rhs_ns(Ur, nel, W.mesh_nodes(nel, lo, hi, q=1, rotation=Q), p, scheme, prm)
    Rq = R.copy()
    Rq[:, 1:4] = np.einsum("ij,ej...->ei...", Q, R[:, 1:4])
    for v in range(5):
        scale = np.abs(R[:, v]).max() if v in (0, 4) else np.abs(R[:, 1:4]).max()
        assert np.abs(Rr[:, v] - Rq[:, v]).max() < 1e-11 * scale, v


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("q,p", [(1, 1), (1, 3), (2, 3), (2, 4)])
def test_uniform_flow_preserved_on_curved_meshes(oracle_lib, scheme, q, p):
    """A uniform flow (all gradients zero, the same flux everywhere) is a
    steady state wherever sum_d D_d S_dm = 0 holds discretely: 2q <= p + 1."""
    prm = oracle_lib.make_params("ns", Re=400.0)
    nel = (4, 3, 4)
    Xg = W.mesh_nodes(nel, *BOX, q=q, displacement=W.periodic_wave_displacement(0.15))
    n = p + 1
    U = np.empty((int(np.prod(nel)), 5, n, n, n))
    for v, val in enumerate(cons(1.1, [0.6, -0.4, 0.3], 70.0)):
        U[:, v] = val
    R = C.rhs_ns(U, nel, Xg, p, scheme, prm)
    # the scale of one flux difference: |F| (p+1)^2 / h
    scale = 80.0 * n ** 2 / (TWO_PI / 4)
    assert np.abs(R).max() < 1e-12 * scale


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_conservation_on_a_curved_mesh(oracle_lib, scheme):
    """sum_e sum_q w_q J R = 0 for the five conserved variables: the
    interface fluxes of the two sides cancel (same Roe flux, same common
    viscous flux, the shared S_d of the face)."""
    prm = oracle_lib.make_params("ns", Re=400.0)
    nel, p = (3, 4, 3), 3
    Xg = W.mesh_nodes(nel, *BOX, q=2, displacement=W.periodic_wave_displacement(0.2))
    U = W.perturbed_tgv_state(nel, p, seed=4, noise=1e-2)
    R = C.rhs_ns(U, nel, Xg, p, scheme, prm)
    _, w = np.polynomial.legendre.leggauss(p + 1)
    W3 = w[:, None, None] * w[None, :, None] * w[None, None, :]
    _, detJ = C.metrics(Xg, p)
    for v in range(5):
        tot = np.sum(W3[None] * detJ * R[:, v])
        mag = np.sum(W3[None] * detJ * np.abs(R[:, v]))
        assert abs(tot) < 1e-13 * mag, v
