"""Pins of the curvilinear reference (section 2.3 with a general adjoint S):
affine meshes reproduce the affine reference (an independent code), a
rigidly rotated mesh (full S, every transverse term active) gives the same
right-hand side, constants and (away from the periodic seam) linear fields
are preserved where the discrete metric identities hold, the scheme is
conservative, and it converges on a curved periodic mesh."""
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


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_affine_nodes_reproduce_the_affine_reference(oracle_lib, scheme, p):
    nel, lo, hi = (3, 4, 2), (0.0, 0.0, 0.0), (1.0, 2.0, 1.5)
    U = W.random_scalar_3d(nel, p, seed=4)
    prm = oracle_lib.make_params("diffusion", nu=0.8)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)[:, 0]
    R = C.rhs(U[:, 0], nel, W.mesh_nodes(nel, lo, hi, q=1), p, scheme, nu=0.8)
    assert np.abs(R - Ro).max() < 1e-13 * np.abs(Ro).max()
    # the same nodes given as a degree-2 map (midpoints on straight edges)
    R2 = C.rhs(U[:, 0], nel, W.mesh_nodes(nel, lo, hi, q=2), p, scheme, nu=0.8)
    assert np.abs(R2 - Ro).max() < 1e-13 * np.abs(Ro).max()


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 3])
def test_rigid_rotation_leaves_the_rhs_unchanged(oracle_lib, scheme, p):
    """Rotating the mesh makes S a full matrix (all the transverse terms of
    the gradient and of the fluxes are active); the Laplacian of the same
    nodal values is unchanged.  A scheme that kept only diagonal metric terms
    would fail."""
    nel, lo, hi = (3, 2, 4), (0.0, 0.0, 0.0), (1.5, 1.0, 2.0)
    U = W.random_scalar_3d(nel, p, seed=8)[:, 0]
    R = C.rhs(U, nel, W.mesh_nodes(nel, lo, hi, q=1), p, scheme)
    Rr = C.rhs(U, nel, W.mesh_nodes(nel, lo, hi, q=1, rotation=rotation(0.7, 0.4, -1.1)), p, scheme)
    assert np.abs(Rr - R).max() < 1e-13 * np.abs(R).max()
    S, _ = C.metrics(W.mesh_nodes(nel, lo, hi, q=1, rotation=rotation(0.7, 0.4, -1.1)), p)
    off = np.abs(S[0][..., 0, 1:]).max()
    assert off > 0.1 * np.abs(S[0][..., 0, 0]).max()


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("q,p", [(1, 1), (1, 2), (1, 3), (2, 3), (2, 4)])
def test_constants_preserved_on_curved_meshes(scheme, q, p):
    """The rows of S at the flux points of family d have degree 2q in xi_d,
    so the discrete metric identities sum_d D_d S_dm = 0 hold when
    2q <= p + 1, and then R(1) = 0."""
    nel = (4, 3, 4)
    Xg = W.mesh_nodes(nel, *BOX, q=q, displacement=W.periodic_wave_displacement(0.15))
    n = p + 1
    R = C.rhs(np.ones((int(np.prod(nel)), n, n, n)), nel, Xg, p, scheme)
    scale = n ** 2 / (TWO_PI / 4) ** 2
    assert np.abs(R).max() < 1e-12 * scale


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [2, 3])
def test_linear_fields_preserved_away_from_the_seam(scheme, p):
    """On straight-edged non-affine hexahedra (q = 1, nodes moved) a field
    linear in x has a degree-1 map in xi and u S_dm has degree 3 <= p + 1,
    so the gradient is exact and R = 0; a linear field jumps across the
    periodic seam, so only elements whose stencil stays inside count."""
    nel = (6, 6, 6)

    def move(X, Y, Z):
        return 0.1 * np.sin(X) * np.cos(2 * Y), 0.1 * np.sin(Z + Y), 0.1 * np.cos(X) * np.sin(Z)
    Xg = W.mesh_nodes(nel, *BOX, q=1, displacement=move)
    u = W.map_points(Xg, p) @ np.array([0.3, -0.7, 0.5])
    R = C.rhs(u, nel, Xg, p, scheme).reshape(6, 6, 6, -1)
    assert np.abs(R).max() > 1.0                       # the seam does show
    assert np.abs(R[2:4, 2:4, 2:4]).max() < 1e-11


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_conservation_on_a_curved_mesh(scheme):
    nel, p = (4, 4, 3), 3
    Xg = W.mesh_nodes(nel, *BOX, q=2, displacement=W.periodic_wave_displacement(0.15))
    n = p + 1
    u = np.random.Generator(np.random.PCG64(1)).normal(size=(int(np.prod(nel)), n, n, n))
    R = C.rhs(u, nel, Xg, p, scheme)
    _, detJ = C.metrics(Xg, p)
    _, w = W.gl_nodes(n)
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]
    assert abs(np.sum(wq * detJ * R)) < 1e-14 * np.sum(wq * detJ * np.abs(R))
    assert np.abs(R - C.rhs(u, nel, Xg, p, "br1" if scheme == "compact" else "compact")).max() > 1e-3


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_refinement_on_a_curved_mesh(scheme):
    """R(u) -> lap u = -3 u for u = sin x sin y sin z on a curved periodic mesh
    (degree-2 elements, wave displacement 0.15): the pointwise error at the
    solution points falls by more than 2^1.5 from 6^3 to 12^3 elements at
    p = 3 (on the affine mesh, 2^1.54)."""
    errs = []
    for N in (6, 12):
        nel = (N, N, N)
        Xg = W.mesh_nodes(nel, *BOX, q=2, displacement=W.periodic_wave_displacement(0.15))
        x = W.map_points(Xg, 3)
        u = np.sin(x[..., 0]) * np.sin(x[..., 1]) * np.sin(x[..., 2])
        errs.append(np.abs(C.rhs(u, nel, Xg, 3, scheme) + 3.0 * u).max())
    assert errs[1] < 0.05 and errs[0] / errs[1] > 2 ** 1.5


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_interior_penalty_on_affine_nodes_is_the_cartesian_one(oracle_lib, scheme, p):
    """Section 3's penalty written with the metric terms (tau n = eta (p+1)^2
    max(J^-1) S_d / 2 (u_R - u_L)) reduces on affine elements of a box with
    three different element sizes to the Cartesian tau = eta (p+1)^2 / h_d
    of the C reference, for degree-1 and degree-2 node sets."""
    nel, lo, hi = (3, 4, 2), (0.0, 0.0, 0.0), (1.0, 2.0, 1.5)
    U = W.random_scalar_3d(nel, p, seed=6)
    prm = oracle_lib.make_params("diffusion", nu=0.8, eta_ip=0.35)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)[:, 0]
    R0 = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, oracle_lib.make_params("diffusion", nu=0.8))[:, 0]
    assert np.abs(Ro - R0).max() > 1e-2 * np.abs(R0).max()          # the penalty matters here
    for q in (1, 2):
        R = C.rhs(U[:, 0], nel, W.mesh_nodes(nel, lo, hi, q=q), p, scheme, nu=0.8, eta_ip=0.35)
        assert np.abs(R - Ro).max() < 1e-13 * np.abs(Ro).max()


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_interior_penalty_rotation_and_conservation(scheme):
    """With the penalty on: a rigidly rotated mesh gives the same RHS (the
    penalty acts along the physical normal), and on a curved mesh the
    J-weighted integral of the RHS vanishes (both elements of a face see the
    same penalty, the larger J^-1 of the two sides)."""
    p = 3
    nel, lo, hi = (3, 2, 4), (0.0, 0.0, 0.0), (1.5, 1.0, 2.0)
    U = W.random_scalar_3d(nel, p, seed=12)[:, 0]
    R = C.rhs(U, nel, W.mesh_nodes(nel, lo, hi, q=1), p, scheme, eta_ip=0.5)
    Rr = C.rhs(U, nel, W.mesh_nodes(nel, lo, hi, q=1, rotation=rotation(0.3, -0.8, 1.2)), p, scheme, eta_ip=0.5)
    assert np.abs(Rr - R).max() < 1e-13 * np.abs(R).max()
    nelc = (4, 3, 4)
    Xg = W.mesh_nodes(nelc, *BOX, q=2, displacement=W.periodic_wave_displacement(0.15))
    u = np.random.Generator(np.random.PCG64(3)).normal(size=(int(np.prod(nelc)), p + 1, p + 1, p + 1))
    Rc = C.rhs(u, nelc, Xg, p, scheme, eta_ip=0.5)
    _, detJ = C.metrics(Xg, p)
    _, w = W.gl_nodes(p + 1)
    wq = w[:, None, None] * w[None, :, None] * w[None, None, :]
    assert abs(np.sum(wq * detJ * Rc)) < 1e-14 * np.sum(wq * detJ * np.abs(Rc))
    assert np.abs(Rc - C.rhs(u, nelc, Xg, p, scheme)).max() > 1e-2 * np.abs(Rc).max()
    # constants stay at rest: the penalty sees no jump
    assert np.abs(C.rhs(np.ones_like(u), nelc, Xg, p, scheme, eta_ip=0.5)).max() < 1e-10
