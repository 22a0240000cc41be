"""Pins of the 3-D oracle (section 2.3 extended to three directions, and the
Navier-Stokes setting of section 4.4)."""
import math

import numpy as np
import pytest

from paper_2608_09615_amd import workloads as W


def quad_weights(p):
    _, ws = W.gl_nodes(p + 1)
    return ws[:, None, None] * ws[None, :, None] * ws[None, None, :]


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_degenerate_3d_mesh_reproduces_1d(oracle_lib, scheme, p):
    """An (N, 1, 1) mesh with a state constant in y and z gives the 1-D RHS."""
    N, n = 7, p + 1
    rng = np.random.Generator(np.random.PCG64(p))
    u1 = rng.uniform(-1, 1, (N, n))
    u3 = np.broadcast_to(u1[:, None, None, None, :], (N, 1, n, n, n)).copy()
    prm = oracle_lib.make_params("diffusion", nu=0.7)
    R3 = oracle_lib.rhs_3d(u3, (N, 1, 1), (0, 0, 0), (1.5, 0.3, 0.2), p, scheme, prm)
    R1 = oracle_lib.rhs_1d(u1, p, 0.0, 1.5, scheme=scheme, coef=0.7)
    ref = np.abs(R1).max()
    assert np.abs(R3 - R1[:, None, None, None, :]).max() < 1e-12 * ref


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_scalar_diffusion_sine_product(oracle_lib, scheme):
    """sin x sin y sin z is an eigenfunction of the Laplacian with -3; the
    3-D RHS approaches -3 nu u and the error falls with refinement."""
    prm = oracle_lib.make_params("diffusion", nu=1.0)
    lo, hi = (0, 0, 0), (2 * math.pi,) * 3
    errs = []
    for N in (4, 8):
        u = W.sine_3d((N, N, N), lo, hi, 3)
        R = oracle_lib.rhs_3d(u, (N, N, N), lo, hi, 3, scheme, prm)
        errs.append(np.abs(R + 3.0 * u).max())
    assert errs[1] < errs[0] / 2 and errs[1] < 0.05


@pytest.mark.parametrize("scheme,width_scalar,width_ns", [("compact", 7, 19), ("br1", 13, 25)])
def test_stencil_width_3d(oracle_lib, scheme, width_scalar, width_ns):
    """Scalar diffusion: the 3-D stencil is the centre plus its face
    neighbours (compact) or two layers along the axes (BR1).  Navier-Stokes
    couples edge neighbours through the cross derivatives of tau."""
    nel = (7, 7, 7)
    c = 3 + 7 * (3 + 7 * 3)
    prs = oracle_lib.make_params("diffusion", nu=1.0)
    u0 = W.random_scalar_3d(nel, 2, 3)
    R0 = oracle_lib.rhs_3d(u0, nel, (0, 0, 0), (1, 1, 1), 2, scheme, prs)
    u1 = u0.copy()
    u1[c] += 0.1
    R1 = oracle_lib.rhs_3d(u1, nel, (0, 0, 0), (1, 1, 1), 2, scheme, prs)
    assert (np.abs(R1 - R0).reshape(len(u0), -1).max(1) > 0).sum() == width_scalar
    prm = oracle_lib.make_params("ns")
    lo, hi = W.tgv_domain()
    u0 = W.perturbed_tgv_state(nel, 1, seed=2, noise=1e-3)
    R0 = oracle_lib.rhs_3d(u0, nel, lo, hi, 1, scheme, prm)
    u1 = u0.copy()
    u1[c] *= 1.001
    R1 = oracle_lib.rhs_3d(u1, nel, lo, hi, 1, scheme, prm)
    changed = np.abs(R1 - R0).reshape(len(u0), -1).max(1) > 0
    assert changed.sum() == width_ns
    # the changed set is the centre, its 6 face and 12 edge neighbours (+ the
    # 6 second-layer axis neighbours for BR1)
    ex, ey, ez = np.arange(343) % 7, (np.arange(343) // 7) % 7, np.arange(343) // 49
    dx, dy, dz = np.abs(ex - 3), np.abs(ey - 3), np.abs(ez - 3)
    expect = (dx + dy + dz <= 2) & (np.maximum(np.maximum(dx, dy), dz) <= 1)
    if scheme == "br1":
        expect |= ((dx == 2) & (dy == 0) & (dz == 0)) | ((dy == 2) & (dx == 0) & (dz == 0)) | \
                  ((dz == 2) & (dx == 0) & (dy == 0))
    assert np.array_equal(changed, expect)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_ns_freestream_preserved(oracle_lib, scheme):
    prm = oracle_lib.make_params("ns")
    lo, hi = W.tgv_domain()
    nel, p = (3, 3, 3), 3
    n = p + 1
    U = np.zeros((27, 5, n, n, n))
    U[:, 0], U[:, 1], U[:, 2], U[:, 3], U[:, 4] = 1.2, 0.3, -0.2, 0.1, 80.0
    R = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    assert np.abs(R).max() < 1e-11


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 3])
def test_ns_conservation(oracle_lib, scheme, p):
    prm = oracle_lib.make_params("ns", Re=100.0)
    lo, hi = W.tgv_domain()
    nel = (3, 4, 5)
    U = W.perturbed_tgv_state(nel, p, seed=5, noise=1e-2)
    R = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    wq = quad_weights(p)
    tot = np.einsum("evkji,kji->v", R, wq)
    mag = np.einsum("evkji,kji->v", np.abs(R), wq)
    assert np.all(np.abs(tot) < 1e-13 * mag)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_ns_translation_permutes_rhs(oracle_lib, scheme):
    """Shifting the state by whole elements shifts the RHS bit for bit."""
    prm = oracle_lib.make_params("ns")
    lo, hi = W.tgv_domain()
    nel = (4, 3, 3)
    U = W.perturbed_tgv_state(nel, 2, seed=7, noise=1e-2)
    R = oracle_lib.rhs_3d(U, nel, lo, hi, 2, scheme, prm)
    shp = (3, 3, 4) + U.shape[1:]
    Us = np.roll(U.reshape(shp), shift=(1, 2, 1), axis=(0, 1, 2)).reshape(U.shape)
    Rs = oracle_lib.rhs_3d(Us, nel, lo, hi, 2, scheme, prm)
    assert np.array_equal(Rs, np.roll(R.reshape(shp), shift=(1, 2, 1), axis=(0, 1, 2)).reshape(R.shape))


def test_tgv_initial_diagnostics(oracle_lib):
    """E_k/|Omega| -> 1/8 and enstrophy/|Omega| -> 3/4 for the TGV initial
    condition (closed forms of the velocity field of section 4.4)."""
    prm = oracle_lib.make_params("ns")
    lo, hi = W.tgv_domain()
    vol = (2 * math.pi) ** 3
    d = oracle_lib.diag_3d(W.tgv_state((8, 8, 8), 3), (8, 8, 8), lo, hi, 3, prm)
    assert abs(d["ke"] / vol - 0.125) < 1e-9
    assert abs(d["enstrophy"] / vol - 0.75) < 1e-5
    assert abs(d["mass"] / vol - 1.0) < 1e-12
    assert d["nonfinite"] == 0.0 and abs(d["umax"] - 1.0) < 0.05


def test_signal_speed(oracle_lib):
    """max(|u| + c), c = sqrt(gamma P / rho): a uniform state gives the closed
    form; the TGV state gives the maximum taken over the primitive fields
    (the oracle goes through the conservative variables); an inadmissible
    state (negative pressure at one point) gives +inf."""
    lo, hi = W.tgv_domain()
    nel, p = (3, 2, 2), 2
    shape = (12, 3, 3, 3)
    for gamma in (1.4, 5.0 / 3.0):
        prm = oracle_lib.make_params("ns", gamma=gamma)
        one = np.ones(shape)
        U = W.conservative(1.3 * one, 0.2 * one, -0.5 * one, 0.1 * one, 2.0 * one, gamma=gamma)
        d = oracle_lib.diag_3d(U, nel, lo, hi, p, prm)
        assert abs(d["smax"] - (math.sqrt(0.3) + math.sqrt(gamma * 2.0 / 1.3))) < 1e-14
    prm = oracle_lib.make_params("ns")
    nel, p = (4, 4, 4), 3
    X, Y, Z = W.points_3d(nel, lo, hi, p)
    rho, u, v, w, pr = W.tgv_primitive(X, Y, Z)
    expect = np.max(np.sqrt(u * u + v * v + w * w) + np.sqrt(1.4 * pr / rho))
    d = oracle_lib.diag_3d(W.tgv_state(nel, p), nel, lo, hi, p, prm)
    assert abs(d["smax"] - expect) < 1e-13 * expect
    assert 10.0 < d["smax"] < 11.1            # c0 = u0 / Ma = 10, |u| <= 1
    U = W.tgv_state(nel, p)
    U[5, 4, 1, 2, 3] = 0.0                    # rho E = 0 with u != 0 there: P < 0
    assert oracle_lib.diag_3d(U, nel, lo, hi, p, prm)["smax"] == math.inf


def test_tgv_initial_dissipation_rate(oracle_lib):
    """dE_k/dt at t = 0 is -nu * enstrophy up to O(Ma^2) and discretisation
    error (kinetic-energy balance of the viscous term)."""
    prm = oracle_lib.make_params("ns", Re=100.0, sutherland_s=-1.0)
    lo, hi = W.tgv_domain()
    nel, p = (6, 6, 6), 3
    U = W.tgv_state(nel, p)
    R = oracle_lib.rhs_3d(U, nel, lo, hi, p, "compact", prm)
    rho = U[:, 0]
    vel = U[:, 1:4] / rho[:, None]
    dvel = (R[:, 1:4] - vel * R[:, 0][:, None]) / rho[:, None]
    J = (2 * math.pi / 6) ** 3 / 8
    dEk = J * np.einsum("ecnkji,kji->", vel[:, :, None] * dvel[:, :, None], quad_weights(p))
    vol = (2 * math.pi) ** 3
    assert abs(dEk / vol + 0.75 / 100.0) < 0.03 * 0.75 / 100.0


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_element_subset_matches_full(oracle_lib, scheme):
    prm = oracle_lib.make_params("ns")
    lo, hi = W.tgv_domain()
    nel = (3, 3, 3)
    U = W.perturbed_tgv_state(nel, 2, seed=3, noise=1e-2)
    R = oracle_lib.rhs_3d(U, nel, lo, hi, 2, scheme, prm)
    sel = np.array([0, 13, 26, 5])
    Rs = oracle_lib.rhs_3d_elems(U, nel, lo, hi, 2, scheme, prm, sel)
    assert np.array_equal(Rs, R[sel])
