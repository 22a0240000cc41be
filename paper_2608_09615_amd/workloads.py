"""Seeded synthetic inputs shaped like the paper's workloads.

This module generates states only; it holds none of the SD method's
arithmetic, so that both the oracle side and the HIP side can be fed from it.
Point coordinates come from numpy's Gauss-Legendre rule.

Layouts: 1-D states are ``[N, n]``; 3-D states are ``[ne, nv, n, n, n]``
indexed ``[e, v, k, j, i]`` with ``e = ex + Nx*(ey + Ny*ez)`` and ``i``
along x; ``n = p + 1``.
"""
import math

import numpy as np


def gl_nodes(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return x, w


def points_1d(N, p, x0, x1):
    """Physical solution-point coordinates, shape [N, p+1]."""
    xs, _ = gl_nodes(p + 1)
    h = (x1 - x0) / N
    left = x0 + h * np.arange(N)
    return left[:, None] + 0.5 * h * (xs[None, :] + 1.0)


def sine_1d(N, p, x0, x1, k=1.0, phase=0.0):
    return np.sin(k * points_1d(N, p, x0, x1) + phase)


def dirac_1d(N, p, x0, x1, seed=0):
    """Discrete delta of unit integral: 1/h on every point of one element
    chosen by the seeded generator (PCG64)."""
    e = int(np.random.Generator(np.random.PCG64(seed)).integers(N))
    u = np.zeros((N, p + 1))
    u[e, :] = N / (x1 - x0)
    return u, e


def barenblatt(x, t, m, C=0.1):
    """Zeldovich-Kompaneets-Barenblatt profile in one dimension (d = 1)."""
    alpha = 1.0 / ((m - 1.0) + 2.0)
    beta = alpha
    arg = C - alpha * (m - 1.0) / (2.0 * m) * x * x * t ** (-2.0 * beta)
    return t ** (-alpha) * np.maximum(arg, 0.0) ** (1.0 / (m - 1.0))


def barenblatt_t0(m, dx, C=0.1):
    """Start time at which the support half-width equals dx/2."""
    a1 = 1.0 / ((m - 1.0) + 2.0)
    return (C * 2.0 * m / (a1 * (m - 1.0)) * (2.0 / dx) ** 2) ** (-1.0 / (2.0 * a1))


def barenblatt_H(m, t, C=0.1):
    a1 = 1.0 / ((m - 1.0) + 2.0)
    return 2.0 * m * C / (a1 * (m - 1.0)) * t ** (2.0 * a1)


def points_3d(nel, lo, hi, p):
    """Coordinates X, Y, Z of shape [ne, n, n, n] (axes k, j, i)."""
    n = p + 1
    xs, _ = gl_nodes(n)
    out = []
    for d in range(3):
        h = (hi[d] - lo[d]) / nel[d]
        out.append(lo[d] + h * np.arange(nel[d])[:, None] + 0.5 * h * (xs[None, :] + 1.0))
    X1, Y1, Z1 = out
    ne = nel[0] * nel[1] * nel[2]
    ex = np.arange(ne) % nel[0]
    ey = (np.arange(ne) // nel[0]) % nel[1]
    ez = np.arange(ne) // (nel[0] * nel[1])
    X = np.broadcast_to(X1[ex][:, None, None, :], (ne, n, n, n))
    Y = np.broadcast_to(Y1[ey][:, None, :, None], (ne, n, n, n))
    Z = np.broadcast_to(Z1[ez][:, :, None, None], (ne, n, n, n))
    return X, Y, Z


def tgv_primitive(X, Y, Z, Ma=0.1, gamma=1.4, rho0=1.0, u0=1.0, L=1.0, phase=(0.0, 0.0, 0.0)):
    """Taylor-Green vortex on [0, 2 pi L]^3 with x* = (x - x_c)/L."""
    xc = math.pi * L
    xs = (X - xc) / L + phase[0]
    ys = (Y - xc) / L + phase[1]
    zs = (Z - xc) / L + phase[2]
    p0 = rho0 / gamma * (u0 / Ma) ** 2
    rho = np.full(X.shape, rho0)
    u = u0 * np.sin(xs) * np.cos(ys) * np.cos(zs)
    v = -u0 * np.cos(xs) * np.sin(ys) * np.cos(zs)
    w = np.zeros(X.shape)
    pr = p0 + rho0 * u0 ** 2 / 16.0 * np.cos(2 * xs) * np.cos(2 * ys) * (np.cos(2 * zs) + 2.0)
    return rho, u, v, w, pr


def conservative(rho, u, v, w, pr, gamma=1.4):
    rhoE = pr / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)
    return np.stack([rho, rho * u, rho * v, rho * w, rhoE], axis=1)


def tgv_state(nel, p, Ma=0.1, gamma=1.4, rho0=1.0, u0=1.0, L=1.0, phase=(0.0, 0.0, 0.0)):
    """Conservative TGV state [ne, 5, n, n, n] on the periodic box [0, 2 pi L]^3."""
    lo = (0.0, 0.0, 0.0)
    hi = (2 * math.pi * L,) * 3
    X, Y, Z = points_3d(nel, lo, hi, p)
    prim = tgv_primitive(X, Y, Z, Ma, gamma, rho0, u0, L, phase)
    return conservative(*prim, gamma=gamma)


def tgv_domain(L=1.0):
    return (0.0, 0.0, 0.0), (2 * math.pi * L,) * 3


def _global_axis(nel_d, lo_d, hi_d, p):
    xs, _ = gl_nodes(p + 1)
    h = (hi_d - lo_d) / nel_d
    return (lo_d + h * np.arange(nel_d)[:, None] + 0.5 * h * (xs[None, :] + 1.0)).ravel()


def _to_elements(field, nel, p):
    """[gz, gy, gx] point field on the global tensor grid -> [ne, n, n, n]."""
    n = p + 1
    f = field.reshape(nel[2], n, nel[1], n, nel[0], n).transpose(0, 2, 4, 1, 3, 5)
    return np.ascontiguousarray(f.reshape(nel[0] * nel[1] * nel[2], n, n, n))


def solenoidal_perturbation(nel, p, rng, kmax=4, lo=(0.0, 0.0, 0.0), hi=None):
    """Random-phase divergence-free velocity field sum_k a_k cos(k.x + phi_k)/|k|^2
    over integer wavevectors with |k|_inf <= kmax (a_k . k = 0), normalised to
    unit maximum; returns three [ne, n, n, n] arrays."""
    if hi is None:
        hi = (2 * math.pi,) * 3
    ks = np.arange(-kmax, kmax + 1)
    KX, KY, KZ = np.meshgrid(ks, ks, ks, indexing="ij")
    K = np.stack([KX.ravel(), KY.ravel(), KZ.ravel()], axis=1).astype(float)
    K = K[np.any(K != 0, axis=1)]
    a = rng.normal(size=(len(K), 3))
    k2 = np.sum(K * K, axis=1)
    a -= K * (np.sum(a * K, axis=1) / k2)[:, None]
    ph = rng.uniform(0.0, 2 * math.pi, len(K))
    nk = len(ks)
    coef = np.zeros((3, nk, nk, nk), dtype=complex)
    idx = (K + kmax).astype(int)
    for c in range(3):
        coef[c, idx[:, 0], idx[:, 1], idx[:, 2]] = a[:, c] * np.exp(1j * ph) / k2
    gx, gy, gz = (_global_axis(nel[d], lo[d], hi[d], p) for d in range(3))
    ex = np.exp(1j * np.outer(ks, gx))
    ey = np.exp(1j * np.outer(ks, gy))
    ez = np.exp(1j * np.outer(ks, gz))
    out = []
    for c in range(3):
        A = np.einsum("abc,cz->abz", coef[c], ez)
        B = np.einsum("abz,by->azy", A, ey)
        F = np.einsum("azy,ax->zyx", B, ex).real
        out.append(F)
    m = max(np.abs(F).max() for F in out)
    return [_to_elements(F / m, nel, p) for F in out]


def perturbed_tgv_state(nel, p, seed, amp=1e-2, Ma=0.1, gamma=1.4, noise=0.0, kmax=4):
    """TGV with a seeded random phase shift and a random-phase solenoidal
    velocity perturbation of wavenumbers |k|_inf <= kmax and amplitude amp;
    ``noise`` adds pointwise seeded noise (uniform in [-noise, noise] on every
    conservative variable) that breaks every symmetry of the flow."""
    rng = np.random.Generator(np.random.PCG64(seed))
    phase = tuple(rng.uniform(0.0, 2 * math.pi, 3))
    lo, hi = tgv_domain()
    X, Y, Z = points_3d(nel, lo, hi, p)
    rho, u, v, w, pr = tgv_primitive(X, Y, Z, Ma, gamma, phase=phase)
    if amp > 0:
        du = solenoidal_perturbation(nel, p, rng, kmax, lo, hi)
        u, v, w = u + amp * du[0], v + amp * du[1], w + amp * du[2]
    U = conservative(rho, u, v, w, pr, gamma)
    if noise > 0:
        U = U + noise * rng.uniform(-1, 1, U.shape)
    return U


def transonic_jet_state(nel, p, peak_mach=1.3, width=0.8, Ma=0.1, gamma=1.4, seed=0):
    """TGV state with a jet along each axis added to the velocity: a Gaussian
    profile of peak ``peak_mach`` times the sound speed of the mean state, of
    half-width ``width`` around a seeded line through the box.  Along the
    profile the normal velocity passes the sound speed, so faces with a
    near-sonic Roe average (u_n -+ c close to zero) occur in every direction."""
    rng = np.random.Generator(np.random.PCG64(seed))
    lo, hi = tgv_domain()
    X, Y, Z = points_3d(nel, lo, hi, p)
    rho, u, v, w, pr = tgv_primitive(X, Y, Z, Ma, gamma)
    c0 = math.sqrt(gamma * pr.mean() / rho.mean())
    C = rng.uniform(2.0, 4.3, (3, 2))
    vel = [u, v, w]
    axes = [(Y, Z), (X, Z), (X, Y)]
    for d in range(3):
        A, B = axes[d]
        r2 = (A - C[d, 0]) ** 2 + (B - C[d, 1]) ** 2
        vel[d] = vel[d] + (1.0 if d != 1 else -1.0) * peak_mach * c0 * np.exp(-r2 / width ** 2)
    return conservative(rho, *vel, pr, gamma)


def sine_3d(nel, lo, hi, p, k=(1, 1, 1)):
    X, Y, Z = points_3d(nel, lo, hi, p)
    return (np.sin(k[0] * X) * np.sin(k[1] * Y) * np.sin(k[2] * Z))[:, None]


def random_scalar_3d(nel, p, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    ne = nel[0] * nel[1] * nel[2]
    return rng.uniform(-1, 1, (ne, 1, p + 1, p + 1, p + 1))


# ---------------------------------------------------------------------------
# Hexahedral meshes given by node coordinates (curvilinear elements).

def mesh_nodes(nel, lo, hi, q=1, displacement=None, rotation=None):
    """Node coordinates Xg[e][c][b][a][3] of a structured nel[0] x nel[1] x
    nel[2] mesh of the box [lo, hi]: q + 1 equispaced nodes per direction
    and element (ends included, a along x fastest), moved by
    displacement(X, Y, Z) -> (dx, dy, dz) and then by the rotation matrix."""
    t = np.linspace(0.0, 1.0, q + 1)
    axes = []
    for d in range(3):
        h = (hi[d] - lo[d]) / nel[d]
        axes.append(lo[d] + h * (np.arange(nel[d])[:, None] + t[None, :]))   # [N_d, q+1]
    X = axes[0][None, None, :, None, None, :]
    Y = axes[1][None, :, None, None, :, None]
    Z = axes[2][:, None, None, :, None, None]
    shape = (nel[2], nel[1], nel[0], q + 1, q + 1, q + 1)
    X, Y, Z = np.broadcast_to(X, shape), np.broadcast_to(Y, shape), np.broadcast_to(Z, shape)
    P = np.stack([X, Y, Z], axis=-1).astype(np.float64)
    if displacement is not None:
        P = P + np.stack(displacement(X, Y, Z), axis=-1)
    if rotation is not None:
        P = P @ np.asarray(rotation, dtype=np.float64).T
    # [ez, ey, ex, c, b, a, 3] -> [e, c, b, a, 3]
    return np.ascontiguousarray(P.reshape(-1, q + 1, q + 1, q + 1, 3))


def periodic_wave_displacement(eps, L=2 * math.pi):
    """A smooth displacement of period L in every coordinate."""
    k = 2 * math.pi / L

    def disp(X, Y, Z):
        return (eps * np.sin(k * Y) * np.sin(k * Z), eps * np.sin(k * Z) * np.sin(k * X),
                eps * np.sin(k * X) * np.sin(k * Y))
    return disp


def map_points(Xg, p):
    """Physical coordinates [e][k][j][i][3] of the solution points of the
    mesh Xg (tensor Lagrange interpolation of the equispaced nodes)."""
    q = Xg.shape[1] - 1
    nodes = np.linspace(-1.0, 1.0, q + 1)
    xs, _ = gl_nodes(p + 1)
    V = np.ones((len(xs), q + 1))
    for a in range(q + 1):
        for b in range(q + 1):
            if b != a:
                V[:, a] *= (xs - nodes[b]) / (nodes[a] - nodes[b])
    return np.einsum("ecbav,ia,jb,kc->ekjiv", Xg, V, V, V)
