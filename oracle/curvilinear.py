"""Reference SD diffusion right-hand side on curvilinear hexahedra (section 2.3
with a general adjoint S), scalar u_t = nu lap u on a periodic structured mesh.

Test infrastructure only: plain numpy, FP64, vectorised over elements; the
steps follow the multi-dimensional construction of section 2.3 in its order
(interpolation to the flux points, continuous and one-sided solutions, the
fluxes H = S^T u, the auxiliary variable at the solution points, its
one-sided (compact) or standard (BR1) values at the interfaces, the
interface averages, the fluxes G = S . F, the divergence), in three
dimensions.

Geometry: element e maps the reference cube by the tensor Lagrange
interpolant of degree q (q + 1 equispaced nodes per direction, including
the ends) of its node coordinates Xg[e][c][b][a][:], a along xi.  J is the
Jacobian matrix dx/dxi, S = adj(J) = det(J) J^{-1}, so row d of S is
J grad_x xi_d; they are evaluated exactly (analytic derivatives of the
mapping) at the points where the scheme uses them: S at the flux points of
each family, det(J) at the solution points.

State layout u[e][k][j][i] (i along xi, the fastest), e = ex + Nx (ey + Ny ez).
"""
import numpy as np

from .oracle import operators

AXIS = {0: 3, 1: 2, 2: 1}     # array axis of direction d in [e][k][j][i]


def _lagrange(nodes, x):
    """Values and derivatives of the Lagrange basis on `nodes` at points x:
    arrays [len(x), len(nodes)]."""
    x = np.asarray(x, dtype=np.float64)
    m = len(nodes)
    V = np.ones((len(x), m))
    dV = np.zeros((len(x), m))
    for a in range(m):
        for b in range(m):
            if b == a:
                continue
            V[:, a] *= (x - nodes[b]) / (nodes[a] - nodes[b])
        for c in range(m):
            if c == a:
                continue
            term = np.ones(len(x)) / (nodes[a] - nodes[c])
            for b in range(m):
                if b != a and b != c:
                    term *= (x - nodes[b]) / (nodes[a] - nodes[b])
            dV[:, a] += term
    return V, dV


def jacobian(Xg, xi, eta, zeta):
    """dx/dxi at the tensor points (zeta_k, eta_j, xi_i) of every element:
    [E, len(zeta), len(eta), len(xi), 3 (x comp), 3 (xi dir)]."""
    q = Xg.shape[1] - 1
    nodes = np.linspace(-1.0, 1.0, q + 1)
    Vx, dVx = _lagrange(nodes, xi)
    Vy, dVy = _lagrange(nodes, eta)
    Vz, dVz = _lagrange(nodes, zeta)
    dxi = np.einsum("ecbav,ia,jb,kc->ekjiv", Xg, dVx, Vy, Vz)
    deta = np.einsum("ecbav,ia,jb,kc->ekjiv", Xg, Vx, dVy, Vz)
    dzeta = np.einsum("ecbav,ia,jb,kc->ekjiv", Xg, Vx, Vy, dVz)
    return np.stack([dxi, deta, dzeta], axis=-1)


def adjugate(Jm):
    """adj(J) = det(J) J^{-1}, row d = (dx/dxi_{d+1}) x (dx/dxi_{d+2})."""
    c = [Jm[..., :, d] for d in range(3)]
    rows = [np.cross(c[(d + 1) % 3], c[(d + 2) % 3]) for d in range(3)]
    return np.stack(rows, axis=-2)


def metrics(Xg, p):
    """S at the flux points of each family d ([E, ..., 3 (d'), 3 (m)], the
    family's flux axis in place of its solution axis) and det J at the
    solution points [E, n, n, n]."""
    xs, _, xf, _, _ = operators(p)
    S = []
    for d in range(3):
        pts = [xs, xs, xs]
        pts[d] = xf
        S.append(adjugate(jacobian(Xg, pts[0], pts[1], pts[2])))
    detJ = np.linalg.det(jacobian(Xg, xs, xs, xs))
    return S, detJ


def _along(A, d, Mat):
    """Apply the matrix Mat [rows, cols] along direction d of A [E, k, j, i]."""
    ax = AXIS[d]
    return np.moveaxis(np.tensordot(A, Mat, axes=([ax], [1])), -1, ax)


def _end(A, d, s):
    """Slice of A at index 0 (s = 0) or -1 (s = 1) along direction d."""
    ax = AXIS[d]
    return np.take(A, 0 if s == 0 else A.shape[ax] - 1, axis=ax)


def _set_end(A, d, s, val):
    ax = AXIS[d]
    idx = [slice(None)] * A.ndim
    idx[ax] = 0 if s == 0 else A.shape[ax] - 1
    A[tuple(idx)] = val


def _neighbour(nel, d, s):
    """Index array: the neighbour of every element across face (d, s)."""
    Nx, Ny, Nz = nel
    e = np.arange(Nx * Ny * Nz)
    c = [e % Nx, (e // Nx) % Ny, e // (Nx * Ny)]
    c[d] = (c[d] + (1 if s == 1 else -1)) % nel[d]
    return c[0] + Nx * (c[1] + Ny * c[2])


def face_det(Xg, p):
    """det J at the flux points of each family d ([E, ...], the family's
    flux axis in place of its solution axis): at its two ends, the points of
    the faces normal to d."""
    xs, _, xf, _, _ = operators(p)
    out = []
    for d in range(3):
        pts = [xs, xs, xs]
        pts[d] = xf
        out.append(np.linalg.det(jacobian(Xg, pts[0], pts[1], pts[2])))
    return out


def rhs(u, nel, Xg, p, scheme="compact", nu=1.0, eta_ip=0.0):
    """du/dt for u[e][k][j][i] on the mesh of node coordinates Xg.

    eta_ip > 0 adds the interior penalty of section 3 to the common gradient
    at every interface: its component along the unit normal n = S_d / |S_d|
    gains tau (u_R - u_L), u_R the trace of the element on the +xi_d side,
    with tau = eta_ip (p+1)^2 / h and 1/h = |S_d| max(J^-1_L, J^-1_R) / 2 at
    the face point (on an affine Cartesian element |S_d| J^-1 = 2 / h_d,
    the element size normal to the face; the larger J^-1 takes the smaller
    of the two sizes)."""
    u = np.asarray(u, dtype=np.float64)
    _, _, _, L, M = operators(p)
    S, detJ = metrics(Xg, p)
    Jinv = 1.0 / detJ
    detJF = face_det(Xg, p) if eta_ip else None
    nbr = {(d, s): _neighbour(nel, d, s) for d in range(3) for s in (0, 1)}
    # 1. discontinuous solution at the flux points of each family
    uF = [_along(u, d, L) for d in range(3)]
    # 2. common interface values, continuous and one-sided solutions
    T = {(d, s): _end(uF[d], d, s) for d in range(3) for s in (0, 1)}
    uhat = {}
    for d in range(3):
        for s in (0, 1):
            other = T[(d, 1 - s)][nbr[(d, s)]]
            uhat[(d, s)] = 0.5 * (other + T[(d, s)]) if s == 0 else 0.5 * (T[(d, s)] + other)
    uC, uSide = [], []
    for d in range(3):
        C = uF[d].copy()
        _set_end(C, d, 0, uhat[(d, 0)])
        _set_end(C, d, 1, uhat[(d, 1)])
        uC.append(C)
        sides = []
        for s in (0, 1):
            X = C.copy()
            # the one-sided solution of face s keeps the own trace at the other face
            _set_end(X, d, 1 - s, T[(d, 1 - s)])
            sides.append(X)
        uSide.append(sides)
    # 3. fluxes H_m = u S_dm and the auxiliary variable at the solution points
    def grad_at_solution_points(uFam):
        return np.stack([Jinv * sum(_along(uFam[dd] * S[dd][..., dd, m], dd, M) for dd in range(3))
                         for m in range(3)], axis=1)      # [E, 3 (m), k, j, i]
    vS = grad_at_solution_points(uC)
    # 4. auxiliary variable at the interfaces: one-sided (compact) or standard
    vface = {}
    for d in range(3):
        for s in (0, 1):
            if scheme == "compact":
                fam = list(uC)
                fam[d] = uSide[d][s]
                vSs = grad_at_solution_points(fam)
            else:
                vSs = vS
            vF = np.stack([_along(vSs[:, m], d, L) for m in range(3)], axis=1)
            vface[(d, s)] = np.stack([_end(vF[:, m], d, s) for m in range(3)], axis=1)
    # 5. interface averages and the continuous auxiliary variable per family
    R = np.zeros_like(u)
    for d in range(3):
        vF = np.stack([_along(vS[:, m], d, L) for m in range(3)], axis=1)
        for s in (0, 1):
            other = vface[(d, 1 - s)][nbr[(d, s)]]
            vh = 0.5 * (other + vface[(d, s)]) if s == 0 else 0.5 * (vface[(d, s)] + other)
            if eta_ip:
                # interior penalty: tau (u_R - u_L) n = eta (p+1)^2 max(J^-1) / 2 (u_R - u_L) S_d
                t_oth = T[(d, 1 - s)][nbr[(d, s)]]
                jump = T[(d, s)] - t_oth if s == 0 else t_oth - T[(d, s)]
                jmax = np.maximum(1.0 / _end(detJF[d], d, s), 1.0 / _end(detJF[d], d, 1 - s)[nbr[(d, s)]])
                coef = eta_ip * (p + 1) ** 2 / 2.0 * jmax * jump
                vh = vh + np.stack([coef * _end(S[d][..., d, m], d, s) for m in range(3)], axis=1)
            for m in range(3):
                sub = vF[:, m]
                _set_end(sub, d, s, vh[:, m])
        # 6. diffusive flux F = -nu v, G_d = S_d . F, and its divergence
        G = -nu * sum(S[d][..., d, m] * vF[:, m] for m in range(3))
        R -= Jinv * _along(G, d, M)
    return R


# ---------------------------------------------------------------------------
# Navier-Stokes on curvilinear hexahedra (section 2.3, eqs. ns:mapped and
# adj:f, with the fluxes of section 4.4).  State U[e][v][k][j][i], v = rho,
# rho u, rho v, rho w, rho E.  The steps are those of `rhs` applied to the
# five conservative variables: traces, common solution, the auxiliary
# variable (the gradient of every conservative variable, all metric terms),
# its one-sided (compact) or standard (BR1) interface values and their
# average, then G_d = S_d . (F_c - F_v) at the flux points of family d and
# the divergence.  At the interfaces the convective part is the Roe flux
# (with Harten's fix on the acoustic waves, reading R7) along the unit normal
# n = S_d / |S_d|, scaled by |S_d|, and the viscous part is F_v of the common
# solution and common gradient (option (a) of section 2.1).  The pointwise
# laws below take a direction vector instead of an axis; for an axis they are
# the C oracle's (pinned in the tests).
# ---------------------------------------------------------------------------

def _p0(prm):
    return prm.rho0 / prm.gamma * (prm.u0 / prm.Ma) ** 2


def _mu(prm, T):
    mu0 = prm.rho0 * prm.u0 * prm.Lref / prm.Re
    if prm.sutherland_s < 0.0:
        return mu0 * np.ones_like(T)
    th = T / (_p0(prm) / prm.rho0)
    return mu0 * th * np.sqrt(th) * (1.0 + prm.sutherland_s) / (th + prm.sutherland_s)


def ns_conv_dir(prm, U, s):
    """F_c . s for states U [..., 5] and direction vectors s [..., 3]:
    (rho u_s, rho u u_s + P s, (rho E + P) u_s), u_s = u . s."""
    g = prm.gamma
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    P = (g - 1.0) * (U[..., 4] - 0.5 * rho * np.sum(u * u, axis=-1))
    us = np.sum(u * s, axis=-1)
    F = np.empty(U.shape)
    F[..., 0] = rho * us
    F[..., 1:4] = U[..., 1:4] * us[..., None] + P[..., None] * s
    F[..., 4] = (U[..., 4] + P) * us
    return F


def ns_visc_dir(prm, U, G, s):
    """F_v . s for states U [..., 5], gradients of the conservative variables
    G [..., 5 (v), 3 (m)] and direction vectors s [..., 3]:
    (0, tau s, u . tau s + kappa grad T . s), tau = mu (grad u + grad u^T)
    + lambda (div u) I, T = P / rho (R = 1), kappa = mu C_p / Pr."""
    g = prm.gamma
    rho = U[..., 0]
    u = U[..., 1:4] / rho[..., None]
    E = U[..., 4] / rho
    T = (g - 1.0) * (E - 0.5 * np.sum(u * u, axis=-1))
    drho = G[..., 0, :]                                      # [..., m]
    du = (G[..., 1:4, :] - u[..., :, None] * drho[..., None, :]) / rho[..., None, None]   # [..., i, m]
    dE = (G[..., 4, :] - E[..., None] * drho) / rho[..., None]
    dT = (g - 1.0) * (dE - np.einsum("...j,...jm->...m", u, du))
    mu = _mu(prm, T)
    lam = prm.lambda_over_mu * mu
    kappa = mu * (g / (g - 1.0)) / prm.Pr
    div = du[..., 0, 0] + du[..., 1, 1] + du[..., 2, 2]
    tau = mu[..., None, None] * (du + np.swapaxes(du, -1, -2)) + (lam * div)[..., None, None] * np.eye(3)
    ts = np.einsum("...ij,...j->...i", tau, s)
    F = np.zeros(U.shape)
    F[..., 1:4] = ts
    F[..., 4] = np.sum(u * ts, axis=-1) + kappa * np.sum(dT * s, axis=-1)
    return F


def ns_roe_normal(prm, UL, UR, n):
    """Roe flux along unit normals n [..., 3]: (F(UL) + F(UR)) . n / 2 -
    sum_k |l_k| a_k r_k / 2 over the acoustic waves u_n -+ c, the entropy wave
    and the shear waves at the square-root-density average, Harten's fix
    |l| -> (l^2 + delta^2) / (2 delta) for |l| < delta on the acoustic pair,
    delta = entropy_fix (|u_n| + c)."""
    g = prm.gamma

    def prim(U):
        rho = U[..., 0]
        u = U[..., 1:4] / rho[..., None]
        P = (g - 1.0) * (U[..., 4] - 0.5 * rho * np.sum(u * u, axis=-1))
        return rho, u, P, (U[..., 4] + P) / rho

    rL, uL, pL, HL = prim(UL)
    rR, uR, pR, HR = prim(UR)
    sL, sR = np.sqrt(rL), np.sqrt(rR)
    w = 1.0 / (sL + sR)
    ut = (sL[..., None] * uL + sR[..., None] * uR) * w[..., None]
    Ht = (sL * HL + sR * HR) * w
    rt = sL * sR
    q2 = np.sum(ut * ut, axis=-1)
    c2 = (g - 1.0) * (Ht - 0.5 * q2)
    c = np.sqrt(c2)
    un = np.sum(ut * n, axis=-1)
    du = uR - uL
    dun = np.sum(du * n, axis=-1)
    dut = du - dun[..., None] * n
    drho, dp = rR - rL, pR - pL
    a1 = (dp - rt * c * dun) / (2.0 * c2)
    a5 = (dp + rt * c * dun) / (2.0 * c2)
    a2 = drho - dp / c2
    l1, l2, l5 = np.abs(un - c), np.abs(un), np.abs(un + c)
    delta = prm.entropy_fix * (np.abs(un) + c)
    with np.errstate(divide="ignore", invalid="ignore"):
        fix = lambda l: np.where((delta > 0.0) & (l < delta), (l * l + delta * delta) / (2.0 * delta), l)
        l1, l5 = fix(l1), fix(l5)
    D = np.empty(UL.shape)
    D[..., 0] = l1 * a1 + l2 * a2 + l5 * a5
    D[..., 1:4] = ((l1 * a1)[..., None] * (ut - c[..., None] * n) + (l2 * a2)[..., None] * ut
                   + (l5 * a5)[..., None] * (ut + c[..., None] * n) + (l2 * rt)[..., None] * dut)
    D[..., 4] = (l1 * a1 * (Ht - c * un) + l2 * a2 * 0.5 * q2 + l5 * a5 * (Ht + c * un)
                 + l2 * rt * np.sum(ut * dut, axis=-1))
    return 0.5 * (ns_conv_dir(prm, UL, n) + ns_conv_dir(prm, UR, n)) - 0.5 * D


def _vars_last(A):
    """[E, 5, ...] -> [E, ..., 5]."""
    return np.moveaxis(A, 1, -1)


def rhs_ns(U, nel, Xg, p, scheme, prm):
    """dU/dt for U[e][v][k][j][i] (FP64) on the mesh of node coordinates Xg:
    the compressible Navier-Stokes equations of section 4.4 on curvilinear
    elements (section 2.3; prm = oracle.make_params("ns", ...))."""
    U = np.asarray(U, dtype=np.float64)
    _, _, _, L, M = operators(p)
    S, detJ = metrics(Xg, p)
    Jinv = 1.0 / detJ
    nbr = {(d, s): _neighbour(nel, d, s) for d in range(3) for s in (0, 1)}
    nv = 5
    comp = [U[:, v] for v in range(nv)]
    # 1.-2. per variable: traces, common solution, continuous and one-sided
    # solutions (as for the scalar equation)
    uF, T, uhat, uC, uSide = [], [], [], [], []
    for v in range(nv):
        f = [_along(comp[v], d, L) for d in range(3)]
        t = {(d, s): _end(f[d], d, s) for d in range(3) for s in (0, 1)}
        h = {}
        for d in range(3):
            for s in (0, 1):
                other = t[(d, 1 - s)][nbr[(d, s)]]
                h[(d, s)] = 0.5 * (other + t[(d, s)]) if s == 0 else 0.5 * (t[(d, s)] + other)
        C, sides = [], []
        for d in range(3):
            Cd = f[d].copy()
            _set_end(Cd, d, 0, h[(d, 0)])
            _set_end(Cd, d, 1, h[(d, 1)])
            C.append(Cd)
            sd_ = []
            for s in (0, 1):
                X = Cd.copy()
                _set_end(X, d, 1 - s, t[(d, 1 - s)])
                sd_.append(X)
            sides.append(sd_)
        uF.append(f)
        T.append(t)
        uhat.append(h)
        uC.append(C)
        uSide.append(sides)

    def grad(fam):
        # auxiliary variable of one conservative variable: [E, 3 (m), k, j, i]
        return np.stack([Jinv * sum(_along(fam[dd] * S[dd][..., dd, m], dd, M) for dd in range(3))
                         for m in range(3)], axis=1)

    # 3. gradients at the solution points [E, 5, 3, k, j, i]
    vS = np.stack([grad(uC[v]) for v in range(nv)], axis=1)
    # 4. interface values of the gradient: one-sided (compact) or standard
    vface = {}
    for d in range(3):
        for s in (0, 1):
            per_v = []
            for v in range(nv):
                if scheme == "compact":
                    fam = list(uC[v])
                    fam[d] = uSide[v][d][s]
                    g_ = grad(fam)
                else:
                    g_ = vS[:, v]
                per_v.append(np.stack([_end(_along(g_[:, m], d, L), d, s) for m in range(3)], axis=1))
            vface[(d, s)] = np.stack(per_v, axis=1)          # [E, 5, 3, a, b]
    R = np.zeros_like(U)
    for d in range(3):
        Sd = S[d][..., d, :]                                 # [E, family d points..., 3]
        # interior flux points: U and the gradient interpolated along d
        UFd = np.stack([uF[v][d] for v in range(nv)], axis=1)                       # [E, 5, ...]
        VFd = np.stack([np.stack([_along(vS[:, v, m], d, L) for m in range(3)], axis=1)
                        for v in range(nv)], axis=1)                               # [E, 5, 3, ...]
        Uv = _vars_last(UFd)                                                       # [E, ..., 5]
        Gv = np.moveaxis(np.moveaxis(VFd, 1, -1), 1, -1)                           # [E, ..., 5, 3]
        Gd = ns_conv_dir(prm, Uv, Sd) - ns_visc_dir(prm, Uv, Gv, Sd)               # [E, ..., 5]
        # interfaces: Roe along the unit normal and the viscous flux of the
        # common solution and common gradient
        for s in (0, 1):
            nb = nbr[(d, s)]
            town = np.stack([T[v][(d, s)] for v in range(nv)], axis=-1)            # [E, a, b, 5]
            toth = np.stack([T[v][(d, 1 - s)][nb] for v in range(nv)], axis=-1)
            UL, UR = (toth, town) if s == 0 else (town, toth)
            Uh = np.stack([uhat[v][(d, s)] for v in range(nv)], axis=-1)
            own = vface[(d, s)]
            oth = vface[(d, 1 - s)][nb]
            vh = 0.5 * (oth + own) if s == 0 else 0.5 * (own + oth)                 # [E, 5, 3, a, b]
            vh = np.moveaxis(np.moveaxis(vh, 1, -1), 1, -1)                        # [E, a, b, 5, 3]
            Sf = _end(Sd[..., 0], d, s)
            Sf = np.stack([_end(Sd[..., m], d, s) for m in range(3)], axis=-1)     # [E, a, b, 3]
            nrm = np.sqrt(np.sum(Sf * Sf, axis=-1))
            Gf = nrm[..., None] * ns_roe_normal(prm, UL, UR, Sf / nrm[..., None]) - ns_visc_dir(prm, Uh, vh, Sf)
            for v in range(nv):
                sub = Gd[..., v]
                _set_end(sub, d, s, Gf[..., v])
        for v in range(nv):
            R[:, v] -= Jinv * _along(Gd[..., v], d, M)
    return R
