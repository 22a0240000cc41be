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
