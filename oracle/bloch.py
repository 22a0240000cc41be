"""Temporal (Bloch) eigenanalysis of the 1-D SD diffusion operator, section 3,
and the combined-mode analysis of the appendix.

Test infrastructure only.  The matrices follow the section's derivation:
the continuous solution operator H(theta), the one-sided gradient operators
W^L and W^R (compact) and the continuous-gradient operator Q(theta); with a
unit diffusion coefficient the semi-discrete system is du/dt = B(theta) u
with B = J^{-1} M Q (the sign and the single Jacobian factor follow from
F = -v and dq/dt = -M G; the printed "-M (Q + Q_IP)" drops both, see the
design notes).  The interior-penalty term Q_IP is included for eta > 0.
"""
import numpy as np

from .oracle import operators


def bloch_matrix(p, theta, J=1.0, scheme="compact", eta_ip=0.0, h=2.0):
    """B(theta) for polynomial degree p, Jacobian J (element size 2J)."""
    _, _, _, L, M = operators(p)
    n = p + 1
    cL = np.zeros((n + 1, 1)); cL[0, 0] = 1.0
    cR = np.zeros((n + 1, 1)); cR[n, 0] = 1.0
    em = np.exp(-1j * theta)
    ep = np.exp(+1j * theta)
    # continuous solution at the flux points, u^{F,C} = H u^S
    H = (L + 0.5 * cL @ cR.T @ L * em - 0.5 * cL @ cL.T @ L
         + 0.5 * cR @ cL.T @ L * ep - 0.5 * cR @ cR.T @ L)
    V = (1.0 / J) * M @ H                       # standard v^S = J^-1 M H u^S
    if scheme == "compact":
        WL = (1.0 / J) * M @ (H - 0.5 * cR @ cL.T @ L * ep + 0.5 * cR @ cR.T @ L)
        WR = (1.0 / J) * M @ (H - 0.5 * cL @ cR.T @ L * em + 0.5 * cL @ cL.T @ L)
    else:
        WL = V
        WR = V
    LV = L @ V
    Q = (LV - cL @ cL.T @ LV - cR @ cR.T @ LV
         + 0.5 * cL @ cR.T @ L @ WR * em + 0.5 * cL @ cL.T @ L @ WL
         + 0.5 * cR @ cL.T @ L @ WL * ep + 0.5 * cR @ cR.T @ L @ WR)
    if eta_ip > 0.0:
        tau = eta_ip * (p + 1) ** 2 / h
        Q = Q + tau * (cL @ cL.T - cL @ cR.T * em) @ L + tau * (cR @ cL.T * ep - cR @ cR.T) @ L
    return (1.0 / J) * M @ Q


def bloch_eigs(p, thetas, J=1.0, scheme="compact", eta_ip=0.0, h=2.0):
    """Eigenvalues -i omega~ of B(theta) for each theta, shape [len(thetas), p+1]."""
    return np.array([np.linalg.eigvals(bloch_matrix(p, t, J, scheme, eta_ip, h)) for t in thetas])


def combined_mode(p, theta, t, J=1.0, scheme="compact", eta_ip=0.0, h=2.0):
    """Combined-mode amplification G(theta, t) and omega~ (appendix A): the
    initial Fourier mode sampled at the solution points is expanded on the
    eigenvectors of B and evolved exactly."""
    from .oracle import operators as _ops
    xs = _ops(p)[0]
    B = bloch_matrix(p, theta, J, scheme, eta_ip, h)
    lam, N = np.linalg.eig(B)
    u0 = np.exp(1j * theta * (xs + 1.0) / 2.0)
    gam = np.linalg.solve(N, u0)
    ut = N @ (gam * np.exp(lam * t))
    G = np.vdot(u0, ut) / np.vdot(u0, u0)
    # u(t) = sum_j gamma_j mu_j exp(-i omega_j t) makes G = exp(-i omega t)
    # for a single mode, so omega = (i / t) log G (printed with the other
    # sign; this one reduces to omega = i lambda when u0 is an eigenvector)
    omega = 1j / t * np.log(G)
    return G, omega
