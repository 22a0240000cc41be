"""Two independent constructions of the 1-D diffusion operator agree: the
brute-force global matrix of the oracle RHS and the Bloch matrices of the
temporal eigenanalysis (section 3); their spectra coincide."""
import math

import numpy as np
import pytest

from oracle import bloch
from paper_2608_09615_amd import workloads as W


def global_matrix(oracle_lib, N, p, scheme):
    n = p + 1
    A = np.zeros((N * n, N * n))
    for c in range(N * n):
        e = np.zeros(N * n)
        e[c] = 1.0
        A[:, c] = oracle_lib.rhs_1d(e.reshape(N, n), p, 0.0, 2 * math.pi, scheme=scheme).ravel()
    return A


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_global_spectrum_is_union_of_bloch_spectra(oracle_lib, scheme, p):
    N = 8
    J = math.pi / N
    lam_g = np.sort_complex(np.linalg.eigvals(global_matrix(oracle_lib, N, p, scheme)))
    thetas = 2 * math.pi * np.arange(N) / N
    lam_b = np.sort_complex(bloch.bloch_eigs(p, thetas, J=J, scheme=scheme).ravel())
    scale = np.abs(lam_g).max()
    assert np.abs(lam_g - lam_b).max() < 1e-10 * scale


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_bloch_low_wavenumber_and_spurious_mode(oracle_lib, p):
    """With unit elements (J = 1/2) one eigenvalue follows the exact
    -theta^2 at small theta.  Besides the constant, BR1 keeps an undamped
    mode (at theta = 0 for odd p, at theta = pi for even p); the compact
    scheme damps both."""
    th = 0.05
    for scheme in ("br1", "compact"):
        lam = bloch.bloch_eigs(p, [th], J=0.5, scheme=scheme)[0]
        k = np.argmin(np.abs(lam + th ** 2))
        assert abs(lam[k] + th ** 2) < 1e-2 * th ** 2
    for scheme, nzero in (("br1", 2), ("compact", 1)):
        lam = bloch.bloch_eigs(p, [0.0, math.pi], J=0.5, scheme=scheme)
        assert np.sum(np.abs(lam) < 1e-9 * np.abs(lam).max()) == nzero
    lb0, lbpi = bloch.bloch_eigs(p, [0.0, math.pi], J=0.5, scheme="br1")
    where = lb0 if p % 2 == 1 else lbpi
    scale = max(np.abs(lb0).max(), np.abs(lbpi).max())
    assert np.sum(np.abs(where) < 1e-9 * scale) == (2 if p % 2 == 1 else 1)


def fourier_mode(p, theta):
    """The Fourier mode exp(i k x) at the solution points of one element,
    k times the element width = theta."""
    xs, _ = W.gl_nodes(p + 1)
    return np.exp(1j * theta * (xs + 1.0) / 2.0)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6])
def test_combined_mode_equals_matrix_exponential(scheme, p):
    """Appendix: expanding u0 on the eigenvectors and evolving each mode is
    exp(B t) u0; checked against scipy's Pade-based expm."""
    import scipy.linalg as sl
    for th in (0.0, 0.3, 1.0, 2.0, math.pi):
        for t in (1e-3, 0.1, 1.0):
            G, _ = bloch.combined_mode(p, th, t, J=0.5, scheme=scheme)
            u0 = fourier_mode(p, th)
            Ge = np.vdot(u0, sl.expm(t * bloch.bloch_matrix(p, th, 0.5, scheme)) @ u0) / np.vdot(u0, u0)
            assert abs(G - Ge) <= 1e-11 * abs(Ge) + 1e-15, (th, t)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_combined_mode_special_cases(scheme, p):
    """The constant (theta = 0) is steady: G = 1.  At small theta on unit
    elements the combined mode decays like the exact exp(-k^2 t): omega ->
    -i theta^2, i.e. a negative dissipation Im(omega).  As t -> 0, omega
    tends to i times the Rayleigh quotient of B at u0.  Centred schemes:
    Re(omega) = 0."""
    G, om = bloch.combined_mode(p, 0.0, 1.0, J=0.5, scheme=scheme)
    assert abs(G - 1.0) < 1e-12 and abs(om) < 1e-11
    th = 0.05
    for t in (0.1, 1.0):
        _, om = bloch.combined_mode(p, th, t, J=0.5, scheme=scheme)
        assert abs(om - (-1j * th ** 2)) < 1e-2 * th ** 2
    for th in (0.7, 2.0, 3.0):
        B = bloch.bloch_matrix(p, th, 0.5, scheme)
        u0 = fourier_mode(p, th)
        rq = np.vdot(u0, B @ u0) / np.vdot(u0, u0)
        _, om = bloch.combined_mode(p, th, 1e-7, J=0.5, scheme=scheme)
        assert abs(om - 1j * rq) < 1e-5 * abs(rq)
        _, om = bloch.combined_mode(p, th, 0.5, J=0.5, scheme=scheme)
        assert om.imag < 0 and abs(om.real) < 1e-10 * abs(om.imag)
