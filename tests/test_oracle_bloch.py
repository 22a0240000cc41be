"""Two independent constructions of the 1-D diffusion operator agree: the
brute-force global matrix of the oracle RHS and the Bloch matrices of the
temporal eigenanalysis (section 3); their spectra coincide."""
import math

import numpy as np
import pytest

from oracle import bloch


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
