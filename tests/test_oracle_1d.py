"""Pins of the 1-D oracle (sections 2.1, 2.2, 3, 4.1-4.3)."""
import json
import math
import os

import numpy as np
import pytest

from paper_2608_09615_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def l2_error(u, ex, p, h):
    _, ws = W.gl_nodes(p + 1)
    return math.sqrt(np.sum((u - ex) ** 2 * ws[None, :]) * h / 2)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_sine_decay_small_config(oracle_lib, scheme):
    """16 elements, p=3, sin x on [0, 2 pi], nu = 1, RK4 with
    dt = 0.05 h^2 / (p+1)^2 to t = 1 against exp(-t) sin x."""
    N, p, x0, x1 = 16, 3, 0.0, 2 * math.pi
    h = (x1 - x0) / N
    nsteps = math.ceil(1.0 / (0.05 * h * h / (p + 1) ** 2))
    u = oracle_lib.rk4_1d(W.sine_1d(N, p, x0, x1), p, x0, x1, 1.0 / nsteps, nsteps, scheme=scheme)
    ex = math.exp(-1.0) * W.sine_1d(N, p, x0, x1)
    assert np.abs(u - ex).max() < 2e-5


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_rhs_of_sine_approaches_minus_k2(oracle_lib, scheme, p):
    """du/dt of sin(kx) tends to -k^2 sin(kx) as the mesh is refined."""
    x0, x1 = 0.0, 2 * math.pi
    errs = []
    for N in (16, 32):
        for k in (1, 4):
            u = W.sine_1d(N, p, x0, x1, k=k)
            R = oracle_lib.rhs_1d(u, p, x0, x1, scheme=scheme)
            errs.append(np.abs(R + k * k * u).max() / (k * k))
    assert errs[2] < errs[0] and errs[3] < errs[1]
    if p >= 3:
        assert max(errs[2:]) < 0.05


def test_convergence_rates_match_table2(oracle_lib):
    """Section 4.1: Gaussian with D t_i = 1/2400 on [0, 1], T = 2e-5, the
    resolutions of Table 1; the rate between the two finest levels
    reproduces Table 2 for both schemes and p = 1..5."""
    g = json.load(open(os.path.join(GOLDEN, "table2_convergence.json")))
    s = g["setup"]
    Dti, T = s["D_times_t_i"], s["T"]

    def exact(x, t):
        return np.exp(-(x - 0.5) ** 2 / (4 * (Dti + t))) / np.sqrt(4 * math.pi * (Dti + t))

    for scheme, key in (("compact", "compact"), ("br1", "standard")):
        for p in range(1, 6):
            errs = []
            for N in s["elements"][str(p)][2:]:
                x = W.points_1d(N, p, 0.0, 1.0)
                h = 1.0 / N
                nsteps = math.ceil(T / (0.05 * h * h / (p + 1) ** 2))
                u = oracle_lib.rk4_1d(exact(x, 0.0), p, 0.0, 1.0, T / nsteps, nsteps, scheme=scheme)
                errs.append(l2_error(u, exact(x, T), p, h))
            rate = math.log(errs[0] / errs[1]) / math.log(2.0)
            assert abs(rate - g["rates"][key][str(p)]) < 0.1, (scheme, p, rate)


@pytest.mark.parametrize("p", range(1, 7))
def test_stencil_width_1d(oracle_lib, p):
    """Perturbing one element changes the residual on 3 elements (compact,
    section 2.2) and on 5 elements (BR1, section 2.1)."""
    N, x0, x1 = 11, 0.0, 1.0
    rng = np.random.Generator(np.random.PCG64(p))
    u = rng.uniform(-1, 1, (N, p + 1))
    for scheme, width in (("compact", 3), ("br1", 5)):
        R0 = oracle_lib.rhs_1d(u, p, x0, x1, scheme=scheme)
        u1 = u.copy()
        u1[5] += rng.uniform(-1, 1, p + 1)
        R1 = oracle_lib.rhs_1d(u1, p, x0, x1, scheme=scheme)
        changed = np.nonzero(np.abs(R1 - R0).max(axis=1))[0]
        assert len(changed) == width
        assert list(changed) == list(range(5 - width // 2, 5 + width // 2 + 1))


@pytest.mark.parametrize("physics", ["diffusion", "pme"])
@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_discrete_conservation_1d(oracle_lib, physics, scheme):
    """Gauss quadrature of du/dt vanishes on a periodic mesh."""
    for p in range(1, 7):
        N = 9
        rng = np.random.Generator(np.random.PCG64(10 + p))
        u = rng.uniform(0.1, 1.0, (N, p + 1))
        R = oracle_lib.rhs_1d(u, p, -1.0, 2.0, scheme=scheme, physics=physics, coef=1.0 if physics == "diffusion" else 2.0)
        _, ws = W.gl_nodes(p + 1)
        tot = np.sum(R * ws[None, :])
        mag = np.sum(np.abs(R) * ws[None, :])
        assert abs(tot) < 1e-13 * mag


def global_matrix(oracle_lib, N, p, scheme, x0=0.0, x1=2 * math.pi):
    n = p + 1
    A = np.zeros((N * n, N * n))
    for c in range(N * n):
        e = np.zeros(N * n)
        e[c] = 1.0
        A[:, c] = oracle_lib.rhs_1d(e.reshape(N, n), p, x0, x1, scheme=scheme).ravel()
    return A


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_spectrum_real_nonpositive_low_modes(oracle_lib, scheme, p):
    """Centred schemes give a real spectrum (section 3, Re(omega) = 0), no
    growth, and the low wavenumbers follow Im(omega) = -theta^2."""
    A = global_matrix(oracle_lib, 8, p, scheme)
    lam = np.linalg.eigvals(A)
    scale = np.abs(lam).max()
    assert np.abs(lam.imag).max() < 1e-10 * scale
    assert lam.real.max() < 1e-10 * scale
    lr = np.sort(lam.real)[::-1]
    assert abs(lr[0]) < 1e-10 * scale                     # constant mode
    if not (scheme == "br1"):
        assert abs(lr[1] + 1.0) < 2e-2 and abs(lr[2] + 1.0) < 2e-2   # k = 1 pair


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_spurious_zero_mode_of_br1(oracle_lib, p):
    """On an even number of elements BR1 has a second zero eigenvalue (an
    undamped non-constant mode: theta = pi for even p, theta = 0 for odd p);
    the compact scheme keeps only the constant (sections 3 and 4.2)."""
    for scheme, nzero in (("br1", 2), ("compact", 1)):
        A = global_matrix(oracle_lib, 8, p, scheme)
        lam = np.linalg.eigvals(A)
        scale = np.abs(lam).max()
        assert np.sum(np.abs(lam) < 1e-9 * scale) == nzero, scheme


def test_dirac_mass_preserved(oracle_lib):
    """Seed-placed discrete delta (1/h on one element): its Gauss integral
    is one and stays one under RK4 (both schemes)."""
    N, p, x0, x1 = 32, 4, 0.0, 1.0
    u, e = W.dirac_1d(N, p, x0, x1, seed=0)
    _, ws = W.gl_nodes(p + 1)
    h = (x1 - x0) / N
    assert abs(np.sum(u * ws[None, :]) * h / 2 - 1.0) < 1e-14
    for scheme in ("br1", "compact"):
        dt = 0.05 * h * h / (p + 1) ** 2
        v = oracle_lib.rk4_1d(u, p, x0, x1, dt, 200, scheme=scheme)
        assert abs(np.sum(v * ws[None, :]) * h / 2 - 1.0) < 1e-12


def test_pme_follows_barenblatt(oracle_lib):
    """Porous medium equation u_t = (u^2)_xx (m = 2, C = 0.1) from the ZKB
    profile: mass is conserved exactly and the error against the exact
    solution (restricted to |x|^2 < 0.9 H) falls with refinement for both
    schemes (section 4.3)."""
    m, C, p, x0, x1 = 2.0, 0.1, 3, -4.0, 4.0
    errs = {}
    for scheme in ("br1", "compact"):
        for N in (64, 128):
            h = (x1 - x0) / N
            t0 = W.barenblatt_t0(m, 1.0, C)
            x = W.points_1d(N, p, x0, x1)
            u = W.barenblatt(x, t0, m, C)
            umax = u.max()
            dt = 0.05 * h * h / (m * umax ** (m - 1) * (p + 1) ** 2)
            T = 4 * t0
            nsteps = math.ceil((T - t0) / dt)
            v = oracle_lib.rk4_1d(u, p, x0, x1, (T - t0) / nsteps, nsteps, scheme=scheme,
                                  physics="pme", coef=m)
            _, ws = W.gl_nodes(p + 1)
            assert abs(np.sum((v - u) * ws[None, :])) < 1e-12 * np.sum(np.abs(u) * ws[None, :])
            mask = x * x < 0.9 * W.barenblatt_H(m, T, C)
            ex = W.barenblatt(x, T, m, C)
            errs[(scheme, N)] = math.sqrt(np.sum(((v - ex) ** 2 * ws[None, :])[mask]) * h / 2)
        assert errs[(scheme, 128)] < errs[(scheme, 64)]
