"""Batched Bloch analysis on the GPU (section 3 and the appendix) against
the reference's Bloch matrices, eigenvalues and combined mode.

B(theta) is built on the device by the solver's own 1-D steps applied to a
Bloch wave (a construction independent of the reference's matrix algebra),
its eigenvalues by Hessenberg reduction and shifted QR, and the combined
mode by scaling and squaring of exp(B t); the reference uses its matrix
formulas, LAPACK's eigensolver and the eigenvector expansion.

Bars (FP64): B to 1e-12 of max|B| over the theta grid; eigenvalues to
1e-12 of that scale (both backward-stable, measured ~5e-15).  G: the
squarings (up to ~14 here) amplify rounding to ~2^s eps of ||exp(B t)|| ~ 1,
so |dG| <= 1e-12 + 1e-11 |G|, and t |d omega| = |d log G| <= 1e-11 +
1e-12 / |G| (the real part of omega t compared modulo 2 pi).
"""
import math

import numpy as np
import pytest

from oracle import bloch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def reference(p, scheme, thetas, ts, J, eta):
    n = p + 1
    B = np.zeros((len(thetas), n, n), complex)
    lam = np.zeros((len(thetas), n), complex)
    G = np.zeros((len(thetas), len(ts)), complex)
    om = np.zeros_like(G)
    for k, th in enumerate(thetas):
        B[k] = bloch.bloch_matrix(p, th, J, scheme, eta, 2 * J)
        ev = np.linalg.eigvals(B[k])
        lam[k] = ev[np.lexsort((ev.imag, -ev.real))]
        for j, t in enumerate(ts):
            G[k, j], om[k, j] = bloch.combined_mode(p, th, t, J, scheme, eta, 2 * J)
    return B, lam, G, om


def run(torch, p, scheme, thetas, ts, J=0.5, eta=0.0):
    from paper_2608_09615_amd.sd import bloch as gpu_bloch
    print(f"[bloch] p={p} {scheme} J={J} eta={eta} ntheta={len(thetas)} nt={len(ts)}", flush=True)
    th = torch.tensor(np.asarray(thetas, dtype=np.float64), device="cuda")
    t = torch.tensor(np.asarray(ts, dtype=np.float64), device="cuda") if len(ts) else None
    out = gpu_bloch(p, scheme, th, t, J=J, eta_ip=eta)
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def check(got, ref, ts):
    B, lam, G, om = ref
    scale = np.abs(B).max()
    eB = np.abs(got["B"] - B).max() / scale
    eL = np.abs(got["lam"] - lam).max() / scale
    print(f"B {eB:.2e}  lam {eL:.2e}", end="")
    assert eB < 1e-12 and eL < 1e-12
    if len(ts):
        dG = np.abs(got["G"] - G)
        assert np.all(dG <= 1e-12 + 1e-11 * np.abs(G))
        # omega t = -arg G + i log|G|: the real part is defined modulo 2 pi
        # (principal log); where G is real and negative (BR1, p = 4 near
        # theta = pi at t = 1) rounding of Im G ~ 1e-17 picks the branch
        d = (got["omega"] - om) * np.asarray(ts)[None, :]
        d = (np.mod(d.real + math.pi, 2 * math.pi) - math.pi) + 1j * d.imag
        dlog = np.abs(d)
        assert np.all(dlog <= 1e-11 + 1e-12 / np.abs(G))
        print(f"  G {(dG / np.abs(G)).max():.2e}  log G {dlog.max():.2e}")
    else:
        print()


THETAS = np.concatenate([np.linspace(-math.pi, math.pi, 41), [1e-3, 0.02, math.pi - 1e-3]])
TS = [1e-3, 0.1, 1.0]


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
def test_bloch_parity(torch_cuda, scheme, p):
    got = run(torch_cuda, p, scheme, THETAS, TS)
    check(got, reference(p, scheme, THETAS, TS, 0.5, 0.0), TS)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p,eta,J", [(3, 0.01, 0.5), (3, 0.05, 0.5), (4, 0.02, 0.25), (2, 1.0, 1.3)])
def test_bloch_parity_interior_penalty_and_element_size(torch_cuda, scheme, p, eta, J):
    got = run(torch_cuda, p, scheme, THETAS, TS, J=J, eta=eta)
    check(got, reference(p, scheme, THETAS, TS, J, eta), TS)


def test_bloch_degenerate_and_edge_cases(torch_cuda):
    torch = torch_cuda
    from paper_2608_09615_amd.sd import bloch as gpu_bloch
    # no wavenumbers: nothing to do; no times: no combined mode
    out = gpu_bloch(3, "compact", torch.zeros(0, dtype=torch.float64, device="cuda"))
    assert out["B"].shape == (0, 4, 4) and out["lam"].shape == (0, 4)
    got = run(torch, 3, "compact", [0.4, 2.0], [])
    assert "G" not in got
    check(got, reference(3, "compact", [0.4, 2.0], [], 0.5, 0.0), [])
    # times that are not positive and finite give NaN, the others are fine
    ts = [0.0, -1.0, float("inf"), float("nan"), 0.5]
    got = run(torch, 2, "br1", [0.3], ts)
    assert np.all(np.isnan(got["G"][0, :4])) and np.all(np.isnan(got["omega"][0, :4]))
    G, om = bloch.combined_mode(2, 0.3, 0.5, 0.5, "br1")
    assert abs(got["G"][0, 4] - G) <= 1e-12 + 1e-11 * abs(G)
    # theta = 0: the constant is steady (G = 1, omega = 0); BR1 keeps a second
    # zero eigenvalue at theta = 0 for odd p, at theta = pi for even p
    got = run(torch, 3, "br1", [0.0, math.pi], [1.0])
    assert abs(got["G"][0, 0] - 1.0) < 1e-12 and abs(got["omega"][0, 0]) < 1e-11
    scale = np.abs(got["B"]).max()
    assert np.sum(np.abs(got["lam"][0]) < 1e-9 * scale) == 2
    got = run(torch, 3, "compact", [0.0], [1.0])
    assert np.sum(np.abs(got["lam"][0]) < 1e-9 * np.abs(got["B"]).max()) == 1


def test_bloch_large_batch_sampled(torch_cuda):
    """The benchmark's sweep size (2^16 wavenumbers, p = 3, three times):
    every output finite, sampled entries against the reference, and the
    eigenvalue ordering."""
    n = 1 << 16
    th = np.linspace(0.0, math.pi, n)
    got = run(torch_cuda, 3, "compact", th, TS)
    for k in ("B", "lam", "G", "omega"):
        assert np.all(np.isfinite(got[k][1:])), k
    assert np.all(np.diff(got["lam"].real, axis=1) <= 0)
    idx = np.random.Generator(np.random.PCG64(5)).choice(n, 64, replace=False)
    ref = reference(3, "compact", th[idx], TS, 0.5, 0.0)
    check({k: v[idx] for k, v in got.items()}, ref, TS)
