"""sd_rk_run: whole RK4 runs of one-dimensional FP64 scalar problems in one
launch (one block, the mesh in LDS), against the same number of sd_rk_step
calls.  The one-launch run evaluates the separate kernels' expressions in
their order; where the compiler contracts a product and a sum into one
fused multiply-add in one kernel and not in the other, the last bit of a
value may differ (measured: 4e-16 after 37 steps with the interior penalty,
1.7e-16 after the 2076 steps of the 1-D diffusion run, 0 in the other
cases), so the bar is a few ulps of the state per step.  Contexts the one-launch path does not cover take the steps one by
one and agree exactly."""
import math

import numpy as np
import pytest

from paper_2608_09615_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def run_pair(torch, make, U0, dt, nsteps):
    """The state after nsteps sd_rk_step calls and after one sd_rk_run."""
    a, b = make(), make()
    ua = torch.from_numpy(np.ascontiguousarray(U0)).to("cuda")
    ub = ua.clone()
    for _ in range(nsteps):
        a.rk_step(ua, dt)
    b.rk_run(ub, dt, nsteps)
    torch.cuda.synchronize()
    xa, xb = ua.cpu().numpy(), ub.cpu().numpy()
    a.close()
    b.close()
    return xa, xb


@pytest.mark.parametrize("scheme", ["compact", "br1"])
@pytest.mark.parametrize("physics", ["diffusion", "pme"])
@pytest.mark.parametrize("p,N,eta", [(1, 7, 0.0), (3, 16, 0.0), (3, 5, 1.5), (6, 9, 0.0), (7, 1, 0.0), (2, 2, 0.5)])
def test_rk_run_matches_steps(torch_cuda, scheme, physics, p, N, eta):
    """Both schemes, both scalar laws, with and without the interior
    penalty; one- and two-element periodic meshes (an element is its own
    neighbour, or both neighbours are the same element) and ragged counts."""
    print(f"[rk_run] {scheme} {physics} p={p} N={N} eta={eta}", flush=True)
    from paper_2608_09615_amd import SD
    x = W.points_1d(N, p, -1.0, 2.0)
    U0 = (1.0 + 0.4 * np.sin(2 * math.pi * x / 3.0) + 0.1 * np.cos(6 * math.pi * x / 3.0))[:, None, :]
    coef = 0.7 if physics == "diffusion" else 2.0
    kw = dict(nu=coef) if physics == "diffusion" else dict(pme_m=int(coef))
    h = 3.0 / N
    dt = 0.02 * h * h / (p + 1) ** 2 / coef
    make = lambda: SD([N], p, scheme=scheme, physics=physics, precision="fp64", lo=[-1.0], hi=[2.0],
                      eta_ip=eta, **kw)
    xa, xb = run_pair(torch_cuda, make, U0, dt, 37)
    d = float(np.abs(xa - xb).max())
    print(f"rk_run {scheme} {physics} p={p} N={N}: max |difference| {d:.3e}", flush=True)
    assert np.isfinite(xa).all()
    assert d <= 37 * 4e-16 * np.abs(xa).max()


def test_rk_run_diffusion_whole_run(torch_cuda):
    """The 1-D diffusion run of 16 elements at p = 3 (sin x on [0, 2 pi],
    nu = 1, 2076 RK4 steps to t = 1): the one-launch run equals the steps
    and is as close to exp(-t) sin x as the scheme is (compact: about 4e-6)."""
    from paper_2608_09615_amd import SD
    N, p = 16, 3
    x = W.points_1d(N, p, 0.0, 2 * math.pi)
    U0 = np.sin(x)[:, None, :]
    h = 2 * math.pi / N
    nst = math.ceil(1.0 / (0.05 * h * h / (p + 1) ** 2))
    dt = 1.0 / nst
    make = lambda: SD([N], p, scheme="compact", physics="diffusion", precision="fp64", lo=[0.0], hi=[2 * math.pi])
    xa, xb = run_pair(torch_cuda, make, U0, dt, nst)
    err = float(np.abs(xb[:, 0, :] - math.exp(-1.0) * np.sin(x)).max())
    print(f"whole run: {nst} steps, difference {np.abs(xa - xb).max():.3e}, error {err:.3e}", flush=True)
    assert nst == 2076
    assert np.abs(xa - xb).max() <= 1e-13
    assert err < 1e-5


def test_rk_run_largest_one_block_mesh(torch_cuda):
    """256 elements at p = 7: 2048 solution points, the largest mesh held in
    one block (117 KB of LDS)."""
    from paper_2608_09615_amd import SD
    N, p = 256, 7
    x = W.points_1d(N, p, 0.0, 1.0)
    U0 = (np.sin(2 * math.pi * x) + 0.3 * np.sin(6 * math.pi * x))[:, None, :]
    h = 1.0 / N
    dt = 0.05 * h * h / (p + 1) ** 2
    make = lambda: SD([N], p, scheme="br1", physics="diffusion", precision="fp64", lo=[0.0], hi=[1.0])
    xa, xb = run_pair(torch_cuda, make, U0, dt, 11)
    assert np.abs(xa - xb).max() <= 11 * 4e-16 * np.abs(xa).max()


@pytest.mark.parametrize("case", ["1d_large", "1d_fp32", "1d_p8", "3d_ns", "1d_ssprk54"])
def test_rk_run_other_contexts_take_the_steps(torch_cuda, case):
    """Contexts outside the one-launch path: more than 2048 points, FP32,
    p = 8, three-dimensional Navier-Stokes, the SSP integrator."""
    from paper_2608_09615_amd import SD
    if case == "3d_ns":
        nel, p = (3, 2, 2), 2
        lo, hi = W.tgv_domain()
        U0 = W.perturbed_tgv_state(nel, p, seed=2, noise=1e-3)
        make = lambda: SD(nel, p, scheme="compact", physics="ns", precision="fp64", lo=lo, hi=hi)
        dt = 1e-3
    else:
        N, p = {"1d_large": (300, 7), "1d_fp32": (16, 3), "1d_p8": (8, 8), "1d_ssprk54": (16, 3)}[case]
        prec = "fp32" if case == "1d_fp32" else "fp64"
        integ = "ssprk54" if case == "1d_ssprk54" else "rk4"
        x = W.points_1d(N, p, 0.0, 1.0)
        U0 = np.sin(2 * math.pi * x)[:, None, :]
        dt = 0.05 * (1.0 / N) ** 2 / (p + 1) ** 2
        make = lambda: SD([N], p, scheme="compact", physics="diffusion", precision=prec, lo=[0.0], hi=[1.0],
                          integrator=integ)
    xa, xb = run_pair(torch_cuda, make, U0, dt, 5)
    assert np.abs(xa - xb).max() == 0.0


def test_rk_run_arguments(torch_cuda):
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd.sd import SDError
    N, p = 4, 3
    x = W.points_1d(N, p, 0.0, 1.0)
    sd = SD([N], p, scheme="compact", physics="diffusion", precision="fp64", lo=[0.0], hi=[1.0])
    u = torch_cuda.from_numpy(np.sin(2 * math.pi * x)[:, None, :].copy()).to("cuda")
    before = u.clone()
    sd.rk_run(u, 1e-4, 0)
    assert torch_cuda.equal(u, before)
    with pytest.raises(SDError):
        sd.rk_run(u, 1e-4, -1)
    with pytest.raises(SDError):
        sd.rk_run(u, float("nan"), 3)
    sd.close()
