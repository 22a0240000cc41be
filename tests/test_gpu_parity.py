"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

Bar: per variable, max |R_gpu - R_oracle| / max |R_oracle| <= 1e-12 in FP64;
FP32 within the tolerances stated below (normwise, per variable).
"""
import math

import numpy as np
import pytest

from paper_2608_09615_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
# FP32 (reference state removed for Navier-Stokes): contractions in single
# precision over n <= 7 terms on O(1) data, fluxes in single precision; the
# bound is a few hundred FP32 ulps of the largest term, normwise (measured
# at most 7.0e-5 for Navier-Stokes, at 32^3 with BR1).
FP32_TOL_SCALAR = 2e-5
FP32_TOL_NS = 1e-4
# BF16x3 (gradient and divergence contractions as hi*hi + hi*lo + lo*hi BF16
# products, FP32 accumulation; everything else as FP32): each split operand
# carries ~2^-18 relative error, so one directional divergence is good to
# ~1e-5 of its size.  The density and energy residuals are sums of three
# directional divergences that cancel to ~1/300 of their size at Ma = 0.1
# (div(rho u) and div((rho E + p) u) ~ Ma^2), which leaves ~3e-3 normwise in
# those two variables (momentum ~3e-5); measured at most 4.8e-3 (p = 5).
BF16X3_TOL_NS = 6e-3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def relerr(R, Ro, floor=0.0):
    """max over variables of max|R - Ro| / max(max|Ro|, floor); the floor is
    the operator's natural scale where the exact result may vanish."""
    R = np.asarray(R).reshape(Ro.shape[0], Ro.shape[1], -1)
    Ro = Ro.reshape(Ro.shape[0], Ro.shape[1], -1)
    out = []
    for v in range(Ro.shape[1]):
        den = max(np.abs(Ro[:, v]).max(), floor)
        out.append(np.abs(R[:, v] - Ro[:, v]).max() / (den if den > 0 else 1.0))
    return max(out)


def gpu_rhs(torch, U, nel, p, scheme, physics, precision="fp64", lo=None, hi=None, **kw):
    from paper_2608_09615_amd import SD
    print(f"[gpu rhs] {physics} {scheme} {precision} p={p} nel={nel}", flush=True)
    sd = SD(nel, p, scheme=scheme, physics=physics, precision=precision, lo=lo, hi=hi, **kw)
    u = torch.from_numpy(np.ascontiguousarray(U)).to("cuda")
    R = sd.rhs(u)
    torch.cuda.synchronize()
    return R.cpu().numpy().reshape(U.shape), sd


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("physics", ["diffusion", "pme"])
@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_1d_parity(torch_cuda, oracle_lib, scheme, physics, precision):
    for p in range(1, 9):
        for N in (1, 2, 11):
            rng = np.random.Generator(np.random.PCG64(100 * p + N))
            u = rng.uniform(0.2, 1.0, (N, p + 1))
            coef = 0.7 if physics == "diffusion" else 3.0
            kw = dict(nu=coef) if physics == "diffusion" else dict(pme_m=coef)
            R, _ = gpu_rhs(torch_cuda, u[:, None, :], [N], p, scheme, physics, precision, [-1.0], [2.0], **kw)
            Ro = oracle_lib.rhs_1d(u, p, -1.0, 2.0, scheme=scheme, physics=physics, coef=coef)
            tol = FP64_TOL if precision == "fp64" else FP32_TOL_SCALAR
            scale = coef * np.abs(u).max() * (N / 3.0) ** 2 * (p + 1) ** 2
            assert relerr(R, Ro[:, None, :], scale) < tol, (p, N, relerr(R, Ro[:, None, :], scale))


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_3d_scalar_diffusion_parity(torch_cuda, oracle_lib, scheme, precision):
    prm = oracle_lib.make_params("diffusion", nu=0.9)
    for p in range(1, 7):
        for nel in ((3, 4, 5), (1, 2, 3)):
            U = W.random_scalar_3d(nel, p, seed=p)
            lo, hi = (0.0, -1.0, 0.5), (1.0, 1.0, 2.0)
            R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "diffusion", precision, lo, hi, nu=0.9)
            Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
            tol = FP64_TOL if precision == "fp64" else FP32_TOL_SCALAR
            scale = 0.9 * np.abs(U).max() * (p + 1) ** 2 / 0.5 ** 2
            assert relerr(R, Ro, scale) < tol, (p, nel, relerr(R, Ro, scale))


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6])
def test_3d_ns_parity_fp64(torch_cuda, oracle_lib, scheme, p):
    prm = oracle_lib.make_params("ns", Re=400.0)
    lo, hi = W.tgv_domain()
    for nel in ((3, 4, 5), (2, 1, 3)):
        U = W.perturbed_tgv_state(nel, p, seed=p, noise=1e-2)
        R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "fp64", lo, hi, Re=400.0)
        Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
        assert relerr(R, Ro) < FP64_TOL, (nel, relerr(R, Ro))


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 3, 5, 7])
def test_3d_ns_parity_fp32(torch_cuda, oracle_lib, scheme, p):
    prm = oracle_lib.make_params("ns", Re=1600.0)
    lo, hi = W.tgv_domain()
    nel = (4, 3, 5)
    U = W.perturbed_tgv_state(nel, p, seed=10 + p, noise=1e-3)
    R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "fp32", lo, hi)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    err = relerr(R, Ro)
    print(f"fp32 NS p={p} {scheme}: normwise relative error {err:.3e}")
    assert err < FP32_TOL_NS


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 3, 4, 5, 7])
def test_3d_ns_parity_bf16x3(torch_cuda, oracle_lib, scheme, p):
    """BF16x3 split-precision path (matrix-core gradient and divergence)
    against the FP64 oracle; p = 4, 5 and 7 take two row and K chunks."""
    prm = oracle_lib.make_params("ns", Re=1600.0)
    lo, hi = W.tgv_domain()
    nel = (4, 3, 5)
    U = W.perturbed_tgv_state(nel, p, seed=30 + p, noise=1e-3)
    R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "bf16x3", lo, hi)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    err = relerr(R, Ro)
    per_var = [relerr(R.reshape(Ro.shape)[:, v:v + 1], Ro[:, v:v + 1]) for v in range(5)]
    print(f"bf16x3 NS p={p} {scheme}: normwise relative error {err:.3e}, per variable "
          + " ".join(f"{e:.2e}" for e in per_var))
    assert err < BF16X3_TOL_NS


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [2, 3, 5])
def test_ns_entropy_fix_branch_parity(torch_cuda, oracle_lib, scheme, p):
    """Faces where Harten's fix acts (section 4.4, Roe flux with entropy fix):
    a TGV state with transonic jets along the three axes.  The oracle's RHS
    with the fix differs from the one without it by far more than the bar,
    so the branch is taken; the GPU matches the oracle with the fix."""
    prm = oracle_lib.make_params("ns", Re=400.0)
    prm_off = oracle_lib.make_params("ns", Re=400.0, entropy_fix=0.0)
    lo, hi = W.tgv_domain()
    nel = (4, 3, 5)
    U = W.transonic_jet_state(nel, p, seed=p)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    Roff = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm_off)
    assert relerr(Roff, Ro) > 1e-5
    R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "fp64", lo, hi, Re=400.0)
    err = relerr(R, Ro)
    print(f"entropy-fix faces, NS p={p} {scheme}: FP64 {err:.2e} (fix changes the RHS by {relerr(Roff, Ro):.1e})")
    assert err < FP64_TOL
    R32, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "fp32", lo, hi, Re=400.0)
    print(f"entropy-fix faces, NS p={p} {scheme}: FP32 {relerr(R32, Ro):.2e}")
    assert relerr(R32, Ro) < FP32_TOL_NS


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 7])
def test_3d_ns_parity_fp32_mfma(torch_cuda, oracle_lib, scheme, p):
    """FP32 with the gradient and divergence line contractions on the FP32
    matrix instruction (4x4x1, one K step per instruction): same tolerance as
    the vector FP32 path; p = 4, 5 and 7 take two row chunks."""
    prm = oracle_lib.make_params("ns", Re=1600.0)
    lo, hi = W.tgv_domain()
    nel = (4, 3, 5)
    U = W.perturbed_tgv_state(nel, p, seed=50 + p, noise=1e-3)
    R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", "fp32mfma", lo, hi)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, prm)
    err = relerr(R, Ro)
    print(f"fp32 matrix-core NS p={p} {scheme}: normwise relative error {err:.3e}")
    assert err < FP32_TOL_NS


def test_ns_p7_runs_in_fp32_only(torch_cuda):
    """p = 7 needs one element's 24 480 LDS values per block: 98 KB in FP32
    and BF16x3, 191 KB in FP64, beyond the 160 KB of a compute unit."""
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd.sd import SDError
    lo, hi = W.tgv_domain()
    with pytest.raises(SDError, match="LDS"):
        SD((2, 2, 2), 7, scheme="compact", physics="ns", precision="fp64", lo=lo, hi=hi)
    SD((2, 2, 2), 7, scheme="compact", physics="ns", precision="fp32", lo=lo, hi=hi).close()


@pytest.mark.parametrize("scheme,width", [("compact", 19), ("br1", 25)])
def test_gpu_stencil_width(torch_cuda, oracle_lib, scheme, width):
    nel, p = (7, 7, 7), 2
    lo, hi = W.tgv_domain()
    U0 = W.perturbed_tgv_state(nel, p, seed=4, noise=1e-3)
    U1 = U0.copy()
    U1[3 + 7 * (3 + 7 * 3)] *= 1.001
    R0, _ = gpu_rhs(torch_cuda, U0, nel, p, scheme, "ns", "fp64", lo, hi)
    R1, _ = gpu_rhs(torch_cuda, U1, nel, p, scheme, "ns", "fp64", lo, hi)
    ch = np.abs(R1 - R0).reshape(len(U0), -1).max(1)
    assert (ch > 1e-13 * np.abs(R0).max()).sum() == width


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_rk4_step_parity(torch_cuda, oracle_lib, scheme):
    nel, p = (3, 3, 4), 3
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns")
    U = W.perturbed_tgv_state(nel, p, seed=8, noise=1e-3)
    from paper_2608_09615_amd import SD
    sd = SD(nel, p, scheme=scheme, physics="ns", lo=lo, hi=hi)
    u = torch_cuda.from_numpy(U).to("cuda")
    dt = 2e-3
    for _ in range(3):
        sd.rk_step(u, dt)
    torch_cuda.cuda.synchronize()
    Uo = oracle_lib.rk4_3d(U, nel, lo, hi, p, scheme, prm, dt, 3)
    dU = u.cpu().numpy() - Uo
    assert np.abs(dU).max() < 1e-12 * np.abs(Uo - U).max() + 1e-13


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16x3", "fp32mfma"])
def test_chained_rk_step_matches_rhs_sequence(torch_cuda, scheme, precision):
    """sd_rk_step keeps the stage state in compute precision and lets each
    stage emit the next stage's traces; that must reproduce classical RK4
    built from sd_rhs calls (FP64 stage combinations on the host) up to the
    rounding of those combinations, on a ragged mesh (partial last block)."""
    torch = torch_cuda
    from paper_2608_09615_amd import SD
    nel, p = (3, 4, 5), 3
    lo, hi = W.tgv_domain()
    U = W.perturbed_tgv_state(nel, p, seed=17, noise=1e-3)
    print(f"[chain] {scheme} {precision}", flush=True)
    sd = SD(nel, p, scheme=scheme, physics="ns", precision=precision, lo=lo, hi=hi)
    dt = 2e-3
    u = torch.from_numpy(U).to("cuda")
    for _ in range(2):
        sd.rk_step(u, dt)
    got = u.cpu().numpy()
    v = torch.from_numpy(U).to("cuda")
    for _ in range(2):
        k1 = sd.rhs(v)
        k2 = sd.rhs(v + 0.5 * dt * k1)
        k3 = sd.rhs(v + 0.5 * dt * k2)
        k4 = sd.rhs(v + dt * k3)
        v = v + dt / 6.0 * (((k1 + 2.0 * k2) + 2.0 * k3) + k4)
    ref = v.cpu().numpy()
    sd.close()
    # the two differ only in the rounding of the FP64 stage combinations
    # (the device may fuse u0 + a R into one FMA); in FP32 and BF16x3 such a
    # one-ulp difference can, very rarely, move the rounding of a stage input
    # to FP32, which then shows at the FP32 level for that element
    d = np.abs(got - ref) / np.abs(ref - U).max()
    if precision == "fp64":
        assert d.max() < 1e-12
    else:
        assert np.mean(d < 1e-12) > 0.9999 and d.max() < 1e-5


def test_diagnostics_parity(torch_cuda, oracle_lib):
    nel, p = (4, 3, 5), 3
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns")
    U = W.perturbed_tgv_state(nel, p, seed=9, noise=1e-3)
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd.sd import SDError
    sd = SD(nel, p, scheme="compact", physics="ns", lo=lo, hi=hi)
    d = sd.diagnostics(torch_cuda.from_numpy(U).to("cuda"))
    do = oracle_lib.diag_3d(U, nel, lo, hi, p, prm)
    for k in ("ke", "enstrophy", "mass", "energy", "umax", "smax"):
        assert abs(d[k] - do[k]) <= 1e-12 * abs(do[k]), k
    for i in range(3):
        assert abs(d["mom"][i] - do[f"mom{i}"]) <= 1e-12 * do["mass"]
    assert d["nonfinite"] is False
    # the convective time step: cfl min h / ((p + 1) smax); the mesh is
    # anisotropic in element count, so the smallest h is h_z = 2 pi / 5
    u = torch_cuda.from_numpy(U).to("cuda")
    for cfl in (0.3, 1.0):
        dt = sd.stable_dt(u, cfl)
        assert abs(dt - cfl * (2 * np.pi / 5) / ((p + 1) * do["smax"])) <= 1e-14 * dt
    for cfl in (0.0, -1.0, float("inf"), float("nan")):
        with pytest.raises(SDError):
            sd.stable_dt(u, cfl)
    Ub = U.copy()
    Ub[2, 4, 0, 1, 2] = 0.0                    # rho E = 0 with u != 0: P < 0
    db = sd.diagnostics(torch_cuda.from_numpy(Ub).to("cuda"))
    assert db["smax"] == float("inf") and db["nonfinite"] is False
    with pytest.raises(SDError):
        sd.stable_dt(torch_cuda.from_numpy(Ub).to("cuda"))
    U[5, 2, 1, 1, 1] = np.nan
    d = sd.diagnostics(torch_cuda.from_numpy(U).to("cuda"))
    assert d["nonfinite"] is True


def ulp_sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm, sel):
    """Relative change of the oracle's RHS when every input value moves by
    about one FP64 ulp: the rounding floor any FP64 evaluation shares."""
    R = oracle_lib.rhs_3d_elems(U, nel, lo, hi, p, scheme, prm, sel)
    U2 = U * (1.0 + 2.2e-16 * np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, U.shape))
    R2 = oracle_lib.rhs_3d_elems(U2, nel, lo, hi, p, scheme, prm, sel)
    return R, relerr(R2, R)


def test_tgv_32cubed_sampled_parity(torch_cuda, oracle_lib):
    """Full size of the Re = 1600 TGV workload (32^3 elements, p = 3), both
    schemes and both precisions: sampled elements against the oracle's
    element-wise RHS.  At this size the RHS moves by ~3e-12 (relative) when
    the input moves by one ulp (rho E ~ 180 at Ma = 0.1, second derivatives
    on h = 2 pi/32), so the FP64 bar is max(1e-12, 4 x that sensitivity)."""
    nel, p = (32, 32, 32), 3
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns", Re=1600.0)
    U = W.perturbed_tgv_state(nel, p, seed=21, noise=1e-3, amp=1e-2)
    rng = np.random.Generator(np.random.PCG64(5))
    sel = np.unique(np.concatenate([rng.integers(0, 32 ** 3, 48), [0, 31, 32 ** 2 - 1, 32 ** 3 - 1]]))
    for scheme in ("compact", "br1"):
        Ro, sens = ulp_sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm, sel)
        assert sens < 1e-11
        for precision, tol in (("fp64", max(FP64_TOL, 4 * sens)), ("fp32", FP32_TOL_NS),
                               ("bf16x3", BF16X3_TOL_NS)):
            R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", precision, lo, hi)
            err = relerr(R[sel], Ro)
            print(f"32^3 {scheme} {precision}: error {err:.3e} (ulp sensitivity {sens:.3e})")
            assert err < tol, (scheme, precision, err, sens)


@pytest.mark.parametrize("nel1,p", [(64, 3), (43, 5)])
def test_tgv_re5000_full_size_sampled_parity(torch_cuda, oracle_lib, nel1, p):
    """Full sizes of the Re = 5000 TGV workloads (64^3 elements at p = 3 and
    43^3 at p = 5, about 17 M and 21 M solution points), both schemes and the
    three precisions, in the launch configuration the benchmark times:
    sampled elements (corners of the box included) against the oracle's
    element-wise RHS.  The state is the phase-shifted TGV with pointwise noise
    (a solenoidal perturbation at this size would dominate the test's time).
    FP64 bar: max(1e-12, 4 x the one-ulp sensitivity measured here)."""
    nel = (nel1,) * 3
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns", Re=5000.0)
    print(f"[re5000] {nel1}^3 p={p}: building the state", flush=True)
    U = W.perturbed_tgv_state(nel, p, seed=33, noise=1e-3, amp=0.0)
    ne = nel1 ** 3
    rng = np.random.Generator(np.random.PCG64(6))
    sel = np.unique(np.concatenate([rng.integers(0, ne, 40), [0, nel1 - 1, nel1 ** 2 - 1, ne - 1]]))
    for scheme in ("compact", "br1"):
        Ro, sens = ulp_sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm, sel)
        assert sens < 1e-10
        for precision, tol in (("fp64", max(FP64_TOL, 4 * sens)), ("fp32", FP32_TOL_NS),
                               ("bf16x3", BF16X3_TOL_NS)):
            R, sd = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", precision, lo, hi, Re=5000.0)
            sd.close()
            err = relerr(R[sel], Ro)
            print(f"{nel1}^3 p={p} {scheme} {precision}: error {err:.3e} (ulp sensitivity {sens:.3e})", flush=True)
            assert err < tol, (scheme, precision, err, sens)
            del R


# ---------------------------------------------------------------------------
# Interior-penalty variant (section 3): the normal component of the common
# gradient gains tau (u_R - u_L), tau = eta_IP (p+1)^2 / h.

@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("physics", ["diffusion", "pme"])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ip_1d_parity(torch_cuda, oracle_lib, scheme, physics, precision):
    p, N, eta = 3, 11, 0.5
    coef = 1.0 if physics == "diffusion" else 2.0
    u = 1.0 + 0.3 * np.random.Generator(np.random.PCG64(12)).uniform(-1, 1, (N, p + 1))
    kw = dict(nu=coef) if physics == "diffusion" else dict(pme_m=coef)
    R, _ = gpu_rhs(torch_cuda, u[:, None, :], [N], p, scheme, physics, precision, [-1.0], [2.0], eta_ip=eta, **kw)
    Ro = oracle_lib.rhs_1d(u, p, -1.0, 2.0, scheme=scheme, physics=physics, coef=coef, eta_ip=eta)
    R0 = oracle_lib.rhs_1d(u, p, -1.0, 2.0, scheme=scheme, physics=physics, coef=coef)
    err = relerr(R, Ro[:, None, :])
    print(f"IP 1-D {physics} {scheme} {precision}: {err:.3e} (IP changes R by {relerr(R0[:, None, :], Ro[:, None, :]):.2e})")
    assert err < (FP64_TOL if precision == "fp64" else FP32_TOL_SCALAR)


@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_ip_3d_diffusion_parity(torch_cuda, oracle_lib, scheme):
    p, nel, eta = 2, (3, 2, 4), 0.5
    lo, hi = (0.0, 0.0, 0.0), (1.0, 2.0, 1.5)
    U = W.random_scalar_3d(nel, p, seed=4)
    R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "diffusion", "fp64", lo, hi, nu=0.8, eta_ip=eta)
    Ro = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, oracle_lib.make_params("diffusion", nu=0.8, eta_ip=eta))
    assert relerr(R, Ro) < FP64_TOL


@pytest.mark.parametrize("scheme", ["br1", "compact"])
@pytest.mark.parametrize("p", [2, 3])
def test_ip_ns_parity(torch_cuda, oracle_lib, scheme, p):
    """NS with the penalty in FP64, FP32 and BF16x3.  The penalty takes the
    jump of two traces of rho E ~ 180 that differ by ~1e-3, so the RHS
    inherits the FP64 rounding of the traces: the FP64 bar is
    max(1e-12, 4 x the oracle's one-ulp sensitivity)."""
    nel, eta = (3, 4, 2), 1.0
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns", Re=400.0, eta_ip=eta)
    U = W.perturbed_tgv_state(nel, p, seed=40 + p, noise=1e-3)
    sel = np.arange(int(np.prod(nel)))
    Ro, sens = ulp_sensitivity(oracle_lib, U, nel, lo, hi, p, scheme, prm, sel)
    R0 = oracle_lib.rhs_3d(U, nel, lo, hi, p, scheme, oracle_lib.make_params("ns", Re=400.0))
    assert relerr(R0, Ro) > 1e-4                      # the penalty acts
    for precision, tol in (("fp64", max(FP64_TOL, 4 * sens)), ("fp32", FP32_TOL_NS), ("bf16x3", BF16X3_TOL_NS)):
        R, _ = gpu_rhs(torch_cuda, U, nel, p, scheme, "ns", precision, lo, hi, Re=400.0, eta_ip=eta)
        err = relerr(R, Ro)
        print(f"IP NS p={p} {scheme} {precision}: {err:.3e} (ulp sensitivity {sens:.2e})")
        assert err < tol, (precision, err, sens)


# ---------------------------------------------------------------------------
# SSP-RK(5,4) (section 4.4's integrator) against the reference integrator.

@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("scheme", ["br1", "compact"])
def test_ssprk54_step_parity(torch_cuda, oracle_lib, scheme, precision):
    from oracle import ssprk
    from paper_2608_09615_amd import SD
    nel, p = (3, 3, 4), 3
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns")
    U = W.perturbed_tgv_state(nel, p, seed=9, noise=1e-3)
    print(f"[ssprk54] {scheme} {precision}", flush=True)
    sd = SD(nel, p, scheme=scheme, physics="ns", precision=precision, lo=lo, hi=hi, integrator="ssprk54")
    u = torch_cuda.from_numpy(U).to("cuda")
    dt = 2e-3
    for _ in range(2):
        sd.rk_step(u, dt)
    got = u.cpu().numpy()
    sd.close()
    ref = ssprk.integrate(lambda x: oracle_lib.rhs_3d(x, nel, lo, hi, p, scheme, prm), U, dt, 2)
    change = np.abs(ref - U).max()
    err = np.abs(got - ref).max() / change
    print(f"ssprk54 {scheme} {precision}: {err:.3e} relative to the change {change:.3e}")
    # The Shu-Osher stages are convex combinations of whole states (rho E ~ 180),
    # so each of the 2 x 5 combinations rounds at the scale of |U|, not of the
    # change (~0.04 here): the device evaluates them with fused multiply-adds,
    # the oracle term by term.  Allow one ulp of max|U| per combination and
    # side on top of the 1e-12 relative bar (~2e-11 of the change here); a
    # coefficient wrong in its 12th digit still moves the result by more.
    floor = 2 * 10 * np.finfo(np.float64).eps * np.abs(U).max() / change
    assert err < (max(1e-12, floor) if precision == "fp64" else FP32_TOL_NS)


def test_ssprk54_1d_diffusion_parity(torch_cuda, oracle_lib):
    from oracle import ssprk
    from paper_2608_09615_amd import SD
    p, N = 4, 9
    u0 = np.random.Generator(np.random.PCG64(19)).normal(size=(N, p + 1))
    sd = SD([N], p, scheme="compact", physics="diffusion", lo=[0.0], hi=[2.0], nu=0.6, integrator="ssprk54")
    u = torch_cuda.from_numpy(u0[:, None, :].copy()).to("cuda")
    dt = 1e-4
    for _ in range(3):
        sd.rk_step(u, dt)
    got = u.cpu().numpy()[:, 0, :]
    sd.close()
    ref = ssprk.integrate(lambda x: oracle_lib.rhs_1d(x, p, 0.0, 2.0, scheme="compact", coef=0.6), u0, dt, 3)
    assert np.abs(got - ref).max() < 1e-12 * np.abs(ref - u0).max()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ns_parity_brick_order(torch_cuda, oracle_lib, precision):
    """Meshes with even element counts whose half x count holds whole block
    runs take the brick order of the blocks (each XCD one octant of the
    box): every element's RHS against the oracle (FP64 bar max(1e-12, 4 x
    the oracle's one-ulp sensitivity), as for the other full meshes with
    small elements), and two chained RK4 steps against the RHS sequence."""
    torch = torch_cuda
    from paper_2608_09615_amd import SD
    lo, hi = W.tgv_domain()
    prm = oracle_lib.make_params("ns")
    for nel in ((8, 4, 6), (16, 2, 4)):
        U = W.perturbed_tgv_state(nel, 3, seed=31, noise=1e-3)
        R, sd = gpu_rhs(torch, U, nel, 3, "compact", "ns", precision, lo, hi)
        sd.close()
        sel = np.arange(int(np.prod(nel)), dtype=np.int64)
        Ro, sens = ulp_sensitivity(oracle_lib, U, nel, lo, hi, 3, "compact", prm, sel)
        Ro = np.asarray(Ro).reshape(U.shape)
        err = relerr(R, Ro)
        print(f"brick order {nel} {precision}: {err:.2e} (ulp sensitivity {sens:.2e})", flush=True)
        assert err < (max(FP64_TOL, 4 * sens) if precision == "fp64" else FP32_TOL_NS), (nel, err, sens)
        sd = SD(nel, 3, scheme="compact", physics="ns", precision=precision, lo=lo, hi=hi)
        dt = 2e-3
        u = torch.from_numpy(U).to("cuda")
        for _ in range(2):
            sd.rk_step(u, dt)
        v = torch.from_numpy(U).to("cuda")
        for _ in range(2):
            k1 = sd.rhs(v)
            k2 = sd.rhs(v + 0.5 * dt * k1)
            k3 = sd.rhs(v + 0.5 * dt * k2)
            k4 = sd.rhs(v + dt * k3)
            v = v + dt / 6.0 * (((k1 + 2.0 * k2) + 2.0 * k3) + k4)
        d = np.abs(u.cpu().numpy() - v.cpu().numpy()) / np.abs(v.cpu().numpy() - U).max()
        sd.close()
        if precision == "fp64":
            assert d.max() < 1e-12
        else:
            assert np.mean(d < 1e-12) > 0.9999 and d.max() < 1e-5
