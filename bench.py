"""Throughput of the SD right-hand side on one MI355X.

Workload: compressible Navier-Stokes Taylor-Green vortex, Re = 1600, Ma = 0.1,
Pr = 0.71, gamma = 1.4 on the periodic box [0, 2 pi]^3 with 32^3 hexahedra
at p = 3 (2 097 152 solution points, 5 conserved variables), compact scheme.
One bench step is one classical RK4 step: four right-hand sides and four FP64
stage updates on the device-resident state (``--integrator ssprk54``: five
right-hand sides and five FP64 combinations).  The metric counts solution
points (DOF) per RK stage: GDOF/s = n_el (p+1)^3 * stages * steps / time.

Prints one JSON line.  ``value`` is the FP32 path (contractions and fluxes in
FP32, reference state removed, FP64 RK accumulation); the FP64 path is timed
beside it under ``fp64``.  The roofline of the right-hand-side kernels uses
HIP events recorded by the library around every RHS inside the timed region
(sd_timing) on the stream the kernels run on.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_FP64_TFLOPS = 78.6
PEAK_BF16_TFLOPS = 2500.0     # dense BF16 matrix cores

# Algorithmic work per solution point and RHS at p = 3, Navier-Stokes:
# contractions 18 nv (n+1) MAC = 450 MAC = 900 flop (interpolation to the three
# flux-point families, gradient, gradient to flux points, divergence) plus the
# pointwise fluxes, ~525 flop-equivalents (sqrt, division counted as one).
FLOP_PER_DOF = {3: 900.0 + 525.0, 5: 1260.0 + 480.0}
# Algorithmic bytes per solution point and RHS: read u, write du/dt, FP64.
BYTES_PER_DOF = 80.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30, help="timed RK4 steps")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nel", type=int, default=32)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--scheme", default="compact")
    ap.add_argument("--Re", type=float, default=1600.0)
    ap.add_argument("--eta-ip", type=float, default=0.0, help="interior-penalty coefficient (0: off)")
    ap.add_argument("--integrator", default="rk4", choices=["rk4", "ssprk54"],
                    help="rk4: 4 RHS per step; ssprk54: 5 RHS per step (section 4.4's scheme)")
    ap.add_argument("--ke-steps", type=int, default=150, help="RK4 steps of the FP32-vs-FP64 KE check")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=32768, help="elements in the oracle sample")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="wall time of the oracle sample")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="before timing, copy this many MiB device to device (calibrates byte counters)")
    ap.add_argument("--precisions", default="fp32,fp64,bf16x3,fp32mfma",
                    help="FP32 (vector), FP64, BF16x3 and FP32 matrix-core paths; fp32 and fp64 are needed for the "
                         "JSON line")
    ap.add_argument("--bloch-theta", type=int, default=1 << 16,
                    help="wavenumbers of the Bloch / combined-mode sweep (0: skip it)")
    ap.add_argument("--large", type=int, default=1,
                    help="also time the Re = 5000 workloads at 64^3 p = 3 and 43^3 p = 5 (0: skip them)")
    ap.add_argument("--developed", type=int, default=1,
                    help="also time the RHS on the state advanced to t* = 9 (0: skip it)")
    ap.add_argument("--curv-nel", type=int, default=32,
                    help="elements per direction of the curvilinear workloads (0: skip them)")
    ap.add_argument("--curv-p", type=int, default=3, help="degree of the curvilinear workloads")
    ap.add_argument("--curv-scheme", default="compact", choices=["compact", "br1"])
    ap.add_argument("--curv-precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the --only curvilinear workloads")
    ap.add_argument("--closure-nel", type=int, default=16,
                    help="elements per direction of the learned-closure timing (0: skip it)")
    ap.add_argument("--only", choices=["bloch", "curvilinear", "curvilinear_ns", "closure", "training", "oned"],
                    default=None,
                    help="time only that workload and print its record")
    return ap.parse_args()


# the sources that define k_traces_ns and k_rhs_ns, their operators and their
# launch configuration, with the compiler flags (any change there invalidates
# the counter record)
TRAFFIC_SOURCES = ["sd_ns_kernel.h", "sd_internal.h", "sd_physics.h", "sd_dispatch.inc", "sd_operators.cpp"]
# dense peaks of the matrix instructions the variants use
PEAK_FP32_MFMA_TFLOPS = 157.3


CURV_TRAFFIC_SOURCES = ["sd_curv_kernel.h", "sd_curv.inc", "sd_internal.h", "sd_physics.h", "sd_operators.cpp"]


# the sources of k_closure_fused and its launch
CLOSURE_TRAFFIC_SOURCES = ["sd_closure.inc", "sd_mlp.h", "sd_internal.h"]


def sources_sha256(names=None):
    from paper_2608_09615_amd.build import sources_sha256 as sha
    return sha(names or TRAFFIC_SOURCES)


def rhs_record(args):
    """The committed counter record of k_rhs_ns on the 32^3 p = 3 compact
    workload, or None when the workload differs or a kernel source has
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "rhs_traffic_tgv32p3.json")
    if not (args.nel == 32 and args.p == 3 and args.scheme == "compact" and not args.eta_ip
            and args.integrator == "rk4" and os.path.exists(path)):
        return None
    with open(path) as f:
        rec = json.load(f)
    if sources_sha256() != rec["sources_sha256"]:
        return None
    return rec


def measured_traffic(args, precision):
    """HBM bytes per RK stage (one k_rhs_ns launch) from the committed
    FETCH_SIZE / WRITE_SIZE counter runs, or None (see rhs_record)."""
    rec = rhs_record(args)
    return None if rec is None else rec["per_stage_bytes"].get(precision)


def mfma_use(args, precision, rhs_ms):
    """Matrix-instruction use of a variant from the committed counter record:
    SQ_INSTS_MFMA per launch, the flops one instruction does, and the rate
    over the live launch time against the instruction type's dense peak."""
    rec = rhs_record(args)
    if rec is None or precision not in rec.get("mfma_insts_per_launch", {}):
        return None
    n = rec["mfma_insts_per_launch"][precision]
    flop, peak = (2048.0, PEAK_BF16_TFLOPS) if precision == "bf16x3" else (512.0, PEAK_FP32_MFMA_TFLOPS)
    rate = n * flop / (rhs_ms * 1e-3) / 1e12
    return {"insts_per_launch": n, "flop_per_inst": flop, "tflops": rate, "peak": peak, "mfma_frac": rate / peak,
            "instruction": "v_mfma_f32_4x4x4_16b_bf16" if precision == "bf16x3" else "v_mfma_f32_4x4x1_16b_f32"}


def ke_record(args):
    """The committed t* = 20 kinetic-energy / enstrophy record of the 32^3
    p = 3 compact workload (histories of every precision against FP64), or
    None when the workload differs or the kernel sources have changed."""
    path = os.path.join(ROOT, "profiles", "ke_history_tgv32p3.json")
    if not (args.nel == 32 and args.p == 3 and args.scheme == "compact" and not args.eta_ip
            and args.integrator == "rk4" and args.Re == 1600.0 and os.path.exists(path)):
        return None
    with open(path) as f:
        rec = json.load(f)
    if sources_sha256(rec["sources"]) != rec["sources_sha256"]:
        return None
    return {"t_end": rec["t_end"], "command": rec["command"], "errors_vs_fp64": rec["errors"]}


def run_path(torch, W, args, precision, U0, dt):
    from paper_2608_09615_amd import SD
    lo, hi = W.tgv_domain()
    nel = (args.nel,) * 3
    sd = SD(nel, args.p, scheme=args.scheme, physics="ns", precision=precision, lo=lo, hi=hi,
            Re=args.Re, Ma=0.1, Pr=0.71, gamma=1.4, eta_ip=args.eta_ip, integrator=args.integrator)
    u = torch.from_numpy(U0).to("cuda")
    for _ in range(args.warmup):
        sd.rk_step(u, dt)
    torch.cuda.synchronize()
    sd.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sd.rk_step(u, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the end state's diagnostics (finiteness, kinetic energy), outside the
    # timed steps
    diag = sd.diagnostics(u)
    rhs_ms, rhs_count = sd.timing_read()
    sd.timing(False)
    ne = args.nel ** 3
    dof = ne * (args.p + 1) ** 3
    sec = t1 - t0
    stages = (5 if args.integrator == "ssprk54" else 4) * args.steps
    out = {
        "gdofs": dof * stages / sec / 1e9,
        "ms_per_step": 1e3 * sec / args.steps,
        "rhs_ms_avg": rhs_ms / max(rhs_count, 1),
        "rhs_count": rhs_count,
        "ke_end": diag["ke"],
        "nonfinite": diag["nonfinite"],
    }
    sd.close()
    return out


def large_bench(torch, W, args, steps=10):
    """The Re = 5000 Taylor-Green workloads at full size, 64^3 elements at
    p = 3 and 43^3 at p = 5 (about 17 M solution points each), both schemes,
    FP32, FP64 and BF16x3: GDOF/s per RK stage from the same timed RK4 steps
    as the headline (the convective step of each mesh)."""
    out = {}
    for nel, p in ((64, 3), (43, 5)):
        a = argparse.Namespace(**{**vars(args), "nel": nel, "p": p, "Re": 5000.0, "steps": steps, "warmup": 2,
                                  "eta_ip": 0.0, "integrator": "rk4"})
        U0 = W.tgv_state((nel,) * 3, p)
        h = 2 * math.pi / nel
        dt = 0.3 * h / ((p + 1) * (1.0 + math.sqrt(1.4 * (1.0 / 1.4 / 0.01))))
        rec = {}
        for scheme in ("compact", "br1"):
            a.scheme = scheme
            for precision in ("fp32", "fp64", "bf16x3"):
                r = run_path(torch, W, a, precision, U0, dt)
                rec[f"{scheme}_{precision}"] = {"value": r["gdofs"], "rhs_ms": r["rhs_ms_avg"]}
        out[f"tgv{nel}_p{p}"] = {"workload": f"TGV Re=5000 Ma=0.1 {nel}^3 hex p={p}",
                                 "dof": nel ** 3 * (p + 1) ** 3, "gdofs": rec}
        print(f"bench: {nel}^3 p={p} done", file=sys.stderr, flush=True)
    return out


def developed_state_bench(torch, W, args, U0, dt, t_dev=9.0):
    """Throughput on a developed flow: the workload's state advanced in FP32
    to t* = t_dev (near the enstrophy peak at Re = 1600), then the same timed
    RK4 steps as the headline on that state, FP32 and FP64; the Roe branches
    (and so the work) depend on the values, nothing else does."""
    from paper_2608_09615_amd import SD
    lo, hi = W.tgv_domain()
    nel = (args.nel,) * 3
    sd = SD(nel, args.p, scheme=args.scheme, physics="ns", precision="fp32", lo=lo, hi=hi, Re=args.Re, Ma=0.1,
            Pr=0.71, gamma=1.4)
    u = torch.from_numpy(U0).to("cuda")
    nst = int(math.ceil(t_dev / dt))
    t0 = time.perf_counter()
    for k in range(nst):
        sd.rk_step(u, t_dev / nst)
        if k % 2000 == 1999:
            torch.cuda.synchronize()
            print(f"bench: developed state t={(k + 1) * t_dev / nst:.2f}", file=sys.stderr, flush=True)
    d = sd.diagnostics(u)
    sd.close()
    wall = time.perf_counter() - t0
    Ud = u.cpu().numpy()
    out = {"t": t_dev, "steps_to_reach": nst, "wall_s_to_reach": wall, "ke": d["ke"], "enstrophy": d["enstrophy"]}
    for precision in ("fp32", "fp64"):
        r = run_path(torch, W, args, precision, Ud, dt)
        out[precision] = {"value": r["gdofs"], "ms_per_step": r["ms_per_step"], "rhs_ms": r["rhs_ms_avg"]}
    return out


def ke_error(torch, W, args, U0, dt, nsteps):
    """max_t |KE_fp32 - KE_fp64| / KE_fp64(0) over nsteps RK4 steps."""
    from paper_2608_09615_amd import SD
    lo, hi = W.tgv_domain()
    nel = (args.nel,) * 3
    hist = {}
    for precision in ("fp64", "fp32"):
        sd = SD(nel, args.p, scheme=args.scheme, physics="ns", precision=precision, lo=lo, hi=hi, Re=args.Re)
        u = torch.from_numpy(U0).to("cuda")
        h = [sd.diagnostics(u)["ke"]]
        for s in range(nsteps):
            sd.rk_step(u, dt)
            if (s + 1) % 10 == 0:
                h.append(sd.diagnostics(u)["ke"])
        hist[precision] = h
        sd.close()
    k64, k32 = hist["fp64"], hist["fp32"]
    return max(abs(a - b) for a, b in zip(k32, k64)) / k64[0], nsteps * dt


def cpu_baseline(W, args, U0, R_gpu64=None):
    """The FP64 oracle on the host cores: the same RHS on a sample of the
    workload's elements, with every host thread (at most 16) and with one
    thread.  With R_gpu64 (the GPU FP64 RHS of U0) the leg also states, per
    variable, the largest difference on the sampled elements relative to the
    oracle's largest value, and that figure over 1e-12."""
    import numpy as np
    from oracle import oracle as O
    lo, hi = W.tgv_domain()
    nel = (args.nel,) * 3
    ne = args.nel ** 3
    threads = min(os.cpu_count() or 1, 16)
    n = min(args.cpu_sample, ne)
    sel = np.arange(n, dtype=np.int64)
    prm = O.make_params("ns", Re=args.Re, Ma=0.1, Pr=0.71)

    # every FP64 evaluation carries the rounding of its input: the input moved
    # by about one ulp (seeded) gives the oracle's own sensitivity, evaluated
    # in alternate repetitions of the timed loop (same cost)
    U0p = U0 * (1.0 + 2.2e-16 * np.random.Generator(np.random.PCG64(1)).uniform(-1, 1, U0.shape))

    def timed(nthreads, elems, seconds):
        # repeated right-hand sides until about `seconds` of work (at least two)
        reps, out = 0, [None, None]
        t0 = time.perf_counter()
        while True:
            out[reps % 2] = O.rhs_3d_elems(U0 if reps % 2 == 0 else U0p, nel, lo, hi, args.p, args.scheme, prm,
                                           elems, nthreads=nthreads)
            reps += 1
            sec = time.perf_counter() - t0
            if reps >= 2 and (sec >= seconds or reps >= 100):
                return reps, sec, out

    reps, sec, (Ro, Rop) = timed(threads, sel, args.cpu_seconds)
    n1 = min(n, 4096)
    reps1, sec1, _ = timed(1, sel[:n1], max(2.0, args.cpu_seconds / 4))
    dof_el = (args.p + 1) ** 3
    out = {"value": reps * n * dof_el / sec / 1e9, "unit": "GDOF/s", "cores": threads, "kind": "oracle",
           "host": {"cpu_model": cpu_model(), "nproc": os.cpu_count()},
           "sample": f"{reps} RHS evaluations on the first {n} of {ne} elements of the same TGV state "
                     f"({sec:.1f} s wall, OpenMP over elements)",
           "single_thread": {"value": reps1 * n1 * dof_el / sec1 / 1e9, "unit": "GDOF/s", "cores": 1,
                             "sample": f"{reps1} RHS evaluations on the first {n1} elements ({sec1:.1f} s wall)"}}
    # the closure network's forward pass (320-128-128-320, BF16 roundings,
    # exact sums): the reference on one batch of the coarse mesh's elements
    from oracle import mlp as M
    nve = 5 * dof_el
    pm = M.init_params(nve, 128, nve, 0)
    xb = np.random.Generator(np.random.PCG64(5)).normal(size=(4096, nve))
    t0 = time.perf_counter()
    M.forward(pm, xb, bf16=True)
    tf = time.perf_counter() - t0
    out["closure_forward"] = {"value": 4096 / tf, "unit": "elements/s",
                              "sample": f"one forward pass of 4096 elements ({tf:.2f} s, numpy FP64, BLAS threads)"}
    if R_gpu64 is not None:
        Ro = np.asarray(Ro).reshape(n, 5, -1)
        Rop = np.asarray(Rop).reshape(n, 5, -1)
        Rg = np.asarray(R_gpu64).reshape(ne, 5, -1)[:n]
        scale = [float(np.abs(Ro[:, v]).max()) for v in range(5)]
        err = [float(np.abs(Rg[:, v] - Ro[:, v]).max()) / scale[v] for v in range(5)]
        sens = [float(np.abs(Rop[:, v] - Ro[:, v]).max()) / scale[v] for v in range(5)]
        out["fp64_parity"] = {
            "per_variable": err, "over_1e-12": [e / 1e-12 for e in err],
            "oracle_one_ulp_sensitivity": sens,
            "bar": [max(1e-12, 4.0 * x) for x in sens],
            "within_bar": all(e < max(1e-12, 4.0 * x) for e, x in zip(err, sens)),
            "sample": f"first {n} elements, the workload's initial state (max|R| per variable: "
                      + ", ".join(f"{x:.2e}" for x in scale) + ")"}
    return out


def cpu_model():
    """The host CPU's model name (Linux /proc/cpuinfo), or None."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def oned_bench(torch, args, p=3, N=16):
    """Whole run of the 1-D diffusion case (u_t = u_xx on [0, 2 pi], N
    elements, p = 3, u0 = sin x, RK4 with dt = 1 / ceil(1 / (0.05 h^2 /
    (p+1)^2)) to t = 1, both schemes, FP64) on the GPU and with the oracle
    on one host thread, and the error against exp(-t) sin x.  The case is
    64 solution points: run step by step, the GPU run is bound by its
    launches; sd_rk_run takes the whole run in one launch of one block."""
    import numpy as np
    from oracle import oracle as O
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd import workloads as W
    h = 2 * math.pi / N
    nst = int(math.ceil(1.0 / (0.05 * h * h / (p + 1) ** 2)))
    dt = 1.0 / nst
    x = W.points_1d(N, p, 0.0, 2 * math.pi)
    u0 = np.sin(x)
    out = {"config": f"1-D diffusion, {N} elements, p={p}, RK4 {nst} steps to t=1, FP64"}
    for scheme in ("compact", "br1"):
        sd = SD([N], p, scheme=scheme, physics="diffusion", precision="fp64", lo=[0.0], hi=[2 * math.pi], nu=1.0)
        u = torch.from_numpy(np.ascontiguousarray(u0[:, None, :])).to("cuda")
        sd.rk_step(u, dt)
        torch.cuda.synchronize()
        u.copy_(torch.from_numpy(np.ascontiguousarray(u0[:, None, :])))
        t0 = time.perf_counter()
        for _ in range(nst):
            sd.rk_step(u, dt)
        torch.cuda.synchronize()
        tg = time.perf_counter() - t0
        ug = u.cpu().numpy()[:, 0, :]
        # the same run with the steps replayed from a captured HIP graph
        # (256 steps per graph): the launches, not the kernels, bound it
        u.copy_(torch.from_numpy(np.ascontiguousarray(u0[:, None, :])))
        sd.rk_steps(u, dt, 257, graph_steps=256)
        torch.cuda.synchronize()
        u.copy_(torch.from_numpy(np.ascontiguousarray(u0[:, None, :])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sd.rk_steps(u, dt, nst, graph_steps=256)
        torch.cuda.synchronize()
        tgg = time.perf_counter() - t0
        ugg = u.cpu().numpy()[:, 0, :]
        # the whole run in one launch (sd_rk_run), after one warm-up run
        u.copy_(torch.from_numpy(np.ascontiguousarray(u0[:, None, :])))
        sd.rk_run(u, dt, nst)
        u.copy_(torch.from_numpy(np.ascontiguousarray(u0[:, None, :])))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sd.rk_run(u, dt, nst)
        torch.cuda.synchronize()
        tgr = time.perf_counter() - t0
        ugr = u.cpu().numpy()[:, 0, :]
        sd.close()
        t0 = time.perf_counter()
        uo = O.rk4_1d(u0, p, 0.0, 2 * math.pi, dt, nst, scheme=scheme)
        to = time.perf_counter() - t0
        ex = math.exp(-1.0) * np.sin(x)
        out[scheme] = {"gpu_s": tg, "gpu_graph_s": tgg, "graph_vs_eager": float(np.abs(ugg - ug).max()),
                       "gpu_one_launch_s": tgr, "one_launch_vs_eager": float(np.abs(ugr - ug).max()),
                       "oracle_1thread_s": to, "gpu_max_err": float(np.abs(ug - ex).max()),
                       "oracle_max_err": float(np.abs(uo - ex).max()),
                       "gpu_vs_oracle": float(np.abs(ug - uo).max())}
    return out


BLOCH_TIMES = (0.01, 0.1, 1.0)
BLOCH_TAYLOR_DEGREE = 18


def bloch_bench(torch, args, p=3, scheme="compact", reps=5):
    """Batched Bloch analysis (section 3, appendix): 2^16 wavenumbers in
    [0, pi], unit elements.  Times (a) B(theta) and its eigenvalues, (b) B and
    the combined mode at three times, (c) everything, with HIP events on the
    stream the kernel runs on.  Roofline of (b): every complex multiply-add is
    8 FP64 flops; per (theta, t) the Taylor polynomial and the squarings cost
    (18 + s) (p+1)^3 of them, s being the squarings the kernel takes
    (||B t||_1 / 2^s <= 1/2, recomputed here from the returned B), and
    building B about 2 (p+1)^3; the eigenvalue iteration is not counted."""
    import numpy as np
    from paper_2608_09615_amd.sd import bloch
    n = p + 1
    th = torch.linspace(0.0, math.pi, args.bloch_theta, dtype=torch.float64, device="cuda")
    t = torch.tensor(BLOCH_TIMES, dtype=torch.float64, device="cuda")
    B = bloch(p, scheme, th, None, eigs=False)["B"]
    norm1 = B.abs().sum(dim=1).max(dim=1).values.cpu().numpy()
    cmacs = 0.0
    for tv in BLOCH_TIMES:
        x = norm1 * tv
        sq = np.zeros_like(x)
        while np.any(x > 0.5):
            big = x > 0.5
            x[big] *= 0.5
            sq[big] += 1
        cmacs += float(np.sum(BLOCH_TAYLOR_DEGREE + sq)) * n ** 3
    cmacs += 2.0 * n ** 3 * args.bloch_theta
    stream = torch.cuda.current_stream()

    def timed(**kw):
        bloch(p, scheme, th, **kw)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            bloch(p, scheme, th, **kw)
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_eig = timed(t=None, matrices=False, eigs=True)
    ms_cm = timed(t=t, matrices=False, eigs=False)
    ms_all = timed(t=t, matrices=True, eigs=True)
    achieved = 8.0 * cmacs / (ms_cm * 1e-3) / 1e12
    return {"config": f"p={p} {scheme}, {args.bloch_theta} wavenumbers in [0, pi], J = 1/2, "
                      f"t = {', '.join(str(x) for x in BLOCH_TIMES)}",
            "mtheta_per_s": {"eigenvalues": args.bloch_theta / ms_eig / 1e3,
                             "combined_mode": args.bloch_theta / ms_cm / 1e3,
                             "all": args.bloch_theta / ms_all / 1e3},
            "ms": {"eigenvalues": ms_eig, "combined_mode": ms_cm, "all": ms_all},
            "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None,
                         "kernels": "k_bloch_lane_cm (combined mode)"}}


def curvilinear_bench(torch, args, reps=20, physics="diffusion", precision="fp64"):
    """Right-hand side on curvilinear hexahedra (degree-2 elements of a
    periodic box moved by a smooth wave of amplitude 0.3), FP64, one RHS per
    step: linear diffusion of a smooth field, or the Navier-Stokes equations
    of the Taylor-Green state at Re = 1600.  Roofline: HBM, with the
    algorithmic bytes per element the state in and the RHS out
    (2 x 8 nv n^3) plus the metric terms the kernels must read (S rows at
    3 (n+1) n^2 flux points, 1/det J at n^3 points: 8 (9 (n+1) n^2 + n^3))."""
    import numpy as np
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd import workloads as W
    N, p, scheme = args.curv_nel, args.curv_p, args.curv_scheme
    nel = (N,) * 3
    n = p + 1
    box = ((0.0, 0.0, 0.0), (2 * math.pi,) * 3)
    Xg = W.mesh_nodes(nel, *box, q=2, displacement=W.periodic_wave_displacement(0.3))
    if physics == "ns":
        nv = 5
        lo, hi = W.tgv_domain()
        sd = SD(nel, p, scheme=scheme, physics="ns", precision=precision, lo=lo, hi=hi, Re=1600.0, Ma=0.1,
                Pr=0.71)
        u = torch.from_numpy(W.perturbed_tgv_state(nel, p, seed=0)).to("cuda")
        what = "compressible Navier-Stokes (Taylor-Green state, Re=1600, Ma=0.1)"
        kernels = "k_cvn_traces + k_cvn_grad + k_cvn_face"
    else:
        nv = 1
        sd = SD(nel, p, scheme=scheme, physics="diffusion", precision=precision, lo=[0.0] * 3, hi=[1.0] * 3)
        x = W.map_points(Xg, p)
        u = torch.from_numpy(np.ascontiguousarray((np.sin(x[..., 0]) * np.sin(x[..., 1]) * np.sin(x[..., 2]))[:, None]))
        u = u.to("cuda")
        what = "linear diffusion"
        kernels = "k_cv_traces + k_cv_grad + k_cv_face"
    sd.set_geometry(Xg)
    out = torch.empty_like(u)
    for _ in range(3):
        sd.rhs(u, out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sd.rhs(u, out)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    sd.close()
    dof = N ** 3 * n ** 3
    # metric terms in the compute type (8 B in FP64, 4 B in FP32)
    mb = 8.0 if precision == "fp64" else 4.0
    bytes_el = 16.0 * nv * n ** 3 + mb * (9 * (n + 1) * n * n + n ** 3)
    gbs = bytes_el * N ** 3 / (ms * 1e-3) / 1e9
    return {"config": f"{what}, {N}^3 degree-2 hexahedra (periodic box, wave displacement 0.3), "
                      f"p={p} {scheme}, {precision.upper()}",
            "gdofs_per_rhs": dof / ms / 1e6, "ms_per_rhs": ms, "variables": nv,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS,
                         "traffic": curv_traffic(N, p, scheme, physics) if precision == "fp64" else None,
                         "traffic_unit": "B per RHS", "kernels": kernels}}


def closure_bench(torch, args, p=3, hidden=128, reps=200):
    """Cost of the learned closure inside the right-hand side: the compact
    FP32 Navier-Stokes RHS of the Taylor-Green state at Re = 5000 on N^3
    elements, p = 3, timed without and with the closure network
    (5 n^3 -> hidden -> hidden -> 5 n^3, GELU, seeded weights; the cost
    does not depend on their values).  The closure adds one launch per RHS
    (k_closure_fused); its figure is the difference of the two times, and
    the achieved rate is that of the network's matrix products in it."""
    from paper_2608_09615_amd import SD, workloads as W
    from paper_2608_09615_amd import closure as CL
    from paper_2608_09615_amd.sd import Mlp
    N = args.closure_nel
    nel = (N,) * 3
    nve = 5 * (p + 1) ** 3
    lo, hi = W.tgv_domain()
    u = torch.from_numpy(W.tgv_state(nel, p)).to("cuda")
    stream = torch.cuda.current_stream()
    us = {}
    for on in (False, True):
        sd = SD(nel, p, scheme="compact", physics="ns", precision="fp32", lo=lo, hi=hi, Re=5000.0)
        if on:
            net = Mlp(nve, hidden, nve, torch.from_numpy(CL.init_params_flat(nve, hidden, nve, seed=1)).to("cuda"))
            sd.closure_set(net, [1.0, 0.0, 0.0, 0.0, 178.57], [0.01, 0.5, 0.5, 0.5, 0.2], [1e-6] * 5, max_ratio=1.0)
        out = torch.empty_like(u)
        for _ in range(5):
            sd.rhs(u, out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            sd.rhs(u, out)
        e1.record(stream)
        torch.cuda.synchronize()
        us[on] = e0.elapsed_time(e1) / reps * 1e3
        if on:
            rejected = sd.closure_rejected()
        sd.close()
    extra = us[True] - us[False]
    flop = 2.0 * (nve * hidden + hidden * hidden + hidden * nve) * N ** 3
    # algorithmic HBM bytes of the launch: the state and R read, R written
    # (FP64), and the BF16 weights and FP32 biases once
    nbytes = 3 * 8.0 * nve * N ** 3 + 2.0 * (nve * hidden + hidden * hidden + hidden * nve) + 4.0 * (2 * hidden + nve)
    gbs = nbytes / (extra * 1e-6) / 1e9
    return {"config": f"compact NS RHS, TGV state, {N}^3 elements, p={p}, FP32, Re=5000; network "
                      f"{nve}-{hidden}-{hidden}-{nve} GELU on BF16 matrix cores",
            "us_per_rhs": us[False], "us_per_rhs_with_closure": us[True], "closure_us": extra,
            "closure_tflops": flop / (extra * 1e-6) / 1e12, "rejected_elements": rejected,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                         "frac": gbs / PEAK_HBM_GBS, "traffic": closure_traffic(N, p, hidden),
                         "traffic_unit": "B per launch", "algorithmic_bytes": nbytes, "kernels": "k_closure_fused",
                         "mfma_frac_bf16": flop / (extra * 1e-6) / 1e12 / PEAK_BF16_TFLOPS,
                         "duration": "closure_us (RHS time with the closure minus without)"}}


def training_bench(torch, args, p=3, hidden=128, batch=1024, steps=200):
    """One training step of the closure network (5 n^3 -> hidden -> hidden ->
    5 n^3, GELU) on seeded random data, all on the library's kernels:
    forward (BF16 matrix cores), MSE gradient, backward (FP32 matrix cores) and Adam,
    batch 1024, timed over ``steps`` steps with HIP events (host launch gaps
    included).  Algorithmic flops per step: the forward products
    2 B (n_in h + h h + h n_out), the weight gradients as many, and the
    products back to the two hidden layers' inputs 2 B (n_out h + h h)."""
    import numpy as np
    from paper_2608_09615_amd.sd import Mlp, mse
    from paper_2608_09615_amd.closure import init_params_flat
    nve = 5 * (p + 1) ** 3
    rng = np.random.Generator(np.random.PCG64(3))
    X = torch.from_numpy(rng.normal(size=(batch, nve)).astype(np.float32)).to("cuda")
    T = torch.from_numpy(rng.normal(size=(batch, nve)).astype(np.float32)).to("cuda")
    net = Mlp(nve, hidden, nve, P=torch.from_numpy(init_params_flat(nve, hidden, nve, 0)).to("cuda"))
    dY = torch.empty((batch, nve), dtype=torch.float32, device="cuda")

    def step():
        # the loss itself is reduced only when reported (as in the training loop)
        Y = net.forward(X)
        mse(Y, T, dY, None)
        net.backward(dY)
        net.adam(1e-4)
    for _ in range(5):
        step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / steps * 1e3
    fwd = 2.0 * batch * (nve * hidden + hidden * hidden + hidden * nve)
    flop = 2 * fwd + 2.0 * batch * (nve * hidden + hidden * hidden)
    tf = flop / (us * 1e-6) / 1e12
    return {"config": f"closure network {nve}-{hidden}-{hidden}-{nve} GELU, batch {batch}, forward + MSE + "
                      f"backward + Adam", "us_per_step": us, "steps_per_s": 1e6 / us, "flop_per_step": flop,
            "tflops": tf, "frac_fp32_mfma": tf / PEAK_FP32_MFMA_TFLOPS}


def closure_record():
    """The trained closure's errors and speedup on the held-out seed(s) of the
    64^3 -> 16^3 case (profiles/closure_64to16_p3_*seed*.json, written by
    paper_2608_09615_amd.closure; the command is in each record)."""
    import glob
    out = []
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "closure_64to16_p3_*seed*.json"))):
        with open(path) as f:
            rec = json.load(f)
        post = rec["a_posteriori"]
        trained = rec["config"].get("trained_with") or rec["config"]
        out.append({"record": os.path.relpath(path, ROOT), "test_seed": rec["config"]["test_seed"],
                    "train_seeds": trained["train_seeds"],
                    "target": rec["config"]["target"], "dt_snap": rec["config"]["dt_snap"],
                    "a_priori_ratio": rec["a_priori"]["ratio"],
                    "ke_err": {k: post[k]["ke_err"] for k in ("plain", "closure")},
                    "ens_err": {k: post[k]["ens_err"] for k in ("plain", "closure")},
                    "wall_s": {"fine": post["wall_fine_s"], "plain": post["plain"]["wall_s"],
                               "closure": post["closure"]["wall_s"]},
                    "speedup_vs_fine": rec.get("speedup_vs_fine")})
    return out


def closure_traffic(N, p, hidden):
    """HBM bytes per k_closure_fused launch from the committed counter
    record, or None for another workload or once a source it is keyed to
    has changed."""
    path = os.path.join(ROOT, "profiles", "closure_traffic_16cubed_p3.json")
    if not (N == 16 and p == 3 and hidden == 128 and os.path.exists(path)):
        return None
    with open(path) as f:
        rec = json.load(f)
    if sources_sha256(CLOSURE_TRAFFIC_SOURCES) != rec["sources_sha256"]:
        return None
    return rec["bytes_per_launch"]


def curv_traffic(N, p, scheme, physics="diffusion"):
    """HBM bytes per curvilinear RHS from the committed counter record, or
    None for another workload or once a source it is keyed to has changed."""
    name = "curv_traffic_32cubed_p3.json" if physics == "diffusion" else "curv_ns_traffic_32cubed_p3.json"
    path = os.path.join(ROOT, "profiles", name)
    if not (N == 32 and p == 3 and scheme == "compact" and os.path.exists(path)):
        return None
    with open(path) as f:
        rec = json.load(f)
    if sources_sha256(CURV_TRAFFIC_SOURCES) != rec["sources_sha256"]:
        return None
    return rec["bytes_per_rhs"]


def fp64_rhs(torch, args, U0):
    """One FP64 right-hand side of the workload's initial state (host copy)."""
    from paper_2608_09615_amd import SD
    from paper_2608_09615_amd import workloads as W
    lo, hi = W.tgv_domain()
    sd = SD((args.nel,) * 3, args.p, scheme=args.scheme, physics="ns", precision="fp64", lo=lo, hi=hi,
            Re=args.Re, Ma=0.1, Pr=0.71, gamma=1.4, eta_ip=args.eta_ip)
    R = sd.rhs(torch.from_numpy(U0).to("cuda")).cpu().numpy()
    sd.close()
    return R


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the right-hand side is "
              "not sharded across GPUs.", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2608_09615_amd import workloads as W
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib * (1 << 18), dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"bench: copy probe {args.copy_probe_mib} MiB", file=sys.stderr, flush=True)
        del src, dst
    if args.only == "bloch":
        print(json.dumps({"bloch": bloch_bench(torch, args)}), flush=True)
        return
    if args.only == "curvilinear":
        print(json.dumps({"curvilinear": curvilinear_bench(torch, args, precision=args.curv_precision)}), flush=True)
        return
    if args.only == "curvilinear_ns":
        print(json.dumps({"curvilinear_ns": curvilinear_bench(torch, args, physics="ns",
                                                              precision=args.curv_precision)}), flush=True)
        return
    if args.only == "closure":
        print(json.dumps({"closure": closure_bench(torch, args)}), flush=True)
        return
    if args.only == "training":
        print(json.dumps({"closure_training": training_bench(torch, args)}), flush=True)
        return
    if args.only == "oned":
        print(json.dumps({"oned_whole_run": oned_bench(torch, args)}), flush=True)
        return
    nel = (args.nel,) * 3
    U0 = W.tgv_state(nel, args.p)
    h = 2 * math.pi / args.nel
    c0 = math.sqrt(1.4 * (1.0 / 1.4 / 0.01) / 1.0)
    dt = 0.3 * h / ((args.p + 1) * (1.0 + c0))
    print(f"bench: TGV {nel} p={args.p} {args.scheme} dt={dt:.3e}", file=sys.stderr, flush=True)
    precs = args.precisions.split(",")
    r32 = run_path(torch, W, args, "fp32", U0, dt) if "fp32" in precs else None
    if r32:
        print(f"bench: fp32 {r32['gdofs']:.2f} GDOF/s", file=sys.stderr, flush=True)
    r64 = run_path(torch, W, args, "fp64", U0, dt) if "fp64" in precs else None
    if r64:
        print(f"bench: fp64 {r64['gdofs']:.2f} GDOF/s", file=sys.stderr, flush=True)
    rbf = run_path(torch, W, args, "bf16x3", U0, dt) if "bf16x3" in precs else None
    if rbf:
        print(f"bench: bf16x3 {rbf['gdofs']:.2f} GDOF/s", file=sys.stderr, flush=True)
    rfm = run_path(torch, W, args, "fp32mfma", U0, dt) if "fp32mfma" in precs else None
    if rfm:
        print(f"bench: fp32mfma {rfm['gdofs']:.2f} GDOF/s", file=sys.stderr, flush=True)
    if r32 is None or r64 is None:
        return
    # the headline FP32 figure is the faster of the two FP32 variants
    best32, path32 = (rfm, "matrix cores (fp32mfma)") if rfm and rfm["gdofs"] > r32["gdofs"] else (r32, "vector")
    kerr, tke = ke_error(torch, W, args, U0, dt, args.ke_steps) if args.ke_steps > 0 else (None, 0.0)
    dof = args.nel ** 3 * (args.p + 1) ** 3
    flop = FLOP_PER_DOF.get(args.p, 1430.0) * dof

    def roof(r, peak_flops, name, precision):
        t = r["rhs_ms_avg"] * 1e-3
        traffic = measured_traffic(args, precision)
        alu = flop / t / 1e12
        hbm = BYTES_PER_DOF * dof / t / 1e9
        # binding ceiling: the lower of the ALU and HBM rooflines for this path
        ceil_alu = peak_flops * 1e12 / FLOP_PER_DOF.get(args.p, 1430.0)
        ceil_hbm = PEAK_HBM_GBS * 1e9 / BYTES_PER_DOF
        if ceil_alu <= ceil_hbm:
            return {"bound": "alu", "achieved": alu, "peak": peak_flops, "unit": "TFLOP/s",
                    "frac": alu / peak_flops, "traffic": traffic, "traffic_unit": "B per RK stage", "kernels": name,
                    "rhs_ms": r["rhs_ms_avg"], "hbm_gbs_algorithmic": hbm}
        return {"bound": "hbm", "achieved": hbm, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": hbm / PEAK_HBM_GBS, "traffic": traffic, "traffic_unit": "B per RK stage", "kernels": name,
                "rhs_ms": r["rhs_ms_avg"], "tflops_algorithmic": alu}

    rec = {
        "metric": "SD RHS GDOF/s per RK stage",
        "value": best32["gdofs"],
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": best32["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"TGV Re={args.Re:g} Ma=0.1 {args.nel}^3 hex p={args.p} {args.scheme}"
                               + (f" eta_ip={args.eta_ip:g}" if args.eta_ip else ""),
                   "dof": dof,
                   "step": ("one SSP-RK(5,4) step = 5 RHS + 5 FP64 stage combinations" if args.integrator == "ssprk54"
                            else "one RK4 step = 4 RHS + 4 FP64 stage updates"),
                   "fp32_path": path32,
                   "ke_error_fp32_vs_fp64": kerr, "ke_error_t_end": tke,
                   "ke_error_t20": ke_record(args)},
        "roofline": roof(best32, PEAK_FP32_TFLOPS, "k_rhs_ns", "fp32mfma" if best32 is rfm else "fp32"),
        "fp32_vector": {"value": r32["gdofs"], "ms_per_step": r32["ms_per_step"], "dtype": "f32",
                        "roofline": roof(r32, PEAK_FP32_TFLOPS, "k_rhs_ns", "fp32")},
        "fp64": {"value": r64["gdofs"], "ms_per_step": r64["ms_per_step"], "dtype": "f64",
                 "roofline": roof(r64, PEAK_FP64_TFLOPS, "k_rhs_ns", "fp64")},
    }
    if rfm:
        rec["fp32_mfma"] = {"value": rfm["gdofs"], "ms_per_step": rfm["ms_per_step"], "dtype": "f32",
                            "roofline": roof(rfm, PEAK_FP32_TFLOPS, "k_rhs_ns", "fp32mfma"),
                            "mfma": mfma_use(args, "fp32mfma", rfm["rhs_ms_avg"])}
    if rbf:
        rec["bf16x3"] = {"value": rbf["gdofs"], "ms_per_step": rbf["ms_per_step"], "dtype": "f32+bf16x3",
                         "roofline": roof(rbf, PEAK_FP32_TFLOPS, "k_rhs_ns", "bf16x3"),
                         "mfma": mfma_use(args, "bf16x3", rbf["rhs_ms_avg"])}
    if args.developed:
        rec["developed_state"] = developed_state_bench(torch, W, args, U0, dt)

    if args.large:
        rec["large"] = large_bench(torch, W, args)
    if args.bloch_theta > 0:
        rec["bloch"] = bloch_bench(torch, args)
    if args.curv_nel > 0:
        rec["curvilinear"] = curvilinear_bench(torch, args)
        rec["curvilinear_ns"] = curvilinear_bench(torch, args, physics="ns")
        rec["curvilinear"]["fp32"] = curvilinear_bench(torch, args, precision="fp32")
        rec["curvilinear_ns"]["fp32"] = curvilinear_bench(torch, args, physics="ns", precision="fp32")
    if args.closure_nel > 0:
        rec["closure"] = closure_bench(torch, args)
        rec["closure"]["a_posteriori_64to16"] = closure_record()
        rec["closure_training"] = training_bench(torch, args)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(W, args, U0, fp64_rhs(torch, args, U0))
        rec["cpu_baseline"]["oned_whole_run"] = oned_bench(torch, args)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
