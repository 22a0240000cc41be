"""Taylor-Green vortex runs on the GPU: kinetic-energy and enstrophy
histories of one discretisation, and the error of one precision against
another (the FP64 path is the reference of the FP32 and BF16x3 ones).

    python -m paper_2608_09615_amd.tgv --nel 32 --p 3 --t-end 20 --precisions fp64,fp32,bf16x3,fp32mfma \
        --record profiles/ke_history_tgv32p3.json

The state is the compressible TGV (Ma = 0.1, gamma = 1.4, Pr = 0.71) on the
periodic box [0, 2 pi]^3; every run takes RK steps of equal size, dt_out / k
with the smallest k that keeps dt below 0.3 h / ((p + 1)(1 + c0)).  With
``--cfl`` the step adapts instead: each output interval takes the smallest k
that keeps dt below the library's convective limit cfl h / ((p + 1) max(|u| + c))
of the state at its start.
"""
import json
import math
import time

from . import workloads as W
from .sd import SD


def step_size(nel, p, dt_out, Ma=0.1, cfl=0.3):
    h = 2 * math.pi / nel
    c0 = 1.0 / Ma
    dt_max = cfl * h / ((p + 1) * (1.0 + c0))
    k = max(1, math.ceil(dt_out / dt_max - 1e-12))
    return dt_out / k, k


class NonFiniteState(FloatingPointError):
    """The state turned non-finite; t is the first output time that saw it."""

    def __init__(self, msg, t):
        super().__init__(msg)
        self.t = t


def history(nel, p, scheme="compact", precision="fp64", Re=1600.0, t_end=20.0, dt_out=0.1, log=print,
            integrator="rk4", cfl=None):
    """KE and enstrophy every dt_out up to t_end, and the wall time of the
    stepping (diagnostics included)."""
    import torch
    lo, hi = W.tgv_domain()
    sd = SD((nel,) * 3, p, scheme=scheme, physics="ns", precision=precision, lo=lo, hi=hi, Re=Re, Ma=0.1, Pr=0.71,
            integrator=integrator)
    u = torch.from_numpy(W.tgv_state((nel,) * 3, p)).to("cuda")
    dt, k = step_size(nel, p, dt_out)
    nout = int(round(t_end / dt_out))
    d = sd.diagnostics(u)
    t, ke, ens = [0.0], [d["ke"]], [d["enstrophy"]]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    steps = 0
    for i in range(1, nout + 1):
        if cfl is not None:
            k = max(1, math.ceil(dt_out / sd.stable_dt(u, cfl) - 1e-12))
            dt = dt_out / k
        for _ in range(k):
            sd.rk_step(u, dt)
        steps += k
        d = sd.diagnostics(u)
        if d["nonfinite"]:
            raise NonFiniteState(f"{precision} run turned non-finite before t={i * dt_out:.2f}", i * dt_out)
        t.append(i * dt_out)
        ke.append(d["ke"])
        ens.append(d["enstrophy"])
        if i % int(round(1.0 / dt_out)) == 0:
            log(f"tgv: {precision} {scheme} {nel}^3 p={p} t={i * dt_out:.1f} KE={d['ke']:.6f} "
                f"enstrophy={d['enstrophy']:.4f} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sd.close()
    return {"nel": nel, "p": p, "scheme": scheme, "precision": precision, "Re": Re, "integrator": integrator,
            "dt": dt, "cfl": cfl, "steps": steps,
            "t": t, "ke": ke, "enstrophy": ens, "wall_s": wall}


def compare(run, ref):
    """max_t |KE - KE_ref| / KE_ref(0) and max_t |ens - ens_ref| / max_t ens_ref."""
    ke = max(abs(a - b) for a, b in zip(run["ke"], ref["ke"])) / ref["ke"][0]
    ens = max(abs(a - b) for a, b in zip(run["enstrophy"], ref["enstrophy"])) / max(ref["enstrophy"])
    return {"ke_err": ke, "enstrophy_err": ens}


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="TGV kinetic-energy / enstrophy histories")
    ap.add_argument("--nel", type=int, default=32)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--scheme", default="compact")
    ap.add_argument("--Re", type=float, default=1600.0)
    ap.add_argument("--t-end", type=float, default=20.0)
    ap.add_argument("--dt-out", type=float, default=0.1)
    ap.add_argument("--precisions", default="fp64,fp32", help="the first one is the reference")
    ap.add_argument("--integrator", default="rk4", choices=["rk4", "ssprk54"])
    ap.add_argument("--cfl", type=float, default=None, help="adaptive step with this Courant number")
    ap.add_argument("--out", default=None, help="JSON file with every run's full histories")
    ap.add_argument("--record", default=None,
                    help="JSON record keyed to the kernel sources: the errors against the first precision, "
                         "the histories every 0.5 and the wall times")
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)
    runs = [history(a.nel, a.p, a.scheme, pr, a.Re, a.t_end, a.dt_out, log, a.integrator, a.cfl)
            for pr in a.precisions.split(",")]
    res = {"runs": runs, "errors": {r["precision"]: compare(r, runs[0]) for r in runs[1:]}}
    for r in runs[1:]:
        log(f"tgv: {r['precision']} vs {runs[0]['precision']}: {json.dumps(res['errors'][r['precision']])}")
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)
    if a.record:
        from .build import NS_RHS_SOURCES, sources_sha256
        every = max(1, int(round(0.5 / a.dt_out)))
        cmd = ("python -m paper_2608_09615_amd.tgv " + " ".join(argv if argv is not None else __import__("sys").argv[1:]))
        rec = {"workload": f"TGV Re={a.Re:g} Ma=0.1 {a.nel}^3 hex p={a.p} {a.scheme}, {a.integrator}",
               "t_end": a.t_end, "dt_out": a.dt_out, "command": cmd,
               "reference": runs[0]["precision"],
               "errors": res["errors"],
               "error_definition": "ke_err = max_t |KE - KE_ref| / KE_ref(0); enstrophy_err = max_t |ens - ens_ref| "
                                   "/ max_t ens_ref; t every dt_out up to t_end",
               "sources": NS_RHS_SOURCES, "sources_sha256": sources_sha256(NS_RHS_SOURCES),
               "runs": {r["precision"]: {"dt": r["dt"], "steps": r["steps"], "wall_s": r["wall_s"],
                                         "t": r["t"][::every], "ke": r["ke"][::every],
                                         "enstrophy": r["enstrophy"][::every]} for r in runs}}
        with open(a.record, "w") as f:
            json.dump(rec, f, indent=1)


if __name__ == "__main__":
    main()
