"""Learned closure of the coarse-grid SD residual (Taylor-Green vortex).

Pipeline (every numerical step of the method and of the network runs in the
library's HIP kernels; torch only holds device memory, numpy only reorders,
scales and scores samples on the host):
  1. fine runs: the plain compact scheme on ``nel_f``^3 elements from seeded,
     phase-shifted, randomly perturbed TGV initial conditions, snapshots
     every ``dt_snap``;
  2. training pairs per snapshot: the filtered state U_c = P_c U_f (L2
     projection onto the coarse elements, ``sd_filter``) and the residual
     target P_c R_f(U_f) - R_c(U_c), i.e. what the coarse right-hand side
     misses of the filtered fine one;
  3. the pairs are multiplied by symmetries of the cube (axis permutations
     and reflections, with the momentum components moved alike): the
     discretisation on a uniform Cartesian mesh commutes with them, so each
     image is again an exact pair;
  4. a per-element MLP (5 n^3 -> h -> h -> 5 n^3, GELU) trained with MSE and
     Adam on normalised pairs (``sd_mlp_*``);
  5. evaluation on a held-out seed: the correction error per snapshot (a
     priori) and coarse runs with and without the closure against the
     filtered fine run (kinetic energy and enstrophy histories, a
     posteriori), with the plain scheme as fallback: an interval in which the
     corrected run turns non-finite or gains kinetic energy is run again
     without the closure.
"""
import itertools
import json
import math
import time

import numpy as np

from . import workloads as W
from .sd import SD, Mlp, filter_state, mse


def cfl_dt(nel, p, Ma=0.1, cfl=0.3):
    h = 2 * math.pi / nel
    c0 = math.sqrt(1.4 * (1.0 / 1.4 / Ma ** 2))
    return cfl * h / ((p + 1) * (1.0 + c0))


# (perm, flips): new direction d is old direction perm[d], reversed if flips[d]
SYMMETRIES = [(perm, flips) for perm in itertools.permutations(range(3))
              for flips in itertools.product((False, True), repeat=3)]


def apply_symmetry(A, n, sym, lead=1):
    """Image of per-element NS data under a cube symmetry.

    ``A`` has ``lead`` leading axes that the map leaves alone (samples), then
    either [5 n^3] or [5][n][n][n] values in the layout u[v][k][j][i]
    (i along x).  With ``lead`` = 4 and leading axes (samples, ez, ey, ex) a
    whole periodic field on a cubic element grid is mapped, elements
    included.  Momentum component d of the image is +-component perm[d]."""
    perm, flips = sym
    shp = A.shape
    a = A.reshape(shp[:lead] + (5, n, n, n))
    nl = lead
    ax = list(range(nl + 4))
    # array axis of direction d among the points: nl + 3 - d; among the
    # elements (lead = 4): 3 - d
    for d in range(3):
        ax[nl + 3 - d] = nl + 3 - perm[d]
        if lead == 4:
            ax[3 - d] = 3 - perm[d]
    b = a.transpose(ax)
    idx = [slice(None)] * (nl + 4)
    idx[nl] = [0, 1 + perm[0], 1 + perm[1], 1 + perm[2], 4]
    b = b[tuple(idx)]
    for d in range(3):
        if flips[d]:
            b = np.flip(b, axis=nl + 3 - d)
            if lead == 4:
                b = np.flip(b, axis=3 - d)
            sel = [slice(None)] * (nl + 4)
            sel[nl] = 1 + d
            b[tuple(sel)] *= -1
    return np.ascontiguousarray(b).reshape(shp)


def augment(X, T, n, k, seed, extra=None):
    """Each sample and k - 1 distinct random images of it under the cube
    symmetries (k <= 48), sample-major; ``extra`` (per-sample values that the
    symmetries leave alone) is repeated alongside."""
    if k <= 1:
        return (X, T) if extra is None else (X, T, extra)
    rng = np.random.Generator(np.random.PCG64(seed))
    N = X.shape[0]
    pick = np.argsort(rng.random((N, len(SYMMETRIES) - 1)), axis=1)[:, :k - 1] + 1
    choice = np.concatenate([np.zeros((N, 1), dtype=pick.dtype), pick], axis=1)
    Xa = np.empty((N * k,) + X.shape[1:], X.dtype)
    Ta = np.empty((N * k,) + T.shape[1:], T.dtype)
    for s, sym in enumerate(SYMMETRIES):
        rows, slot = np.nonzero(choice == s)
        if rows.size:
            Xa[rows * k + slot] = apply_symmetry(X[rows], n, sym)
            Ta[rows * k + slot] = apply_symmetry(T[rows], n, sym)
    return (Xa, Ta) if extra is None else (Xa, Ta, np.repeat(extra, k, axis=0))


class Problem:
    def __init__(self, nel_f=64, ratio=4, p=3, Re=5000.0, precision="fp32", scheme="compact"):
        self.nel_f, self.ratio, self.p, self.Re = nel_f, ratio, p, Re
        self.nel_c = nel_f // ratio
        self.precision, self.scheme = precision, scheme
        lo, hi = W.tgv_domain()
        kw = dict(scheme=scheme, physics="ns", precision=precision, lo=lo, hi=hi, Re=Re, Ma=0.1, Pr=0.71)
        self.fine = SD((nel_f,) * 3, p, **kw)
        self.coarse = SD((self.nel_c,) * 3, p, **kw)
        self.dt_f = cfl_dt(nel_f, p)
        self.dt_c = cfl_dt(self.nel_c, p)
        self.n = p + 1
        self.nve = 5 * self.n ** 3

    def filt(self, Uf):
        return filter_state(Uf, (self.nel_f,) * 3, self.ratio, self.p, 5)

    def pair(self, Uf):
        """(U_c, target) for one fine snapshot as host FP64 arrays
        [n_el_c, 5 n^3]: the filtered state and P_c R_f(U_f) - R_c(U_c)."""
        Rf = self.fine.rhs(Uf)
        Uc = self.filt(Uf)
        PRf = self.filt(Rf).cpu().numpy()
        Rc = self.coarse.rhs(Uc).cpu().numpy()
        return Uc.cpu().numpy().reshape(-1, self.nve), (PRf - Rc).reshape(-1, self.nve)

    def initial(self, torch, seed):
        return torch.from_numpy(W.perturbed_tgv_state((self.nel_f,) * 3, self.p, seed=seed)).to("cuda")

    def fine_run(self, torch, seed, t_end, dt_snap, each, log=None):
        """Fine run of one seed; ``each(t, U_f)`` at t = 0 and every dt_snap;
        ``log`` gets a progress line every two time units."""
        U = self.initial(torch, seed)
        nsub = max(1, round(dt_snap / self.dt_f))
        dt = dt_snap / nsub
        each(0.0, U)
        for s in range(1, int(round(t_end / dt_snap)) + 1):
            for _ in range(nsub):
                self.fine.rk_step(U, dt)
            each(s * dt_snap, U)
            if log and abs(s * dt_snap / 2.0 - round(s * dt_snap / 2.0)) < 1e-9:
                log(f"closure: fine run seed {seed} at t={s * dt_snap:.2f}")
        return U


def interval_targets(torch, prob, Uc, dt_snap):
    """Trajectory defects of the coarse scheme over the snapshot intervals:
    for consecutive filtered fine states Uc[k], Uc[k+1] (host FP64
    [n_el_c, 5 n^3]) the target of Uc[k] is (Uc[k+1] - Phi(Uc[k])) / dt_snap,
    Phi the plain coarse scheme over one interval (RK4 steps of the coarse
    step size).  A closure that adds it to the coarse right-hand side keeps
    the coarse run on the filtered fine trajectory to first order in the
    interval, and the averaging over the interval removes the part of the
    instantaneous defect that the coarse state cannot predict."""
    ncc = max(1, round(dt_snap / prob.dt_c))
    dtc = dt_snap / ncc
    X, T = [], []
    for k in range(len(Uc) - 1):
        U = torch.from_numpy(Uc[k].reshape((prob.coarse.ne, 5) + (prob.n,) * 3)).to("cuda")
        for _ in range(ncc):
            prob.coarse.rk_step(U, dtc)
        X.append(Uc[k])
        T.append((Uc[k + 1] - U.cpu().numpy().reshape(Uc[k].shape)) / dt_snap)
    return X, T


def generate(torch, prob, seeds, t_end, dt_snap, log=print, target="rhs"):
    """Training pairs from fine runs: host FP64 arrays X, T [samples, 5 n^3]
    and the snapshot number of every sample.  target "rhs": the residual
    defect P_c R_f(U_f) - R_c(P_c U_f) at every snapshot t > 0; "interval":
    the coarse scheme's trajectory defect over each snapshot interval
    (interval_targets), from t = 0."""
    X, T, S = [], [], []
    for seed in seeds:
        t0 = time.perf_counter()
        Uc = []

        def each(t, U):
            if target == "interval":
                Uc.append(prob.filt(U).cpu().numpy().reshape(-1, prob.nve))
            elif t > 0:
                x, y = prob.pair(U)
                S.append(np.full(x.shape[0], len(X)))
                X.append(x)
                T.append(y)
        prob.fine_run(torch, seed, t_end, dt_snap, each, log=log)
        if target == "interval":
            xs, ts = interval_targets(torch, prob, Uc, dt_snap)
            for x, y in zip(xs, ts):
                S.append(np.full(x.shape[0], len(X)))
                X.append(x)
                T.append(y)
        log(f"closure: fine run seed {seed} to t={t_end:.2f} in {time.perf_counter() - t0:.1f} s")
    return np.concatenate(X), np.concatenate(T), np.concatenate(S)


def snapshot_weights(T, snap, out_scale, power=0.5):
    """Per-sample loss weights (mean 1): 1 / m_s^power with m_s the mean square
    of the normalised targets of the sample's snapshot, so that the nearly
    resolved early snapshots, whose targets are orders of magnitude smaller,
    still bound the network's output there."""
    os_ = np.repeat(out_scale, T.shape[1] // 5)[None, :]
    ns = int(snap.max()) + 1
    ms = np.zeros(ns)
    cnt = np.bincount(snap, minlength=ns)
    for b in range(0, T.shape[0], 65536):
        np.add.at(ms, snap[b:b + 65536], ((T[b:b + 65536] / os_) ** 2).mean(axis=1))
    ms /= np.maximum(cnt, 1)
    w = 1.0 / np.maximum(ms[snap], 1e-300) ** power
    return w / w.mean()


def normalisation(X, T, nve):
    """Per-variable shift/scale of inputs and scale of targets."""
    xs = X.reshape(-1, 5, nve // 5)
    ts = T.reshape(-1, 5, nve // 5)
    shift = xs.mean(axis=(0, 2))
    scale = xs.std(axis=(0, 2)) + 1e-12
    out_scale = ts.std(axis=(0, 2)) + 1e-30
    return shift, scale, out_scale


def normalise(X, T, shift, scale, out_scale, nve):
    """Normalised FP32 host arrays [samples, nve] (chunked)."""
    sh, sc, os_ = (np.repeat(a, nve // 5)[None, :] for a in (shift, scale, out_scale))
    Xn = np.empty(X.shape, np.float32)
    Tn = np.empty(T.shape, np.float32)
    for b in range(0, X.shape[0], 65536):
        Xn[b:b + 65536] = (X[b:b + 65536] - sh) / sc
        Tn[b:b + 65536] = T[b:b + 65536] / os_
    return Xn, Tn


def init_params_flat(n_in, n_h, n_out, seed):
    """Seeded uniform fan-in initialisation, layout of sd_closure.h."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for (o, i) in ((n_h, n_in), (n_h, n_h), (n_out, n_h)):
        lim = 1.0 / math.sqrt(i)
        parts.append(rng.uniform(-lim, lim, o * i))
        parts.append(np.zeros(o))
    return np.concatenate(parts).astype(np.float32)


def fit(torch, Xn, Tn, hidden=128, iters=3000, batch=1024, lr=1e-3, seed=0, weights=None, log=print):
    """Adam on the (sample-weighted) MSE of the normalised targets with the library's kernels;
    batches are consecutive slices of a host-drawn permutation of the samples,
    the learning rate decays geometrically to lr / 10."""
    nve = Xn.shape[1]
    net = Mlp(nve, hidden, nve, P=torch.from_numpy(init_params_flat(nve, hidden, nve, seed)).to("cuda"))
    N = Xn.shape[0]
    perm = np.random.Generator(np.random.PCG64(seed + 1)).permutation(N)
    Xs = torch.from_numpy(Xn[perm]).to("cuda")
    Ts = torch.from_numpy(Tn[perm]).to("cuda")
    Ws = None if weights is None else torch.from_numpy(weights[perm].astype(np.float32)).to("cuda")
    nb = max(1, N // batch)
    dY = torch.empty((batch, nve), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    t0 = time.perf_counter()
    for it in range(iters):
        b = it % nb
        sl = slice(b * batch, (b + 1) * batch)
        xb, tb = Xs[sl], Ts[sl]
        Y = net.forward(xb)
        report = it % 1000 == 0 or it == iters - 1
        mse(Y, tb, dY[:xb.shape[0]], loss if report else None, w=None if Ws is None else Ws[sl])
        net.backward(dY[:xb.shape[0]])
        net.adam(lr * (0.1 ** (it / iters)))
        if report:
            losses.append((it, loss.item()))
            log(f"closure: iter {it} loss {losses[-1][1]:.4e} ({time.perf_counter() - t0:.1f} s)")
    return net, losses


def a_priori(torch, net, Xn, Tn, batch=4096):
    """L2 norms of the (normalised) targets without and with the network's
    correction: ||T|| and ||T - net(X)||."""
    num0 = num1 = 0.0
    for b in range(0, Xn.shape[0], batch):
        Y = net.forward(torch.from_numpy(np.ascontiguousarray(Xn[b:b + batch])).to("cuda")).cpu().numpy()
        t = Tn[b:b + batch].astype(np.float64)
        num0 += float((t ** 2).sum())
        num1 += float(((t - Y) ** 2).sum())
    return math.sqrt(num0), math.sqrt(num1)


# (name, max_ratio, ke_tol) of the corrected coarse runs evaluated by default
VARIANTS = [("closure", 1.0, 1e-3)]


def evaluate(torch, prob, seed, t_end, dt_snap, net, norm, variants=VARIANTS, log=print, target="rhs"):
    """Held-out seed: one fine run gives the filtered reference history and
    the a-priori pairs; then the coarse runs, plain and with the closure for
    each (name, max_ratio, ke_tol) of ``variants``: max_ratio bounds each
    element's correction against its residual (sd_closure_set), and an
    interval in which the kinetic energy grows by more than the factor
    1 + ke_tol (or the state turns non-finite) is run again without it."""
    shift, scale, out_scale = (np.asarray(a) for a in norm)
    ref, apri = [], []
    t0 = time.perf_counter()

    Ucs = []

    def each(t, U):
        Uc = prob.filt(U)
        ref.append(prob.coarse.diagnostics(Uc))
        if target == "interval":
            Ucs.append(Uc.cpu().numpy().reshape(-1, prob.nve))
        elif t > 0:
            x, y = prob.pair(U)
            xn, tn = normalise(x, y, shift, scale, out_scale, prob.nve)
            apri.append((t,) + a_priori(torch, net, xn, tn))
    Uf = prob.fine_run(torch, seed, t_end, dt_snap, each, log=log)
    if target == "interval":
        for k, (x, y) in enumerate(zip(*interval_targets(torch, prob, Ucs, dt_snap))):
            xn, tn = normalise(x, y, shift, scale, out_scale, prob.nve)
            apri.append((k * dt_snap,) + a_priori(torch, net, xn, tn))
        del Ucs
    torch.cuda.synchronize()
    wall_fine_total = time.perf_counter() - t0
    del Uf
    # the fine run alone, untimed work (pairs, diagnostics) excluded
    U = prob.initial(torch, seed)
    nsub = max(1, round(dt_snap / prob.dt_f))
    nchk = int(round(t_end / dt_snap))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(nchk):
        for _ in range(nsub):
            prob.fine.rk_step(U, dt_snap / nsub)
        if k % 4 == 3:
            torch.cuda.synchronize()
            log(f"closure: timed fine run at t={(k + 1) * dt_snap:.2f}")
    torch.cuda.synchronize()
    wall_fine = time.perf_counter() - t0
    del U
    n0 = math.sqrt(sum(a[1] ** 2 for a in apri))
    n1 = math.sqrt(sum(a[2] ** 2 for a in apri))
    log(f"closure: held-out residual error {n0:.4e} -> {n1:.4e} (ratio {n1 / n0:.3f}); fine run {wall_fine:.1f} s")
    out = {"t": [dt_snap * i for i in range(nchk + 1)], "wall_fine_s": wall_fine,
           "wall_fine_with_sampling_s": wall_fine_total,
           "a_priori": {"target_norm": n0, "residual_norm": n1, "ratio": n1 / n0,
                        "per_snapshot": [{"t": a[0], "ratio": a[2] / a[1]} for a in apri]},
           "ref_ke": [r["ke"] for r in ref], "ref_enstrophy": [r["enstrophy"] for r in ref]}
    Uc0 = prob.filt(prob.initial(torch, seed))
    ncc = max(1, round(dt_snap / prob.dt_c))
    dtc = dt_snap / ncc
    ke0 = ref[0]["ke"]
    ens_peak = max(r["enstrophy"] for r in ref)
    for name, cfg in [("plain", None)] + [(v[0], v[1:]) for v in variants]:
        max_ratio, ke_tol = cfg if cfg else (0.0, 0.0)
        on = lambda: prob.coarse.closure_set(net, *norm, max_ratio=max_ratio)
        off = lambda: prob.coarse.closure_set(None)
        if cfg:
            on()
        U = Uc0.clone()
        hist = [prob.coarse.diagnostics(U)]
        fallback = []
        rejected = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(nchk):
            saved = U.clone() if cfg else None
            for _ in range(ncc):
                prob.coarse.rk_step(U, dtc)
            d = prob.coarse.diagnostics(U)
            if cfg and (d["nonfinite"] or d["ke"] > hist[-1]["ke"] * (1.0 + ke_tol)):
                # fallback: redo this interval with the plain scheme
                fallback.append(out["t"][k])
                rejected += prob.coarse.closure_rejected()
                off()
                U.copy_(saved)
                for _ in range(ncc):
                    prob.coarse.rk_step(U, dtc)
                d = prob.coarse.diagnostics(U)
                on()
            hist.append(d)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if cfg:
            rejected += prob.coarse.closure_rejected()
            off()
        out[name] = {
            "max_ratio": max_ratio, "ke_tol": ke_tol,
            "ke_err": max(abs(h["ke"] - r["ke"]) for h, r in zip(hist, ref)) / ke0,
            "ens_err": max(abs(h["enstrophy"] - r["enstrophy"]) for h, r in zip(hist, ref)) / ens_peak,
            "wall_s": wall, "fallback_intervals": fallback, "element_corrections_rejected": rejected,
            "element_evaluations": (nchk * ncc * 4 * prob.coarse.ne) if cfg else 0,
            "ke": [h["ke"] for h in hist], "enstrophy": [h["enstrophy"] for h in hist],
        }
        log(f"closure: {name} KE err {out[name]['ke_err']:.3e} enstrophy err {out[name]['ens_err']:.3e} "
            f"wall {wall:.2f} s plain-scheme intervals {fallback} rejected {rejected}")
    return out


def train(torch, prob, seeds, t_end, dt_snap, n_sym=8, hidden=128, iters=10000, batch=1024, lr=1e-3,
          weight_power=0.5, log=print, target="rhs"):
    """Pairs from the fine runs of ``seeds``, symmetry images, normalisation,
    snapshot weights and the fit; returns (net, normalisation, losses, samples)."""
    X, T, snap = generate(torch, prob, seeds, t_end, dt_snap, log=log, target=target)
    X, T, snap = augment(X, T, prob.n, n_sym, seed=12345, extra=snap)
    shift, scale, out_scale = normalisation(X, T, prob.nve)
    w = snapshot_weights(T, snap, out_scale, weight_power) if weight_power else None
    Xn, Tn = normalise(X, T, shift, scale, out_scale, prob.nve)
    del X, T
    log(f"closure: {Xn.shape[0]} training samples")
    net, losses = fit(torch, Xn, Tn, hidden, iters, batch, lr, weights=w, log=log)
    return net, (shift.tolist(), scale.tolist(), out_scale.tolist()), losses, int(Xn.shape[0])


def run(nel_f=64, ratio=4, p=3, Re=5000.0, train_seeds=range(7), test_seed=7, t_end=4.0, dt_snap=0.5,
        n_sym=8, hidden=128, iters=10000, batch=1024, lr=1e-3, weight_power=0.5, log=print, out_path=None,
        load=None, variants=VARIANTS, target="rhs"):
    """Train (or load ``load`` = (params .npy, norm .json)) and evaluate."""
    import torch
    prob = Problem(nel_f, ratio, p, Re)
    cfg = {"nel_fine": nel_f, "nel_coarse": nel_f // ratio, "p": p, "Re": Re, "train_seeds": list(train_seeds),
           "test_seed": test_seed, "t_end": t_end, "dt_snap": dt_snap, "n_sym": n_sym, "hidden": hidden,
           "iters": iters, "batch": batch, "lr": lr, "weight_power": weight_power, "target": target}
    res = {"config": cfg}
    if load:
        nve = prob.nve
        net = Mlp(nve, hidden, nve, P=torch.from_numpy(np.load(load[0])).to("cuda"))
        net.round_weights()
        with open(load[1]) as f:
            saved = json.load(f)
        norm = tuple(saved["norm"])
        res["train"] = saved.get("train")
        # the loaded network's own training configuration replaces the
        # training fields of this run's
        for k in ("train_seeds", "n_sym", "hidden", "iters", "batch", "lr", "weight_power"):
            cfg.pop(k, None)
        cfg["loaded"] = list(load)
        cfg["trained_with"] = saved.get("config")
    else:
        net, norm, losses, ns = train(torch, prob, list(train_seeds), t_end, dt_snap, n_sym, hidden, iters, batch,
                                      lr, weight_power, log=log, target=target)
        res["train"] = {"losses": losses, "samples": ns}
        if out_path:
            np.save(out_path.replace(".json", "_params.npy"), net.P.cpu().numpy())
            with open(out_path.replace(".json", "_norm.json"), "w") as f:
                json.dump({"norm": norm, "train": res["train"], "config": cfg}, f)
    if test_seed is not None:
        post = evaluate(torch, prob, test_seed, t_end, dt_snap, net, norm, variants, log=log, target=target)
        res["a_priori"] = post.pop("a_priori")
        res["a_posteriori"] = post
        if variants:
            res["speedup_vs_fine"] = post["wall_fine_s"] / post[variants[0][0]]["wall_s"]
    if out_path:
        with open(out_path, "w") as f:
            json.dump(res, f)
    return res


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="train and evaluate the learned coarse-grid closure")
    ap.add_argument("--nel-fine", type=int, default=64)
    ap.add_argument("--ratio", type=int, default=4)
    ap.add_argument("--p", type=int, default=3)
    ap.add_argument("--Re", type=float, default=5000.0)
    ap.add_argument("--train-seeds", type=int, default=7)
    ap.add_argument("--test-seed", type=int, default=None, help="default: the seed after the training seeds")
    ap.add_argument("--no-eval", action="store_true")
    ap.add_argument("--t-end", type=float, default=4.0)
    ap.add_argument("--dt-snap", type=float, default=0.5)
    ap.add_argument("--n-sym", type=int, default=8)
    ap.add_argument("--hidden", type=int, default=128)
    ap.add_argument("--iters", type=int, default=10000)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--weight-power", type=float, default=0.5, help="0: unweighted loss")
    ap.add_argument("--load", nargs=2, default=None, metavar=("PARAMS_NPY", "NORM_JSON"))
    ap.add_argument("--variants", default=None,
                    help="corrected runs as name:max_ratio:ke_tol,... (default: %s)" %
                    ",".join(f"{n}:{m}:{k}" for n, m, k in VARIANTS))
    ap.add_argument("--target", default="rhs", choices=["rhs", "interval"],
                    help="rhs: residual defect at each snapshot; interval: trajectory defect over each interval")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    variants = VARIANTS if a.variants is None else [
        (w.split(":")[0], float(w.split(":")[1]), float(w.split(":")[2])) for w in a.variants.split(",")]
    test_seed = None if a.no_eval else (a.train_seeds if a.test_seed is None else a.test_seed)
    res = run(a.nel_fine, a.ratio, a.p, a.Re, range(a.train_seeds), test_seed, a.t_end, a.dt_snap, a.n_sym,
              a.hidden, a.iters, a.batch, a.lr, a.weight_power, log=lambda s: print(s, flush=True), out_path=a.out,
              load=a.load, variants=variants, target=a.target)
    short = {k: res[k] for k in ("config", "a_priori", "speedup_vs_fine") if k in res}
    if "a_priori" in short:
        short["a_priori"] = {k: v for k, v in short["a_priori"].items() if k != "per_snapshot"}
    print(json.dumps(short), flush=True)
    for k in ["plain"] + [v[0] for v in variants]:
        r = res.get("a_posteriori", {}).get(k)
        if r:
            print(json.dumps({k: {x: r[x] for x in ("ke_err", "ens_err", "wall_s", "fallback_intervals")}}), flush=True)


if __name__ == "__main__":
    main()
