"""ctypes front end of the C oracle (test infrastructure only).

Thin marshalling around ``libsd_oracle.so``: numpy float64 arrays in, numpy
arrays out.  Nothing here does any of the method's arithmetic.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsd_oracle.so")
SRC_PATH = os.path.join(HERE, "sd_oracle.c")

BR1, COMPACT = 0, 1
DIFFUSION, PME, NAVIER_STOKES = 0, 1, 2
SCHEMES = {"br1": BR1, "compact": COMPACT}


def build(force=True):
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    if not force and os.path.exists(LIB_PATH) and os.path.getmtime(LIB_PATH) >= os.path.getmtime(SRC_PATH):
        return LIB_PATH
    cmd = ["gcc", "-O2", "-std=gnu99", "-fopenmp", "-fPIC", "-shared", "-Wall",
           "-o", LIB_PATH, SRC_PATH, "-lm"]
    subprocess.check_call(cmd)
    return LIB_PATH


class Params(ctypes.Structure):
    _fields_ = [
        ("physics", ctypes.c_int),
        ("nu", ctypes.c_double),
        ("pme_m", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("Re", ctypes.c_double),
        ("Ma", ctypes.c_double),
        ("Pr", ctypes.c_double),
        ("rho0", ctypes.c_double),
        ("u0", ctypes.c_double),
        ("Lref", ctypes.c_double),
        ("sutherland_s", ctypes.c_double),
        ("lambda_over_mu", ctypes.c_double),
        ("entropy_fix", ctypes.c_double),
        ("eta_ip", ctypes.c_double),
    ]


def make_params(physics="ns", nu=1.0, pme_m=2.0, gamma=1.4, Re=1600.0, Ma=0.1, Pr=0.71,
                rho0=1.0, u0=1.0, Lref=1.0, sutherland_s=110.4 / 300.0,
                lambda_over_mu=0.0, entropy_fix=0.1, eta_ip=0.0):
    phys = {"diffusion": DIFFUSION, "pme": PME, "ns": NAVIER_STOKES}[physics]
    return Params(phys, nu, pme_m, gamma, Re, Ma, Pr, rho0, u0, Lref, sutherland_s,
                  lambda_over_mu, entropy_fix, eta_ip)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        lp = ctypes.POINTER(ctypes.c_long)
        pp = ctypes.POINTER(Params)
        L.or_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.or_operators.argtypes = [ctypes.c_int, dp, dp, dp, dp, dp]
        L.or_rhs_1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp, dp]
        L.or_rk4_1d.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, dp,
                                ctypes.c_double, ctypes.c_int]
        L.or_rhs_3d.argtypes = [ip, dp, dp, ctypes.c_int, ctypes.c_int, pp, dp, dp, ctypes.c_int]
        L.or_rhs_3d_elems.argtypes = [ip, dp, dp, ctypes.c_int, ctypes.c_int, pp, dp, lp,
                                      ctypes.c_long, dp, ctypes.c_int]
        L.or_rk4_3d.argtypes = [ip, dp, dp, ctypes.c_int, ctypes.c_int, pp, dp, ctypes.c_double,
                                ctypes.c_int, ctypes.c_int]
        L.or_diag_3d.argtypes = [ip, dp, dp, ctypes.c_int, pp, dp, dp, ctypes.c_int]
        for f in ("or_ns_flux_conv",):
            getattr(L, f).argtypes = [pp, dp, ctypes.c_int, dp]
        L.or_ns_flux_visc.argtypes = [pp, dp, dp, ctypes.c_int, dp]
        L.or_ns_roe.argtypes = [pp, dp, dp, ctypes.c_int, dp]
        L.or_ns_roe_signed_waves.argtypes = [pp, dp, dp, ctypes.c_int, dp]
        for f in ("or_gauss_legendre", "or_operators", "or_rhs_1d", "or_rk4_1d", "or_rhs_3d",
                  "or_rhs_3d_elems", "or_rk4_3d", "or_diag_3d"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def gauss_legendre(n):
    x = np.zeros(n)
    w = np.zeros(n)
    _check(lib().or_gauss_legendre(n, _p(x), _p(w)), "gauss_legendre")
    return x, w


def operators(p):
    """(xs, ws, xf, L, M) for polynomial degree p."""
    n = p + 1
    xs, ws, xf = np.zeros(n), np.zeros(n), np.zeros(n + 1)
    L = np.zeros((n + 1, n))
    M = np.zeros((n, n + 1))
    _check(lib().or_operators(p, _p(xs), _p(ws), _p(xf), _p(L), _p(M)), "operators")
    return xs, ws, xf, L, M


def rhs_1d(u, p, x0, x1, scheme="compact", physics="diffusion", coef=1.0, eta_ip=0.0):
    u = _f64(u)
    N = u.shape[0]
    out = np.zeros_like(u)
    phys = {"diffusion": DIFFUSION, "pme": PME}[physics]
    _check(lib().or_rhs_1d(N, p, x0, x1, SCHEMES[scheme], phys, coef, eta_ip, _p(u), _p(out)), "rhs_1d")
    return out


def rk4_1d(u, p, x0, x1, dt, nsteps, scheme="compact", physics="diffusion", coef=1.0, eta_ip=0.0):
    u = _f64(u).copy()
    phys = {"diffusion": DIFFUSION, "pme": PME}[physics]
    _check(lib().or_rk4_1d(u.shape[0], p, x0, x1, SCHEMES[scheme], phys, coef, eta_ip, _p(u), dt,
                           nsteps), "rk4_1d")
    return u


def _mesh(nel, lo, hi):
    nel_a = (ctypes.c_int * 3)(*[int(v) for v in nel])
    lo_a = np.asarray(lo, dtype=np.float64)
    hi_a = np.asarray(hi, dtype=np.float64)
    return nel_a, lo_a, hi_a


def rhs_3d(u, nel, lo, hi, p, scheme, params, nthreads=0):
    u = _f64(u)
    out = np.zeros_like(u)
    nel_a, lo_a, hi_a = _mesh(nel, lo, hi)
    _check(lib().or_rhs_3d(nel_a, _p(lo_a), _p(hi_a), p, SCHEMES[scheme], ctypes.byref(params),
                           _p(u), _p(out), nthreads), "rhs_3d")
    return out


def rhs_3d_elems(u, nel, lo, hi, p, scheme, params, elems, nthreads=0):
    u = _f64(u)
    elems = np.ascontiguousarray(elems, dtype=np.int64)
    out = np.zeros((len(elems),) + u.shape[1:], dtype=np.float64)
    nel_a, lo_a, hi_a = _mesh(nel, lo, hi)
    _check(lib().or_rhs_3d_elems(nel_a, _p(lo_a), _p(hi_a), p, SCHEMES[scheme],
                                 ctypes.byref(params), _p(u),
                                 elems.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), len(elems),
                                 _p(out), nthreads), "rhs_3d_elems")
    return out


def rk4_3d(u, nel, lo, hi, p, scheme, params, dt, nsteps, nthreads=0):
    u = _f64(u).copy()
    nel_a, lo_a, hi_a = _mesh(nel, lo, hi)
    _check(lib().or_rk4_3d(nel_a, _p(lo_a), _p(hi_a), p, SCHEMES[scheme], ctypes.byref(params),
                           _p(u), dt, nsteps, nthreads), "rk4_3d")
    return u


def diag_3d(u, nel, lo, hi, p, params, nthreads=0):
    u = _f64(u)
    out = np.zeros(10)
    nel_a, lo_a, hi_a = _mesh(nel, lo, hi)
    _check(lib().or_diag_3d(nel_a, _p(lo_a), _p(hi_a), p, ctypes.byref(params), _p(u), _p(out),
                            nthreads), "diag_3d")
    keys = ["ke", "enstrophy", "mass", "mom0", "mom1", "mom2", "energy", "umax", "nonfinite", "smax"]
    return dict(zip(keys, out.tolist()))


def ns_flux_conv(params, U, d):
    U = _f64(U)
    F = np.zeros(5)
    lib().or_ns_flux_conv(ctypes.byref(params), _p(U), d, _p(F))
    return F


def ns_flux_visc(params, U, G, d):
    """G[v, m] = dU_v/dx_m."""
    U = _f64(U)
    G = _f64(G).reshape(15)
    F = np.zeros(5)
    lib().or_ns_flux_visc(ctypes.byref(params), _p(U), _p(G), d, _p(F))
    return F


def ns_roe(params, UL, UR, d):
    UL, UR = _f64(UL), _f64(UR)
    F = np.zeros(5)
    lib().or_ns_roe(ctypes.byref(params), _p(UL), _p(UR), d, _p(F))
    return F


def ns_roe_signed_waves(params, UL, UR, d):
    UL, UR = _f64(UL), _f64(UR)
    D = np.zeros(5)
    lib().or_ns_roe_signed_waves(ctypes.byref(params), _p(UL), _p(UR), d, _p(D))
    return D
