"""FP64 reference of the closure network and of the fine-to-coarse filter
(test infrastructure only).

Network: y = W3 g(W2 g(W1 x + b1) + b2) + b3 with the exact-erf GELU
g(z) = z (1 + erf(z / sqrt 2)) / 2; weights stored row-major [out][in].
``bf16=True`` states the arithmetic of the GPU kernels: weights and every
layer input are rounded to bfloat16 (round to nearest even) before the
product, products and sums are exact here (FP64) and FP32 on the GPU.
The backward pass is the exact gradient of that computation with the
roundings taken as fixed values (the usual straight-through convention).

Filter: L2 projection of a fine degree-p solution onto the degree-p space of
each coarse element (r^3 fine elements per coarse element), evaluated at the
coarse solution points; every integral uses the fine elements' Gauss rule,
exact for the products involved.
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


def bf16_round(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    a = np.asarray(x, dtype=np.float32)
    b = a.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(a)
    if np.any(nan):
        out[nan] = np.nan
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_prime(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def param_shapes(n_in, n_h, n_out):
    return [("W1", (n_h, n_in)), ("b1", (n_h,)), ("W2", (n_h, n_h)), ("b2", (n_h,)),
            ("W3", (n_out, n_h)), ("b3", (n_out,))]


def unflatten(flat, n_in, n_h, n_out):
    out, o = {}, 0
    for name, shp in param_shapes(n_in, n_h, n_out):
        size = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + size], dtype=np.float64).reshape(shp)
        o += size
    return out


def flatten(p):
    return np.concatenate([p[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def forward(p, x, bf16=False):
    """x [B, n_in] -> y [B, n_out] and the cache for backward."""
    rnd = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    W1, W2, W3 = (rnd(p[k]) for k in ("W1", "W2", "W3"))
    a0 = rnd(x)
    z1 = a0 @ W1.T + p["b1"]
    a1 = rnd(gelu(z1))
    z2 = a1 @ W2.T + p["b2"]
    a2 = rnd(gelu(z2))
    y = a2 @ W3.T + p["b3"]
    return y, dict(a0=a0, z1=z1, a1=a1, z2=z2, a2=a2, W1=W1, W2=W2, W3=W3)


def backward(cache, dy):
    """Gradient of sum(dy * y) with respect to every parameter."""
    c = cache
    g = {}
    g["W3"] = dy.T @ c["a2"]
    g["b3"] = dy.sum(axis=0)
    da2 = dy @ c["W3"]
    dz2 = da2 * gelu_prime(c["z2"])
    g["W2"] = dz2.T @ c["a1"]
    g["b2"] = dz2.sum(axis=0)
    da1 = dz2 @ c["W2"]
    dz1 = da1 * gelu_prime(c["z1"])
    g["W1"] = dz1.T @ c["a0"]
    g["b1"] = dz1.sum(axis=0)
    return g


def mse(y, t, w=None):
    """Mean square error of y against t ([rows, cols]), each row weighted by
    w[row] (default 1), and its gradient with respect to y."""
    d = y - t
    wr = np.ones(d.shape[0]) if w is None else np.asarray(w, dtype=np.float64)
    wd = wr.reshape((-1,) + (1,) * (d.ndim - 1)) * d
    return float(np.sum(wd * d) / d.size), 2.0 * wd / d.size


def adam(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba) on flat arrays; returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(n_in, n_h, n_out, seed):
    """Seeded uniform fan-in initialisation."""
    rng = np.random.Generator(np.random.PCG64(seed))
    p = {}
    for name, shp in param_shapes(n_in, n_h, n_out):
        if name.startswith("W"):
            lim = 1.0 / math.sqrt(shp[1])
            p[name] = rng.uniform(-lim, lim, shp)
        else:
            p[name] = np.zeros(shp)
    return p


def lagrange_matrix(nodes, x):
    """L[i, a] = l_i(x_a) for the Lagrange basis on ``nodes``."""
    L = np.ones((len(nodes), len(x)))
    for i, xi in enumerate(nodes):
        for k, xk in enumerate(nodes):
            if k != i:
                L[i] *= (x - xk) / (xi - xk)
    return L


def filter_matrix(p, r):
    """1-D projection operator P[i, a]: coarse coefficient i from the r (p+1)
    fine solution-point values along one direction of a coarse element."""
    xs, ws = np.polynomial.legendre.leggauss(p + 1)
    # fine point a (fine element f, local point j) in coarse reference coordinates
    xa = np.concatenate([-1.0 + (2.0 * f + xs + 1.0) / r for f in range(r)])
    wa = np.concatenate([ws / r for _ in range(r)])          # fine weights in coarse coordinates
    L = lagrange_matrix(xs, xa)                                 # l_i(x_a)
    # coefficient c_i of the projection with the (diagonal, exact) coarse
    # Gauss mass matrix: c_i = sum_a w_a l_i(x_a) u_a / w_i
    return (L * wa[None, :]) / ws[:, None]


def filter_state(Uf, nel_f, p, r):
    """Fine state [ne_f, nv, n, n, n] on nel_f elements -> coarse state on
    nel_f / r elements (same p)."""
    n = p + 1
    nv = Uf.shape[1]
    nxf, nyf, nzf = nel_f
    nxc, nyc, nzc = nxf // r, nyf // r, nzf // r
    P = filter_matrix(p, r)
    # global fine grid [v, gz, gy, gx]
    G = Uf.reshape(nzf, nyf, nxf, nv, n, n, n).transpose(3, 0, 4, 1, 5, 2, 6).reshape(nv, nzf * n, nyf * n, nxf * n)
    G = G.reshape(nv, nzc, r * n, nyc, r * n, nxc, r * n)
    C = np.einsum("iz,vZzYyXx->vZiYyXx", P, G)
    C = np.einsum("jy,vZiYyXx->vZiYjXx", P, C)
    C = np.einsum("kx,vZiYjXx->vZiYjXk", P, C)
    # [v, Zc, k(z), Yc, j(y), Xc, i(x)] -> [e_c, v, k, j, i]
    return np.ascontiguousarray(C.transpose(1, 3, 5, 0, 2, 4, 6).reshape(nxc * nyc * nzc, nv, n, n, n))
