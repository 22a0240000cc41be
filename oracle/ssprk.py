"""Strong-stability-preserving Runge-Kutta (5 stages, order 4) of Spiteri &
Ruuth, the time integrator of the paper's TGV runs (section 4.4 names the
scheme; its coefficients are not printed there).  Test infrastructure only.

Shu-Osher form: u^(i) = sum_{j<i} alpha_ij u^(j) + dt beta_ij L(u^(j)),
u^(0) = u^n, u^{n+1} = u^(5).  The coefficients are the published ones; the
tests check the eight order-4 conditions of the equivalent Butcher tableau
and the SSP coefficient min alpha/beta (1.508) against them.
"""
import numpy as np

# (alpha, beta) per stage i = 1..5, nonzero entries only: {j: (alpha_ij, beta_ij)}
STAGES = [
    {0: (1.0, 0.391752226571890)},
    {0: (0.444370493651235, 0.0), 1: (0.555629506348765, 0.368410593050371)},
    {0: (0.620101851488403, 0.0), 2: (0.379898148511597, 0.251891774271694)},
    {0: (0.178079954393132, 0.0), 3: (0.821920045606868, 0.544974750228521)},
    {2: (0.517231671970585, 0.0), 3: (0.096059710526147, 0.063692468666290),
     4: (0.386708617503269, 0.226007483236906)},
]


def shu_osher():
    """Dense alpha, beta [6][5] (row i = stage i, columns j < i)."""
    a = np.zeros((6, 5))
    b = np.zeros((6, 5))
    for i, st in enumerate(STAGES, start=1):
        for j, (al, be) in st.items():
            a[i, j], b[i, j] = al, be
    return a, b


def butcher():
    """Equivalent Butcher tableau (A [5][5], b [5], c [5]) of the Shu-Osher form."""
    a, bb = shu_osher()
    A = np.zeros((6, 5))
    for i in range(1, 6):
        for j in range(i):
            A[i] += a[i, j] * A[j]
            A[i, j] += bb[i, j]
    Am = A[:5]
    return Am, A[5], Am.sum(axis=1)


def step(rhs, u, dt):
    """One step: rhs(u) returns L(u) for an array u."""
    stages = [u]
    L = {}
    for i, st in enumerate(STAGES, start=1):
        v = np.zeros_like(u)
        for j, (al, be) in st.items():
            v = v + al * stages[j]
            if be != 0.0:
                if j not in L:
                    L[j] = rhs(stages[j])
                v = v + dt * be * L[j]
        stages.append(v)
    return stages[5]


def integrate(rhs, u, dt, nsteps):
    for _ in range(nsteps):
        u = step(rhs, u, dt)
    return u
