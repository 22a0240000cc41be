/*
 * Plain FP64 CPU oracle for the Spectral Difference (SD) right-hand side with
 * the standard BR1 and the compact second-order flux treatment
 * (Lodato & Tonicello, "A novel compact scheme for second-order fluxes applied
 * to the Spectral Difference method").
 *
 * TEST INFRASTRUCTURE ONLY.  This code exists to check the HIP path: only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code with the GPU library.  It is written to be read
 * against the paper, not to be fast: every element is computed on its own
 * from the literal definitions, recomputing whatever it needs from its
 * neighbours.
 *
 * Conventions
 *   n = p + 1 solution points per direction (Gauss-Legendre), n + 1 flux
 *   points (the two element ends plus the n - 1 Gauss-Legendre points),
 *   ascending in [-1, 1].
 *   1-D state: u[e][i], e < N, i < n.
 *   3-D state: u[e][v][k][j][i], e = ex + Nx*(ey + Ny*ez), i along x.
 *   Meshes are uniform Cartesian and periodic in every direction.
 */
#ifndef SD_ORACLE_H
#define SD_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAXN 10

enum { OR_BR1 = 0, OR_COMPACT = 1 };
enum { OR_DIFFUSION = 0, OR_PME = 1, OR_NAVIER_STOKES = 2 };

typedef struct {
  int physics;
  double nu;              /* linear diffusion coefficient                     */
  double pme_m;           /* porous-medium exponent (integer >= 1)            */
  double gamma, Re, Ma, Pr;
  double rho0, u0, Lref;  /* reference density, velocity, length             */
  double sutherland_s;    /* Sutherland constant over the reference
                             temperature; a negative value means constant mu */
  double lambda_over_mu;  /* second viscosity coefficient over mu            */
  double entropy_fix;     /* Harten delta = entropy_fix * (|u_n| + c)        */
  double eta_ip;          /* interior penalty (section 3): the normal
                             component of the common gradient at an
                             interface gains tau (u_R - u_L), tau =
                             eta_ip (p+1)^2 / h, h the element size normal
                             to the interface; 0 = off                       */
} or_params;

/* Gauss-Legendre nodes (ascending) and weights on [-1, 1]. */
int or_gauss_legendre(int n, double *x, double *w);

/* Solution points xs[n], weights ws[n], flux points xf[n+1],
 * interpolation L[(n+1) x n] and differentiation M[n x (n+1)], row major. */
int or_operators(int p, double *xs, double *ws, double *xf, double *L, double *M);

/* 1-D semi-discrete RHS du/dt for u[N][n] on the periodic [x0, x1].
 * physics: OR_DIFFUSION (coef = nu) or OR_PME (coef = m); eta_ip: interior
 * penalty coefficient (0 = off), as in or_params. */
int or_rhs_1d(int N, int p, double x0, double x1, int scheme, int physics,
              double coef, double eta_ip, const double *u, double *dudt);

/* Classical RK4 for the 1-D problem, nsteps steps of size dt, in place. */
int or_rk4_1d(int N, int p, double x0, double x1, int scheme, int physics,
              double coef, double eta_ip, double *u, double dt, int nsteps);

/* 3-D semi-discrete RHS on a periodic nel[0] x nel[1] x nel[2] box.
 * Scalar physics (diffusion, PME) has one variable, Navier-Stokes five.
 * nthreads <= 0 uses the OpenMP default. */
int or_rhs_3d(const int *nel, const double *lo, const double *hi, int p,
              int scheme, const or_params *prm, const double *u, double *dudt,
              int nthreads);

/* The same RHS for a list of elements only: dudt_sel[k] holds element
 * elems[k] (nv * n^3 values each). */
int or_rhs_3d_elems(const int *nel, const double *lo, const double *hi, int p,
                    int scheme, const or_params *prm, const double *u,
                    const long *elems, long n_elems, double *dudt_sel,
                    int nthreads);

/* Classical RK4 steps on the 3-D problem, in place. */
int or_rk4_3d(const int *nel, const double *lo, const double *hi, int p,
              int scheme, const or_params *prm, double *u, double dt,
              int nsteps, int nthreads);

/* Diagnostics of a Navier-Stokes state: out[0] kinetic energy, out[1]
 * enstrophy, out[2] mass, out[3..5] momentum, out[6] total energy,
 * out[7] max |u|, out[8] 1 if any value is non-finite, out[9] max(|u| + c)
 * with c = sqrt(gamma P / rho), infinite if rho <= 0 or P < 0 anywhere. */
int or_diag_3d(const int *nel, const double *lo, const double *hi, int p,
               const or_params *prm, const double *u, double *out,
               int nthreads);

/* Navier-Stokes pointwise laws, exported for their own tests.
 * U[5] conservative state, G[15] conservative gradient G[v*3 + m],
 * d the flux direction. */
void or_ns_flux_conv(const or_params *prm, const double *U, int d, double *F);
void or_ns_flux_visc(const or_params *prm, const double *U, const double *G,
                     int d, double *F);
void or_ns_roe(const or_params *prm, const double *UL, const double *UR, int d,
               double *F);
/* Sum of lambda_k alpha_k r_k with signed eigenvalues and no entropy fix
 * (equals F(UR) - F(UL) for a Roe linearisation). */
void or_ns_roe_signed_waves(const or_params *prm, const double *UL,
                            const double *UR, int d, double *D);

#ifdef __cplusplus
}
#endif
#endif
