/*
 * sd.h - C ABI of the MI355X Spectral Difference right-hand side.
 *
 * The library evaluates the semi-discrete SD right-hand side of
 *     du/dt + div F(u, grad u) = 0,
 * written as the first-order system with the auxiliary gradient v = grad u
 * and mapped to the reference hexahedron (Lodato & Tonicello, section 2,
 * eqs. ns and ns:mapped/adj:f), on structured periodic hexahedral meshes:
 * uniform Cartesian ones, or (3-D diffusion and Navier-Stokes, FP64 or
 * FP32) curvilinear elements given by their node coordinates
 * (sd_set_geometry).
 * The
 * auxiliary gradient is reconstructed either with the standard BR1-type
 * centred treatment (section 2.1: common solution eq. c:flux, gradient
 * eqs. w:e/v:e, common gradient eq. aux:v:int; five-element stencil in 1-D)
 * or with the compact one-sided continuous fluxes (section 2.2: eqs.
 * c:flux:l/r, v:s:l/r, cmp:int:fp, cmp:int:avg; three-element stencil), and
 * in three dimensions with the direction-by-direction construction of
 * section 2.3.  Interface viscous fluxes use option (a) of section 2.1
 * (flux of the averaged solution and averaged gradient).  Physics: linear
 * diffusion, the porous medium equation (section 4.3) and the compressible
 * Navier-Stokes equations of section 4.4 (Roe flux with Harten's entropy fix
 * at interfaces, Sutherland viscosity, gradients of conservative
 * variables).
 *
 * Points: n = p + 1 Gauss-Legendre solution points per direction; n + 1 flux
 * points (the two element ends and the (n-1)-point Gauss-Legendre rule).
 *
 * State layout (device memory, FP64, owned by the caller):
 *   dim = 3: u[e][v][k][j][i], e = ex + Nx*(ey + Ny*ez), i along x fastest;
 *   dim = 1: u[e][v][i].
 *   nv = 1 for scalar physics, 5 for Navier-Stokes (rho, rho u, rho v,
 *   rho w, rho E).
 *
 * Streams: every call is enqueued asynchronously on the context's HIP stream
 * (the one given to sd_init or sd_set_stream); only sd_diagnostics waits for
 * that stream, to fill its host-side result.
 *
 * Errors: every entry point returns SD_OK (0) or a negative code, and sets a
 * thread-local message readable with sd_last_error().  On error nothing has
 * been enqueued, except for SD_EHIP, where a launch may have failed midway.
 */
#ifndef SD_H
#define SD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SD_OK 0
#define SD_EINVAL (-1)       /* bad argument: null pointer, size, enum      */
#define SD_ENOMEM (-2)       /* device or host allocation failed            */
#define SD_EHIP (-3)         /* a HIP runtime call or kernel launch failed  */
#define SD_ENONFINITE (-4)   /* diagnostics found a NaN or an infinity      */
#define SD_EUNSUPPORTED (-5) /* valid but not built: p, dim x physics combo */

typedef enum { SD_BR1 = 0, SD_COMPACT = 1 } sd_scheme;
typedef enum { SD_DIFFUSION = 0, SD_PME = 1, SD_NAVIER_STOKES = 2 } sd_physics;
/* Arithmetic of the contractions and fluxes.  The public state, the RHS and
 * the RK accumulation stay FP64 in every mode.  SD_FP32: FP32 on the vector
 * units.  SD_BF16X3: as SD_FP32, with the gradient and divergence line
 * contractions as three BF16 products on the matrix cores (3-D
 * Navier-Stokes only).  SD_FP32_MFMA: as SD_FP32, with those contractions on
 * the FP32 matrix instruction (3-D Navier-Stokes only). */
typedef enum { SD_FP64 = 0, SD_FP32 = 1, SD_BF16X3 = 2, SD_FP32_MFMA = 3 } sd_precision;
/* Time integrator of sd_rk_step: classical RK4 (4 stages), or the
 * five-stage, fourth-order strong-stability-preserving scheme of Spiteri and
 * Ruuth that section 4.4 integrates the TGV with (Shu-Osher form, published
 * coefficients; the paper does not print them). */
typedef enum { SD_RK4 = 0, SD_SSPRK54 = 1 } sd_integrator;

/* Uniform periodic Cartesian mesh: dim 1 uses nelem[0], lo[0], hi[0] only. */
typedef struct {
  int dim;
  int nelem[3];
  double lo[3];
  double hi[3];
} sd_mesh;

typedef struct {
  int physics;            /* sd_physics                                      */
  double nu;              /* diffusion coefficient                           */
  double pme_m;           /* porous-medium exponent m, integer in [1, 8]     */
  double gamma;           /* heat-capacity ratio (section 4.4: 1.4)          */
  double Re, Ma, Pr;      /* mu0 = rho0 u0 L / Re, p0 = rho0 (u0/Ma)^2 / gamma */
  double rho0, u0, Lref;  /* reference density, velocity and length         */
  double sutherland_s;    /* Sutherland constant over the reference
                             temperature p0/(rho0 R); negative: constant mu */
  double lambda_over_mu;  /* second viscosity coefficient (section 4.4: 0)   */
  double entropy_fix;     /* Harten delta = entropy_fix * (|u_n| + c), applied
                             to the two acoustic waves; 0 disables it        */
  int precision;          /* sd_precision                                    */
  int ref_state;          /* 1: subtract the constant state (rho0, 0, 0, 0,
                             p0/(gamma-1)) before the contractions (exact
                             algebra: L reproduces constants, M annihilates
                             them); -1: automatic (on unless FP64)          */
  double eta_ip;          /* interior penalty (section 3): the normal
                             component of the common gradient at every
                             interface gains tau (u_R - u_L),
                             tau = eta_ip (p+1)^2 / h, h the element size
                             normal to the interface; 0 (default) = off,
                             negative or non-finite = SD_EINVAL             */
  int integrator;         /* sd_integrator of sd_rk_step (default SD_RK4)    */
} sd_params;

typedef struct {
  double ke;         /* 1/2 int u.u dV (section 4.4), Gauss quadrature      */
  double enstrophy;  /* int w.w dV, w = curl u from the standard gradient   */
  double mass;       /* int rho dV                                          */
  double mom[3];     /* int rho u dV                                        */
  double energy;     /* int rho E dV                                        */
  double umax;       /* max |u| over the solution points                    */
  int nonfinite;     /* 1 if any state value is NaN or infinite             */
  double smax;       /* max (|u| + c) over the solution points, c^2 =
                        gamma P / rho; +inf if rho <= 0 or P < 0 anywhere  */
} sd_diag;

typedef struct sd_ctx sd_ctx;

/* Fill *prm with the Taylor-Green defaults (Navier-Stokes, gamma 1.4,
 * Re 1600, Ma 0.1, Pr 0.71, rho0 = u0 = L = 1, Sutherland 110.4/300,
 * lambda 0, entropy fix 0.1, FP64, automatic reference state). */
int sd_params_default(sd_params *prm);

/* Create a context for polynomial degree p (n = p + 1 points) and scheme
 * (sd_scheme).  Supported: dim 1 with diffusion or PME, p in [1, 8]; dim 3
 * with diffusion, p in [1, 6]; dim 3 Navier-Stokes, p in [1, 6] (FP64) or
 * [1, 7] (FP32, BF16x3); anything else returns SD_EUNSUPPORTED.
 * stream: a hipStream_t (NULL = the default stream).  Allocates the
 * operators and the scratch buffers (face traces, RK registers) on the
 * current device; the context owns them until sd_free. */
int sd_init(const sd_mesh *mesh, int p, int scheme, const sd_params *prm,
            void *stream, sd_ctx **out);

/* Release every resource of the context (waits for its stream). NULL is ok. */
int sd_free(sd_ctx *ctx);

/* Change the stream later calls are enqueued on. */
int sd_set_stream(sd_ctx *ctx, void *stream);

/* Number of FP64 values of one state: ne * nv * n^dim. */
long long sd_state_size(const sd_ctx *ctx);

/* dudt = R(u): the semi-discrete right-hand side at the solution points.
 * u and dudt are device pointers of sd_state_size() doubles each and must
 * not overlap.  u is read only. */
int sd_rhs(sd_ctx *ctx, const double *u, double *dudt);

/* One time step of size dt, in place on the device state u, with the
 * integrator of sd_params.integrator (classical RK4, or SSP-RK(5,4)); the
 * stage combinations and the accumulation are FP64 (with RK4 in FP32 or
 * BF16x3, the intermediate stage states are kept as the compute-precision
 * values the RHS would round them to). */
int sd_rk_step(sd_ctx *ctx, double *u, double dt);

/* nsteps time steps of size dt, in place on the device state u: the state
 * of nsteps calls of sd_rk_step (to the last bit of a value, where the
 * compiler fuses a product and a sum differently in the one-launch kernel
 * and the separate ones).  A one-dimensional FP64
 * problem of linear diffusion or the porous medium equation (section 3)
 * with classical RK4, n = p + 1 <= 8 and at most 2048 solution points runs
 * the whole run in one launch of one block, the mesh held in on-chip memory
 * (such meshes give the separate kernels of a step too little work to be
 * anything but launch bound); every other context takes the steps one by
 * one.  nsteps < 0 or a non-finite dt: SD_EINVAL; nsteps = 0 does nothing.
 * The one-launch run records no sd_timing events. */
int sd_rk_run(sd_ctx *ctx, double *u, double dt, long long nsteps);

/* Diagnostics of a Navier-Stokes state (FP64 reductions, deterministic):
 * waits for the stream and fills the host struct *out.  Returns
 * SD_ENONFINITE (with *out filled) when the state holds NaN or Inf. */
int sd_diagnostics(sd_ctx *ctx, const double *u, sd_diag *out);

/* Largest stable time step of a Navier-Stokes state for the convective
 * limit (section 4.4's TGV runs): *dt = cfl * min_d h_d / ((p + 1) smax),
 * smax from sd_diagnostics of u (this call waits for the stream).  cfl is
 * the Courant number (0.3 in the TGV runs; > 0 and finite, else SD_EINVAL).
 * The viscous limit is not included.  Returns SD_ENONFINITE, *dt untouched,
 * when the state is non-finite, has rho <= 0 or P < 0 somewhere, or has no
 * positive signal speed; SD_EUNSUPPORTED for scalar physics. */
int sd_stable_dt(sd_ctx *ctx, const double *u, double cfl, double *dt);

/* Curvilinear hexahedra (section 2.3: q = J u, G = S.F, H = S^T u with
 * S = adj(dx/dxi)) for a 3-D diffusion or Navier-Stokes context in FP64 or
 * FP32 (SD_FP32: the metric terms are stored and used in FP32, and the
 * Navier-Stokes reference state is removed before the rounding as on
 * Cartesian meshes; the state and the RHS stay FP64 in memory).
 * Navier-Stokes (p <= 5): G_d = S_d . (F_c - F_v) at the flux points of
 * family d; at a face the Roe flux along n = S_d / |S_d| times |S_d| (the
 * Harten fix as on Cartesian meshes) minus S_d . F_v of the averaged
 * solution and gradient; the gradient of every conservative variable is the
 * auxiliary variable of the scalar case.  Diagnostics, sd_stable_dt, the
 * closure and the interior penalty stay Cartesian-only on such a context
 * (SD_EUNSUPPORTED).  nodes: HOST array
 * [ne][q+1][q+1][q+1][3] (copied), the coordinates of q + 1 equispaced
 * nodes per direction of every element (ends included, the first index
 * along zeta, the last along xi), q = 1 or 2; element e keeps its place in
 * the structured periodic connectivity of the mesh given to sd_init (the
 * box lo/hi is no longer used), and shared faces must carry the same nodes.
 * The library evaluates S at the flux points and 1/det J at the solution
 * points, stores them on the device (about 9(p+2)(p+1)^2 + (p+1)^3 doubles
 * per element) and from then on sd_rhs and sd_rk_step use them.  Constants
 * are preserved exactly when 2q <= p + 1.  Returns SD_EINVAL for a null
 * argument, q outside {1, 2} or an element whose det J is not positive at
 * a solution point (or, with the interior penalty on, at a face point);
 * SD_EUNSUPPORTED for other physics, dimensions or precisions (BF16x3,
 * FP32 matrix cores), for
 * Navier-Stokes at p > 5 or with the interior penalty, and for a context
 * whose closure is set; SD_ENOMEM /
 * SD_EHIP on device failures.  With eta_ip > 0 the penalty uses, at each
 * face point, 1/h = |S_d| max(J^-1 of the two sides) / 2 (on an affine
 * Cartesian element the 2/h_d of the box) and acts along n = S_d / |S_d|.
 * Calling it again replaces the geometry. */
int sd_set_geometry(sd_ctx *ctx, const double *nodes, int q);

/* Timing of the right-hand side kernels: with enable = 1 every later RHS
 * evaluation of the context (sd_rhs and the four inside sd_rk_step) is
 * bracketed by a pair of HIP events on the context's stream (up to 4096
 * evaluations; later ones go untimed); enable = 0 stops recording.
 * sd_timing_read waits for the stream and returns the summed elapsed time
 * (ms) and the number of timed evaluations since the last enable. */
int sd_timing(sd_ctx *ctx, int enable);
int sd_timing_read(sd_ctx *ctx, double *total_ms, long long *count);

/* Message of the last error on this thread ("" if none). */
const char *sd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SD_H */
