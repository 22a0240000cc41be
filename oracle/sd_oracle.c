/*
 * Plain FP64 CPU oracle for the SD right-hand side (standard BR1 and compact
 * second-order fluxes).  TEST INFRASTRUCTURE ONLY: see sd_oracle.h.
 *
 * Every function below follows a passage of the paper:
 *   - operators: section 2.1, Lagrange bases (eq. lagr:poly), the
 *     interpolation matrix (eq. Lmat), the differentiation matrix (eq. Mmat)
 *     and the log-derivative identity of its footnote;
 *   - the 1-D standard scheme: section 2.1, steps 1-5 (eqs. c:flux, w:e,
 *     v:e, c:aux:v, aux:v:int), interface flux option (a);
 *   - the 1-D compact scheme: section 2.2 (eqs. c:flux:l, c:flux:r, v:s:l,
 *     v:s:r, cmp:int:fp, cmp:int:avg);
 *   - multi-D: section 2.3 (eqs. int:2d, c:sol:2d:xi/eta, aux:v:std:2d,
 *     aux:v:cmp:l..t, aux:cmp:lr:2d, aux:cmp:bt:2d, c:aux:v:2d) extended to
 *     three directions, with the mapped system (eqs. ns:mapped, adj:f);
 *   - Navier-Stokes: section 4.4 (convective and viscous fluxes, constitutive
 *     relations, Roe flux with entropy fix at interfaces, centred viscous flux
 *     on averaged solution and gradient, gradients of conservative variables).
 * The one-sided fluxes H^{C,L}, H^{C,R} are built explicitly (first form of
 * eqs. c:flux:l/r), never through the correction shortcut, so that elements
 * outside the stencil see bit-identical inputs.
 */
#include "sd_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Operators (section 2.1)                                                  */
/* ------------------------------------------------------------------------ */

/* Legendre polynomial P_n(x) and its derivative by the three-term recurrence. */
static void legendre(int n, double x, double *P, double *dP) {
  double pm1 = 1.0, pk = x;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    double pn = ((2.0 * k - 1.0) * x * pk - (k - 1.0) * pm1) / k;
    pm1 = pk;
    pk = pn;
  }
  *P = pk;
  *dP = n * (x * pk - pm1) / (x * x - 1.0);
}

/* n-point Gauss-Legendre rule by Newton iteration on P_n, sorted ascending. */
int or_gauss_legendre(int n, double *x, double *w) {
  if (n < 1 || n > 64) return -1;
  for (int i = 0; i < n; ++i) {
    double z = cos(M_PI * (i + 0.75) / (n + 0.5));
    double P, dP;
    for (int it = 0; it < 100; ++it) {
      legendre(n, z, &P, &dP);
      double dz = P / dP;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    legendre(n, z, &P, &dP);
    x[n - 1 - i] = z;                       /* roots come out descending */
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dP * dP);
  }
  return 0;
}

/* Lagrange basis on the nodes pts[0..np-1], basis index j, evaluated at x
 * (eq. lagr:poly). */
static double lagrange(const double *pts, int np, int j, double x) {
  double r = 1.0;
  for (int k = 0; k < np; ++k)
    if (k != j) r *= (x - pts[k]) / (pts[j] - pts[k]);
  return r;
}

int or_operators(int p, double *xs, double *ws, double *xf, double *L, double *M) {
  int n = p + 1;
  if (p < 1 || n > OR_MAXN) return -1;
  /* solution points: n-point Gauss-Legendre; flux points: the ends plus the
     (n-1)-point Gauss-Legendre rule (section 2). */
  or_gauss_legendre(n, xs, ws);
  double tmpx[OR_MAXN], tmpw[OR_MAXN];
  or_gauss_legendre(n - 1, tmpx, tmpw);
  xf[0] = -1.0;
  for (int i = 0; i < n - 1; ++i) xf[i + 1] = tmpx[i];
  xf[n] = 1.0;
  /* L_ij = l_j(xi_{i-1/2}) (eq. Lmat) */
  for (int i = 0; i <= n; ++i)
    for (int j = 0; j < n; ++j) L[i * n + j] = lagrange(xs, n, j, xf[i]);
  /* M_ij = d/dxi l_{j-1/2}(xi_i), through the footnote's identity
     l'(x) = l(x) * sum_{k != j} 1 / (x - x_k); solution and flux points never
     coincide (the two Gauss-Legendre rules interlace). */
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= n; ++j) {
      double s = 0.0;
      for (int k = 0; k <= n; ++k)
        if (k != j) s += 1.0 / (xs[i] - xf[k]);
      M[i * (n + 1) + j] = lagrange(xf, n + 1, j, xs[i]) * s;
    }
  return 0;
}

/* integer power for the porous-medium diffusivity m u^{m-1} */
static double ipow(double u, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= u;
  return r;
}

/* scalar flux law F(u, v): -nu v (diffusion) or -m u^{m-1} v (PME,
   eq. pme, non-linear term taken from the flux-point solution) */
static double scalar_flux(int physics, double coef, double u, double v) {
  if (physics == OR_PME) {
    int m = (int)coef;
    return -coef * ipow(u, m - 1) * v;
  }
  return -coef * v;
}

/* ------------------------------------------------------------------------ */
/* 1-D scheme (sections 2.1 and 2.2)                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
  int N, n, scheme, physics;
  double coef, J, tau;
  double L[(OR_MAXN + 1) * OR_MAXN], M[OR_MAXN * (OR_MAXN + 1)];
  const double *u;
} ctx1;

static int wrap(int e, int N) { return ((e % N) + N) % N; }

/* u^F_x = L u^S_x */
static void c1_uF(const ctx1 *c, int x, double *uF) {
  int n = c->n;
  const double *uS = c->u + (long)wrap(x, c->N) * n;
  for (int i = 0; i <= n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += c->L[i * n + j] * uS[j];
    uF[i] = s;
  }
}

/* common values H^L_x, H^R_x = (u_L + u_R)/2 at the two interfaces of x */
static void c1_hat(const ctx1 *c, int x, double *hL, double *hR) {
  int n = c->n;
  double a[OR_MAXN + 1], b[OR_MAXN + 1], d[OR_MAXN + 1];
  c1_uF(c, x - 1, a);
  c1_uF(c, x, b);
  c1_uF(c, x + 1, d);
  *hL = 0.5 * (a[n] + b[0]);
  *hR = 0.5 * (b[n] + d[0]);
}

/* continuous flux H with the chosen ends corrected: both (eq. c:flux),
   left only (H^{C,L}, eq. c:flux:l) or right only (H^{C,R}, eq. c:flux:r) */
static void c1_H(const ctx1 *c, int x, int corrL, int corrR, double *H) {
  int n = c->n;
  double hL, hR;
  c1_uF(c, x, H);
  c1_hat(c, x, &hL, &hR);
  if (corrL) H[0] = hL;
  if (corrR) H[n] = hR;
}

/* v^S = J^{-1} M H (eq. w:e and eqs. v:s:l/r with the matching H) */
static void c1_vS(const ctx1 *c, const double *H, double *vS) {
  int n = c->n;
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j <= n; ++j) s += c->M[i * (n + 1) + j] * H[j];
    vS[i] = s / c->J;
  }
}

/* v^F = L v^S (eq. v:e) */
static void c1_interp(const ctx1 *c, const double *vS, double *vF) {
  int n = c->n;
  for (int i = 0; i <= n; ++i) {
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += c->L[i * n + j] * vS[j];
    vF[i] = s;
  }
}

/* gradient value that element x contributes at its left (side 0) or right
   (side 1) interface: standard v^F end (BR1) or the one-sided value of
   eq. cmp:int:fp (compact) */
static double c1_face_grad(const ctx1 *c, int x, int side) {
  int n = c->n;
  double H[OR_MAXN + 1], vS[OR_MAXN], vF[OR_MAXN + 1];
  if (c->scheme == OR_COMPACT)
    c1_H(c, x, side == 0, side == 1, H);
  else
    c1_H(c, x, 1, 1, H);
  c1_vS(c, H, vS);
  c1_interp(c, vS, vF);
  return side == 0 ? vF[0] : vF[n];
}

static void c1_rhs_elem(const ctx1 *c, int e, double *out) {
  int n = c->n;
  double HC[OR_MAXN + 1], vS[OR_MAXN], vFC[OR_MAXN + 1], G[OR_MAXN + 1];
  /* steps 1-3: continuous solution, gradient at solution points, v^F */
  c1_H(c, e, 1, 1, HC);
  c1_vS(c, HC, vS);
  c1_interp(c, vS, vFC);
  /* step 4: common gradient at the interfaces, eq. aux:v:int (BR1) or
     eq. cmp:int:avg (compact); interior flux points keep v^F */
  vFC[0] = 0.5 * (c1_face_grad(c, e - 1, 1) + c1_face_grad(c, e, 0));
  vFC[n] = 0.5 * (c1_face_grad(c, e, 1) + c1_face_grad(c, e + 1, 0));
  if (c->tau != 0.0) {
    /* interior penalty (section 3): v_hat += tau (u_R - u_L) at each interface */
    double a[OR_MAXN + 1], b[OR_MAXN + 1], d[OR_MAXN + 1];
    c1_uF(c, e - 1, a);
    c1_uF(c, e, b);
    c1_uF(c, e + 1, d);
    vFC[0] += c->tau * (b[0] - a[n]);
    vFC[n] += c->tau * (d[0] - b[n]);
  }
  /* flux G = F(u^{F,C}, v^{F,C}) at every flux point; at the interfaces
     this is option (a): G(H_hat, v_hat) */
  for (int i = 0; i <= n; ++i) G[i] = scalar_flux(c->physics, c->coef, HC[i], vFC[i]);
  /* step 5: dq/dt = -M G, u = J^{-1} q  (S = 1 in 1-D) */
  for (int i = 0; i < n; ++i) {
    double s = 0.0;
    for (int j = 0; j <= n; ++j) s += c->M[i * (n + 1) + j] * G[j];
    out[i] = -s / c->J;
  }
}

static int c1_setup(ctx1 *c, int N, int p, double x0, double x1, int scheme,
                    int physics, double coef, double eta_ip, const double *u) {
  double xs[OR_MAXN], ws[OR_MAXN], xf[OR_MAXN + 1];
  if (N < 1 || p < 1 || p + 1 > OR_MAXN || !(x1 > x0)) return -1;
  if (scheme != OR_BR1 && scheme != OR_COMPACT) return -1;
  if (physics != OR_DIFFUSION && physics != OR_PME) return -1;
  if (physics == OR_PME && (coef < 1.0 || coef != floor(coef))) return -1;
  c->N = N; c->n = p + 1; c->scheme = scheme; c->physics = physics; c->coef = coef;
  c->J = 0.5 * (x1 - x0) / N;      /* J_e = (x_{e+1} - x_e)/2, S_e = 1 */
  if (!(eta_ip >= 0.0)) return -1;
  c->tau = eta_ip * (double)(p + 1) * (double)(p + 1) / (2.0 * c->J);   /* h = element size */
  c->u = u;
  return or_operators(p, xs, ws, xf, c->L, c->M);
}

int or_rhs_1d(int N, int p, double x0, double x1, int scheme, int physics,
              double coef, double eta_ip, const double *u, double *dudt) {
  ctx1 c;
  if (c1_setup(&c, N, p, x0, x1, scheme, physics, coef, eta_ip, u)) return -1;
  for (int e = 0; e < N; ++e) c1_rhs_elem(&c, e, dudt + (long)e * c.n);
  return 0;
}

int or_rk4_1d(int N, int p, double x0, double x1, int scheme, int physics,
              double coef, double eta_ip, double *u, double dt, int nsteps) {
  long sz = (long)N * (p + 1);
  double *k = malloc(sizeof(double) * sz * 5);
  if (!k) return -2;
  double *k1 = k, *k2 = k + sz, *k3 = k + 2 * sz, *k4 = k + 3 * sz, *w = k + 4 * sz;
  int rc = 0;
  for (int s = 0; s < nsteps && !rc; ++s) {
    rc |= or_rhs_1d(N, p, x0, x1, scheme, physics, coef, eta_ip, u, k1);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + 0.5 * dt * k1[i];
    rc |= or_rhs_1d(N, p, x0, x1, scheme, physics, coef, eta_ip, w, k2);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + 0.5 * dt * k2[i];
    rc |= or_rhs_1d(N, p, x0, x1, scheme, physics, coef, eta_ip, w, k3);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + dt * k3[i];
    rc |= or_rhs_1d(N, p, x0, x1, scheme, physics, coef, eta_ip, w, k4);
    for (long i = 0; i < sz; ++i)
      u[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  free(k);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Navier-Stokes pointwise laws (section 4.4)                               */
/* ------------------------------------------------------------------------ */

static double ns_p0(const or_params *q) {
  return q->rho0 / q->gamma * (q->u0 / q->Ma) * (q->u0 / q->Ma);
}

/* Sutherland's law mu(T), reference temperature T0 = p0 / (rho0 R), R = 1 */
static double ns_mu(const or_params *q, double T) {
  double mu0 = q->rho0 * q->u0 * q->Lref / q->Re;
  if (q->sutherland_s < 0.0) return mu0;
  double T0 = ns_p0(q) / q->rho0;
  double th = T / T0;
  return mu0 * th * sqrt(th) * (1.0 + q->sutherland_s) / (th + q->sutherland_s);
}

/* F_c e_d: (rho u_d, rho u u_d + P e_d, (rho E + P) u_d) */
void or_ns_flux_conv(const or_params *q, const double *U, int d, double *F) {
  double rho = U[0];
  double u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  double P = (q->gamma - 1.0) * (U[4] - 0.5 * rho * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]));
  F[0] = U[1 + d];
  for (int i = 0; i < 3; ++i) F[1 + i] = U[1 + i] * u[d] + (i == d ? P : 0.0);
  F[4] = (U[4] + P) * u[d];
}

/* F_v e_d = (0, tau e_d, u . tau e_d + kappa dT/dx_d), tau = mu (grad u +
   grad u^T) + lambda (div u) I, kappa = mu C_p / Pr, T = P / (rho R), R = 1;
   primitive gradients from the conservative ones G[v*3 + m] */
void or_ns_flux_visc(const or_params *q, const double *U, const double *G, int d,
                     double *F) {
  double g = q->gamma, rho = U[0];
  double u[3] = {U[1] / rho, U[2] / rho, U[3] / rho};
  double E = U[4] / rho;
  double ke = 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
  double T = (g - 1.0) * (E - ke);
  double du[3][3], dT[3];
  for (int m = 0; m < 3; ++m) {
    double drho = G[0 * 3 + m];
    for (int i = 0; i < 3; ++i) du[i][m] = (G[(1 + i) * 3 + m] - u[i] * drho) / rho;
    double dE = (G[4 * 3 + m] - E * drho) / rho;
    dT[m] = (g - 1.0) * (dE - (u[0] * du[0][m] + u[1] * du[1][m] + u[2] * du[2][m]));
  }
  double mu = ns_mu(q, T);
  double lam = q->lambda_over_mu * mu;
  double kappa = mu * (g / (g - 1.0)) / q->Pr;
  double div = du[0][0] + du[1][1] + du[2][2];
  double tau[3];
  for (int i = 0; i < 3; ++i) tau[i] = mu * (du[i][d] + du[d][i]) + (i == d ? lam * div : 0.0);
  F[0] = 0.0;
  for (int i = 0; i < 3; ++i) F[1 + i] = tau[i];
  F[4] = u[0] * tau[0] + u[1] * tau[1] + u[2] * tau[2] + kappa * dT[d];
}

/* Roe-averaged state and wave decomposition along e_d; ws[k] are the wave
   speeds, the dissipation is sum_k f(ws[k]) * (wave k). */
static void roe_waves(const or_params *q, const double *UL, const double *UR, int d,
                      int use_abs, int fix, double *D) {
  double g = q->gamma;
  double rL = UL[0], rR = UR[0];
  double uL[3], uR[3], ut[3], du[3];
  for (int i = 0; i < 3; ++i) { uL[i] = UL[1 + i] / rL; uR[i] = UR[1 + i] / rR; }
  double pL = (g - 1.0) * (UL[4] - 0.5 * rL * (uL[0] * uL[0] + uL[1] * uL[1] + uL[2] * uL[2]));
  double pR = (g - 1.0) * (UR[4] - 0.5 * rR * (uR[0] * uR[0] + uR[1] * uR[1] + uR[2] * uR[2]));
  double HL = (UL[4] + pL) / rL, HR = (UR[4] + pR) / rR;
  double sL = sqrt(rL), sR = sqrt(rR);
  for (int i = 0; i < 3; ++i) ut[i] = (sL * uL[i] + sR * uR[i]) / (sL + sR);
  double Ht = (sL * HL + sR * HR) / (sL + sR);
  double rt = sL * sR;
  double q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  double c2 = (g - 1.0) * (Ht - 0.5 * q2);
  double c = sqrt(c2);
  double un = ut[d];
  for (int i = 0; i < 3; ++i) du[i] = uR[i] - uL[i];
  double drho = rR - rL, dp = pR - pL, dun = du[d];
  double a1 = (dp - rt * c * dun) / (2.0 * c2);
  double a5 = (dp + rt * c * dun) / (2.0 * c2);
  double a2 = drho - dp / c2;
  double l1 = un - c, l2 = un, l5 = un + c;
  if (use_abs) {
    l1 = fabs(l1); l2 = fabs(l2); l5 = fabs(l5);
    if (fix) {
      /* Harten's fix on the two acoustic (genuinely non-linear) fields */
      double delta = q->entropy_fix * (fabs(un) + c);
      if (delta > 0.0) {
        if (l1 < delta) l1 = (l1 * l1 + delta * delta) / (2.0 * delta);
        if (l5 < delta) l5 = (l5 * l5 + delta * delta) / (2.0 * delta);
      }
    }
  }
  /* acoustic waves r1, r5 */
  double r1[5], r5[5], r2[5], rs[5];
  r1[0] = 1.0; r5[0] = 1.0;
  for (int i = 0; i < 3; ++i) {
    r1[1 + i] = ut[i] - (i == d ? c : 0.0);
    r5[1 + i] = ut[i] + (i == d ? c : 0.0);
  }
  r1[4] = Ht - c * un;
  r5[4] = Ht + c * un;
  /* entropy wave and the two shear waves (tangential velocity jump) */
  r2[0] = 1.0;
  for (int i = 0; i < 3; ++i) r2[1 + i] = ut[i];
  r2[4] = 0.5 * q2;
  double dut[3];
  for (int i = 0; i < 3; ++i) dut[i] = du[i] - (i == d ? dun : 0.0);
  rs[0] = 0.0;
  for (int i = 0; i < 3; ++i) rs[1 + i] = rt * dut[i];
  rs[4] = rt * (ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2]);
  for (int k = 0; k < 5; ++k)
    D[k] = l1 * a1 * r1[k] + l2 * (a2 * r2[k] + rs[k]) + l5 * a5 * r5[k];
}

/* Roe flux with Harten's entropy fix: (F(UL) + F(UR))/2 - |A~| (UR - UL)/2 */
void or_ns_roe(const or_params *q, const double *UL, const double *UR, int d, double *F) {
  double FL[5], FR[5], D[5];
  or_ns_flux_conv(q, UL, d, FL);
  or_ns_flux_conv(q, UR, d, FR);
  roe_waves(q, UL, UR, d, 1, 1, D);
  for (int k = 0; k < 5; ++k) F[k] = 0.5 * (FL[k] + FR[k]) - 0.5 * D[k];
}

void or_ns_roe_signed_waves(const or_params *q, const double *UL, const double *UR,
                            int d, double *D) {
  roe_waves(q, UL, UR, d, 0, 0, D);
}

/* ------------------------------------------------------------------------ */
/* 3-D scheme (section 2.3, three directions)                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  int nel[3], n, nv, scheme;
  or_params prm;
  double h[3], J, S[3][3];
  double L[(OR_MAXN + 1) * OR_MAXN], M[OR_MAXN * (OR_MAXN + 1)];
  double ws[OR_MAXN];
  const double *u;
} ctx3;

static long c3_index(const ctx3 *c, int ex, int ey, int ez) {
  ex = wrap(ex, c->nel[0]);
  ey = wrap(ey, c->nel[1]);
  ez = wrap(ez, c->nel[2]);
  return ex + (long)c->nel[0] * (ey + (long)c->nel[1] * ez);
}

static void c3_coords(const ctx3 *c, long e, int *ex) {
  ex[0] = (int)(e % c->nel[0]);
  ex[1] = (int)((e / c->nel[0]) % c->nel[1]);
  ex[2] = (int)(e / ((long)c->nel[0] * c->nel[1]));
}

/* neighbour of e across its face (d, s): s = 0 towards -x_d, s = 1 towards +x_d */
static long c3_nbr(const ctx3 *c, long e, int d, int s) {
  int ex[3];
  c3_coords(c, e, ex);
  ex[d] += s ? 1 : -1;
  return c3_index(c, ex[0], ex[1], ex[2]);
}

/* extents of a family-d array (n + 1 points along d, n along the others) */
static void fam_ext(const ctx3 *c, int d, int *ext) {
  ext[0] = ext[1] = ext[2] = c->n;
  if (d >= 0) ext[d] = c->n + 1;
}

static long aidx(const int *ext, int v, int i, int j, int k) {
  return (((long)v * ext[2] + k) * ext[1] + j) * ext[0] + i;
}

/* out = Op applied along axis d of in (rows x cols operator, cols = extent of
   in along d); the other axes keep their extent; nv variables */
static void apply_axis(const double *Op, int rows, int cols, int d, int nv,
                       const int *ein, const double *in, double *out) {
  int eo[3] = {ein[0], ein[1], ein[2]};
  eo[d] = rows;
  for (int v = 0; v < nv; ++v)
    for (int k = 0; k < eo[2]; ++k)
      for (int j = 0; j < eo[1]; ++j)
        for (int i = 0; i < eo[0]; ++i) {
          int o[3] = {i, j, k};
          double s = 0.0;
          for (int t = 0; t < cols; ++t) {
            int a[3] = {i, j, k};
            a[d] = t;
            s += Op[o[d] * cols + t] * in[aidx(ein, v, a[0], a[1], a[2])];
          }
          out[aidx(eo, v, i, j, k)] = s;
        }
}

/* u^{Fd}_x: solution interpolated to the family-d flux points (eq. int:2d) */
static void c3_uF(const ctx3 *c, long x, int d, double *UF) {
  int es[3] = {c->n, c->n, c->n};
  long n3 = (long)c->n * c->n * c->n;
  apply_axis(c->L, c->n + 1, c->n, d, c->nv, es, c->u + x * c->nv * n3, UF);
}

/* u^{Fd} of x with its left end (corrL) and/or right end (corrR) replaced by
   the common value (u_left + u_right)/2 of eqs. c:sol:2d:xi/eta:
   both -> u^{Fd,C}; left only -> u^{Fd,L}; right only -> u^{Fd,R} */
static void c3_uFcont(const ctx3 *c, long x, int d, int corrL, int corrR, double *UF,
                      double *tmp) {
  int ext[3];
  fam_ext(c, d, ext);
  int n = c->n;
  c3_uF(c, x, d, UF);
  for (int side = 0; side < 2; ++side) {
    if ((side == 0 && !corrL) || (side == 1 && !corrR)) continue;
    c3_uF(c, c3_nbr(c, x, d, side), d, tmp);
    int mine = side == 0 ? 0 : n, theirs = side == 0 ? n : 0;
    for (int v = 0; v < c->nv; ++v)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          int im[3], it[3], o = 0;
          for (int ax = 0; ax < 3; ++ax) {
            if (ax == d) { im[ax] = mine; it[ax] = theirs; }
            else { im[ax] = it[ax] = (o == 0 ? a : b); ++o; }
          }
          long pm = aidx(ext, v, im[0], im[1], im[2]);
          long pt = aidx(ext, v, it[0], it[1], it[2]);
          UF[pm] = 0.5 * (UF[pm] + tmp[pt]);
        }
  }
}

/* auxiliary gradient at the solution points, v^S_m = [J^-1] (sum_d M_d
   (u^{Fd,X} S_{dm})), with X = C in every direction (standard,
   eq. aux:v:std:2d) or, for the one-sided variant of face (dd, ss),
   X = L or R along dd and C elsewhere (eqs. aux:v:cmp:l..t).
   vS layout: [m][v][k][j][i]. */
static void c3_vS(const ctx3 *c, long x, int dd, int ss, double *vS, double *UF,
                  double *tmp, double *H, double *dH) {
  int n = c->n, nv = c->nv;
  long n3 = (long)n * n * n;
  int es[3] = {n, n, n};
  for (long i = 0; i < 3 * nv * n3; ++i) vS[i] = 0.0;
  for (int d = 0; d < 3; ++d) {
    int ext[3];
    fam_ext(c, d, ext);
    long nf = (long)nv * ext[0] * ext[1] * ext[2];
    if (d == dd)
      c3_uFcont(c, x, d, ss == 0, ss == 1, UF, tmp);
    else
      c3_uFcont(c, x, d, 1, 1, UF, tmp);
    for (int m = 0; m < 3; ++m) {
      if (c->S[d][m] == 0.0) continue;          /* H^{Fd}_m = u^{Fd} S_{dm} = 0 */
      for (long i = 0; i < nf; ++i) H[i] = UF[i] * c->S[d][m];
      apply_axis(c->M, n, n + 1, d, nv, ext, H, dH);
      for (long i = 0; i < nv * n3; ++i) vS[m * nv * n3 + i] += dH[i];
    }
    (void)es;
  }
  for (long i = 0; i < 3 * nv * n3; ++i) vS[i] /= c->J;
}

/* gradient values that element x contributes at its face (d, s): all 3*nv
   components at the n*n face points, layout [m][v][a][b] with (a, b) the
   transverse axes in increasing order.  Standard (BR1): end of L_d v^S.
   Compact: end of L_d v^{S,side} (eqs. aux:cmp:lr:2d, aux:cmp:bt:2d). */
static void c3_face_grad(const ctx3 *c, long x, int d, int s, double *out, double *vS,
                         double *UF, double *tmp, double *H, double *dH) {
  int n = c->n, nv = c->nv;
  long n3 = (long)n * n * n;
  int es[3] = {n, n, n}, ext[3];
  fam_ext(c, d, ext);
  if (c->scheme == OR_COMPACT)
    c3_vS(c, x, d, s, vS, UF, tmp, H, dH);
  else
    c3_vS(c, x, -1, -1, vS, UF, tmp, H, dH);
  int end = s == 0 ? 0 : n;
  for (int m = 0; m < 3; ++m) {
    apply_axis(c->L, n + 1, n, d, nv, es, vS + m * nv * n3, H);
    for (int v = 0; v < nv; ++v)
      for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
          int id[3], o = 0;
          for (int ax = 0; ax < 3; ++ax) id[ax] = (ax == d) ? end : (o++ == 0 ? a : b);
          out[(((long)m * nv + v) * n + a) * n + b] = H[aidx(ext, v, id[0], id[1], id[2])];
        }
  }
}

typedef struct {
  double *UF, *tmp, *H, *dH, *vS, *vS2, *fg1, *fg2;
  double *UFC[3], *VF[3], *G[3], *UFraw, *UFnb, *UFnb2;
} work3;

static int work3_alloc(const ctx3 *c, work3 *w) {
  int n = c->n, nv = c->nv;
  long nfam = (long)nv * (n + 1) * n * n;
  long n3 = (long)n * n * n;
  long tot = 4 * nfam + 2 * 3 * nv * n3 + 2 * 3 * nv * n * n + 3 * nfam + 3 * 3 * nfam +
             3 * nfam + 3 * nfam;
  double *b = malloc(sizeof(double) * tot);
  if (!b) return -1;
  memset(b, 0, sizeof(double) * tot);
  w->UF = b; b += nfam;
  w->tmp = b; b += nfam;
  w->H = b; b += nfam;
  w->dH = b; b += nfam;
  w->vS = b; b += 3 * nv * n3;
  w->vS2 = b; b += 3 * nv * n3;
  w->fg1 = b; b += 3 * nv * n * n;
  w->fg2 = b; b += 3 * nv * n * n;
  for (int d = 0; d < 3; ++d) { w->UFC[d] = b; b += nfam; }
  for (int d = 0; d < 3; ++d) { w->VF[d] = b; b += 3 * nfam; }
  for (int d = 0; d < 3; ++d) { w->G[d] = b; b += nfam; }
  w->UFraw = b; b += nfam;
  w->UFnb = b; b += nfam;
  w->UFnb2 = b; b += nfam;
  return 0;
}

/* flux G_d = sum_m S_dm F_m(U, V) at one flux point (scalar physics or the
   Navier-Stokes F_c - F_v); U[nv], V[m*nv + v] */
static void c3_point_flux(const ctx3 *c, int d, const double *U, const double *V,
                          double *Gd) {
  int nv = c->nv;
  for (int v = 0; v < nv; ++v) Gd[v] = 0.0;
  for (int m = 0; m < 3; ++m) {
    if (c->S[d][m] == 0.0) continue;
    if (c->prm.physics == OR_NAVIER_STOKES) {
      double Fc[5], Fv[5], Gc[15];
      for (int v = 0; v < 5; ++v)
        for (int mm = 0; mm < 3; ++mm) Gc[v * 3 + mm] = V[mm * 5 + v];
      or_ns_flux_conv(&c->prm, U, m, Fc);
      or_ns_flux_visc(&c->prm, U, Gc, m, Fv);
      for (int v = 0; v < 5; ++v) Gd[v] += c->S[d][m] * (Fc[v] - Fv[v]);
    } else {
      double coef = c->prm.physics == OR_PME ? c->prm.pme_m : c->prm.nu;
      Gd[0] += c->S[d][m] * scalar_flux(c->prm.physics, coef, U[0], V[m]);
    }
  }
}

static void c3_rhs_elem(const ctx3 *c, long e, double *out, work3 *w) {
  int n = c->n, nv = c->nv;
  long n3 = (long)n * n * n;
  int es[3] = {n, n, n};
  /* step 2: continuous solution u^{Fd,C} for the three families */
  for (int d = 0; d < 3; ++d) c3_uFcont(c, e, d, 1, 1, w->UFC[d], w->tmp);
  /* step 3: standard gradient at the solution points, then at the interior
     flux points of every family (eq. aux:v:std:2d) */
  c3_vS(c, e, -1, -1, w->vS, w->UF, w->tmp, w->H, w->dH);
  for (int d = 0; d < 3; ++d) {
    int ext[3];
    fam_ext(c, d, ext);
    long nf = (long)nv * ext[0] * ext[1] * ext[2];
    for (int m = 0; m < 3; ++m)
      apply_axis(c->L, n + 1, n, d, nv, es, w->vS + m * nv * n3, w->VF[d] + m * nf);
  }
  /* step 4: common interface gradient from the two sides' face values
     (eq. c:aux:v:2d with aux:v:int (BR1) or the one-sided values) */
  for (int d = 0; d < 3; ++d) {
    int ext[3];
    fam_ext(c, d, ext);
    long nf = (long)nv * ext[0] * ext[1] * ext[2];
    /* interior penalty (section 3): the normal component gains
       tau_d (u_R - u_L), tau_d = eta_ip (p+1)^2 / h_d */
    const double tau = c->prm.eta_ip * (double)n * (double)n / c->h[d];
    for (int s = 0; s < 2; ++s) {
      long nb = c3_nbr(c, e, d, s);
      c3_face_grad(c, e, d, s, w->fg1, w->vS2, w->UF, w->tmp, w->H, w->dH);
      c3_face_grad(c, nb, d, 1 - s, w->fg2, w->vS2, w->UF, w->tmp, w->H, w->dH);
      if (tau != 0.0) {
        c3_uF(c, e, d, w->UFraw);
        c3_uF(c, nb, d, w->UFnb);
      }
      int end = s == 0 ? 0 : n;
      for (int m = 0; m < 3; ++m)
        for (int v = 0; v < nv; ++v)
          for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
              int id[3], o = 0;
              for (int ax = 0; ax < 3; ++ax) id[ax] = (ax == d) ? end : (o++ == 0 ? a : b);
              long f = (((long)m * nv + v) * n + a) * n + b;
              /* left element's value first, as in eq. cmp:int:avg */
              double lv = s == 0 ? w->fg2[f] : w->fg1[f];
              double rv = s == 0 ? w->fg1[f] : w->fg2[f];
              double vh = 0.5 * (lv + rv);
              if (tau != 0.0 && m == d) {
                int io[3] = {id[0], id[1], id[2]};
                io[d] = s == 0 ? n : 0;              /* the neighbour's end */
                double uo = w->UFraw[aidx(ext, v, id[0], id[1], id[2])];
                double un = w->UFnb[aidx(ext, v, io[0], io[1], io[2])];
                vh += tau * (s == 0 ? uo - un : un - uo);
              }
              w->VF[d][m * nf + aidx(ext, v, id[0], id[1], id[2])] = vh;
            }
    }
  }
  /* flux at every flux point of every family */
  for (int d = 0; d < 3; ++d) {
    int ext[3];
    fam_ext(c, d, ext);
    long nf = (long)nv * ext[0] * ext[1] * ext[2];
    long npts = (long)ext[0] * ext[1] * ext[2];
    if (c->prm.physics == OR_NAVIER_STOKES) {
      c3_uF(c, e, d, w->UFraw);
      c3_uF(c, c3_nbr(c, e, d, 0), d, w->UFnb);
      c3_uF(c, c3_nbr(c, e, d, 1), d, w->UFnb2);
    }
    for (int k = 0; k < ext[2]; ++k)
      for (int j = 0; j < ext[1]; ++j)
        for (int i = 0; i < ext[0]; ++i) {
          int id[3] = {i, j, k};
          double U[5], V[15], Gd[5];
          for (int v = 0; v < nv; ++v) {
            U[v] = w->UFC[d][aidx(ext, v, i, j, k)];
            for (int m = 0; m < 3; ++m) V[m * nv + v] = w->VF[d][m * nf + aidx(ext, v, i, j, k)];
          }
          int at_end = (id[d] == 0 || id[d] == n);
          if (c->prm.physics == OR_NAVIER_STOKES && at_end) {
            /* interface: Roe flux on the two discontinuous traces, minus the
               centred viscous flux on (u_hat, v_hat) */
            int s = id[d] == 0 ? 0 : 1;
            const double *nbF = s == 0 ? w->UFnb : w->UFnb2;
            int io[3] = {i, j, k};
            io[d] = s == 0 ? n : 0;
            double Um[5], Un[5], Fr[5], Fv[5], Gc[15];
            for (int v = 0; v < 5; ++v) {
              Um[v] = w->UFraw[aidx(ext, v, i, j, k)];
              Un[v] = nbF[aidx(ext, v, io[0], io[1], io[2])];
            }
            if (s == 0) or_ns_roe(&c->prm, Un, Um, d, Fr);
            else or_ns_roe(&c->prm, Um, Un, d, Fr);
            for (int v = 0; v < 5; ++v)
              for (int mm = 0; mm < 3; ++mm) Gc[v * 3 + mm] = V[mm * 5 + v];
            or_ns_flux_visc(&c->prm, U, Gc, d, Fv);
            for (int v = 0; v < 5; ++v) Gd[v] = c->S[d][d] * (Fr[v] - Fv[v]);
          } else {
            c3_point_flux(c, d, U, V, Gd);
          }
          for (int v = 0; v < nv; ++v) w->G[d][aidx(ext, v, i, j, k)] = Gd[v];
          (void)npts;
        }
  }
  /* step 5: dq/dt = -sum_d M_d G_d, du/dt = [J^-1] dq/dt */
  for (long i = 0; i < nv * n3; ++i) out[i] = 0.0;
  for (int d = 0; d < 3; ++d) {
    int ext[3];
    fam_ext(c, d, ext);
    apply_axis(c->M, n, n + 1, d, nv, ext, w->G[d], w->dH);
    for (long i = 0; i < nv * n3; ++i) out[i] -= w->dH[i];
  }
  for (long i = 0; i < nv * n3; ++i) out[i] /= c->J;
}

static int c3_setup(ctx3 *c, const int *nel, const double *lo, const double *hi, int p,
                    int scheme, const or_params *prm, const double *u) {
  double xs[OR_MAXN], xf[OR_MAXN + 1];
  if (p < 1 || p + 1 > OR_MAXN) return -1;
  if (scheme != OR_BR1 && scheme != OR_COMPACT) return -1;
  for (int d = 0; d < 3; ++d) {
    if (nel[d] < 1 || !(hi[d] > lo[d])) return -1;
    c->nel[d] = nel[d];
    c->h[d] = (hi[d] - lo[d]) / nel[d];
  }
  if (!(prm->eta_ip >= 0.0)) return -1;
  c->n = p + 1;
  c->scheme = scheme;
  c->prm = *prm;
  if (prm->physics == OR_NAVIER_STOKES) c->nv = 5;
  else if (prm->physics == OR_DIFFUSION || prm->physics == OR_PME) c->nv = 1;
  else return -1;
  /* affine hexahedron: J = det(dx/dxi) = prod h_d/2, S = adj(dx/dxi) is
     diagonal with S_dd = prod_{d' != d} h_d'/2 */
  c->J = 0.125 * c->h[0] * c->h[1] * c->h[2];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) c->S[a][b] = 0.0;
  c->S[0][0] = 0.25 * c->h[1] * c->h[2];
  c->S[1][1] = 0.25 * c->h[0] * c->h[2];
  c->S[2][2] = 0.25 * c->h[0] * c->h[1];
  c->u = u;
  return or_operators(p, xs, c->ws, xf, c->L, c->M);
}

int or_rhs_3d_elems(const int *nel, const double *lo, const double *hi, int p, int scheme,
                    const or_params *prm, const double *u, const long *elems, long n_elems,
                    double *dudt_sel, int nthreads) {
  ctx3 c;
  if (c3_setup(&c, nel, lo, hi, p, scheme, prm, u)) return -1;
  long ne = (long)nel[0] * nel[1] * nel[2];
  long esz = (long)c.nv * c.n * c.n * c.n;
  for (long k = 0; k < n_elems; ++k)
    if (elems[k] < 0 || elems[k] >= ne) return -1;
  int rc = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(| : rc)
#endif
  {
    work3 w;
    if (work3_alloc(&c, &w)) {
      rc = -2;
    } else {
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 4)
#endif
      for (long k = 0; k < n_elems; ++k) c3_rhs_elem(&c, elems[k], dudt_sel + k * esz, &w);
      free(w.UF);
    }
  }
  return rc;
}

int or_rhs_3d(const int *nel, const double *lo, const double *hi, int p, int scheme,
              const or_params *prm, const double *u, double *dudt, int nthreads) {
  long ne = (long)nel[0] * nel[1] * nel[2];
  long *idx = malloc(sizeof(long) * (ne > 0 ? ne : 1));
  if (!idx) return -2;
  for (long k = 0; k < ne; ++k) idx[k] = k;
  int rc = or_rhs_3d_elems(nel, lo, hi, p, scheme, prm, u, idx, ne, dudt, nthreads);
  free(idx);
  return rc;
}

int or_rk4_3d(const int *nel, const double *lo, const double *hi, int p, int scheme,
              const or_params *prm, double *u, double dt, int nsteps, int nthreads) {
  int nv = prm->physics == OR_NAVIER_STOKES ? 5 : 1;
  long sz = (long)nel[0] * nel[1] * nel[2] * nv * (p + 1) * (p + 1) * (p + 1);
  double *k = malloc(sizeof(double) * sz * 5);
  if (!k) return -2;
  double *k1 = k, *k2 = k + sz, *k3 = k + 2 * sz, *k4 = k + 3 * sz, *w = k + 4 * sz;
  int rc = 0;
  for (int s = 0; s < nsteps && !rc; ++s) {
    rc |= or_rhs_3d(nel, lo, hi, p, scheme, prm, u, k1, nthreads);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + 0.5 * dt * k1[i];
    rc |= or_rhs_3d(nel, lo, hi, p, scheme, prm, w, k2, nthreads);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + 0.5 * dt * k2[i];
    rc |= or_rhs_3d(nel, lo, hi, p, scheme, prm, w, k3, nthreads);
    for (long i = 0; i < sz; ++i) w[i] = u[i] + dt * k3[i];
    rc |= or_rhs_3d(nel, lo, hi, p, scheme, prm, w, k4, nthreads);
    for (long i = 0; i < sz; ++i) u[i] += dt / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
  }
  free(k);
  return rc;
}

/* Kinetic energy 1/2 int u.u and enstrophy int w.w (section 4.4), by
   Gauss-Legendre quadrature on the solution points (weight J w_i w_j w_k);
   the vorticity comes from the standard auxiliary gradient of the
   conservative variables, converted to velocity gradients. */
int or_diag_3d(const int *nel, const double *lo, const double *hi, int p,
               const or_params *prm, const double *u, double *out, int nthreads) {
  ctx3 c;
  if (prm->physics != OR_NAVIER_STOKES) return -1;
  if (c3_setup(&c, nel, lo, hi, p, OR_BR1, prm, u)) return -1;
  long ne = (long)nel[0] * nel[1] * nel[2];
  int n = c.n;
  long n3 = (long)n * n * n;
  double ke = 0, ens = 0, mass = 0, m0 = 0, m1 = 0, m2 = 0, en = 0, umax = 0, smax = 0;
  int bad = 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel reduction(+ : ke, ens, mass, m0, m1, m2, en) reduction(max : umax, smax) \
    reduction(| : bad)
#endif
  {
    work3 w;
    if (work3_alloc(&c, &w)) {
      bad |= 2;
    } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
      for (long e = 0; e < ne; ++e) {
        const double *ue = u + e * 5 * n3;
        c3_vS(&c, e, -1, -1, w.vS, w.UF, w.tmp, w.H, w.dH);
        for (int k = 0; k < n; ++k)
          for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
              long q = ((long)k * n + j) * n + i;
              double wq = c.J * c.ws[i] * c.ws[j] * c.ws[k];
              double U[5];
              for (int v = 0; v < 5; ++v) {
                U[v] = ue[v * n3 + q];
                if (!isfinite(U[v])) bad |= 1;
              }
              double vel[3] = {U[1] / U[0], U[2] / U[0], U[3] / U[0]};
              double du[3][3];
              for (int a = 0; a < 3; ++a)
                for (int m = 0; m < 3; ++m)
                  du[a][m] = (w.vS[(m * 5 + 1 + a) * n3 + q] - vel[a] * w.vS[(m * 5 + 0) * n3 + q]) / U[0];
              double om[3] = {du[2][1] - du[1][2], du[0][2] - du[2][0], du[1][0] - du[0][1]};
              double v2 = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
              ke += wq * 0.5 * v2;
              ens += wq * (om[0] * om[0] + om[1] * om[1] + om[2] * om[2]);
              mass += wq * U[0];
              m0 += wq * U[1];
              m1 += wq * U[2];
              m2 += wq * U[3];
              en += wq * U[4];
              if (sqrt(v2) > umax) umax = sqrt(v2);
              /* fastest acoustic signal |u| + c, c^2 = gamma P / rho (the
                 convective time-step limit of section 4.4) */
              double P = (prm->gamma - 1.0) * (U[4] - 0.5 * U[0] * v2);
              double sp = (U[0] > 0.0 && P >= 0.0) ? sqrt(v2) + sqrt(prm->gamma * P / U[0]) : INFINITY;
              if (sp > smax) smax = sp;
            }
      }
      free(w.UF);
    }
  }
  out[0] = ke; out[1] = ens; out[2] = mass; out[3] = m0; out[4] = m1; out[5] = m2;
  out[6] = en; out[7] = umax; out[8] = (bad & 1) ? 1.0 : 0.0; out[9] = smax;
  return (bad & 2) ? -2 : 0;
}
