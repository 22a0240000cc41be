/* Batched temporal (Bloch) eigenanalysis and combined-mode analysis of the
 * 1-D SD discretisation of the diffusion equation u_t = u_xx (section 3 and
 * the appendix), on the GPU.
 *
 * For the Bloch wave u_e = exp(i theta e) u_0 on a uniform periodic mesh of
 * elements of width 2J, the semi-discrete operator acts on the p+1 solution
 * values of one element as the complex matrix B(theta); its eigenvalues
 * lambda = -i omega are the dissipation (Re lambda) and dispersion curves of
 * section 3.  The combined mode of the appendix expands the Fourier mode
 * u0_i = exp(i theta (xi_i + 1) / 2) (xi_i the solution points) on the
 * eigenvectors and evolves it: u(t) = exp(B t) u0, G(theta, t) =
 * u0^H u(t) / u0^H u0, omega(theta, t) = (i / t) log G (principal log).
 *
 * Numbers are FP64; complex values are stored as (re, im) pairs.  Every
 * array is device memory owned by the caller; the call enqueues one kernel
 * on `stream` (a hipStream_t, NULL = default stream) and returns without
 * waiting. */
#ifndef SD_BLOCH_H
#define SD_BLOCH_H

#include "sd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int p;          /* polynomial degree, 1..8 (else SD_EUNSUPPORTED)           */
  int scheme;     /* SD_BR1 (standard gradient) or SD_COMPACT (section 2.2)   */
  double J;       /* element Jacobian, element width 2J; > 0 and finite       */
  double eta_ip;  /* interior penalty, tau = eta_ip (p+1)^2 / (2J) (section 3);
                     >= 0 and finite, 0 = off                                 */
} sd_bloch_cfg;

/* For each theta[k], k < ntheta (device, FP64):
 *   B     [ntheta][p+1][p+1] complex, row-major: B(theta) (NULL: skip)
 *   lam   [ntheta][p+1] complex: eigenvalues of B(theta), real part
 *         descending, ties by imaginary part; NaN where the QR iteration
 *         does not converge (NULL: skip)
 *   G     [ntheta][nt] complex: combined-mode amplification at t[j] (device,
 *         FP64, nt >= 0); NaN where t[j] is not positive and finite (NULL:
 *         skip)
 *   omega [ntheta][nt] complex: (i / t[j]) log G (NULL: skip)
 * Returns SD_EINVAL for a null cfg, a bad scheme, J or eta_ip, a negative
 * count, or a null theta (ntheta > 0) or t (nt > 0 with G or omega
 * requested); SD_EHIP if the launch fails.  ntheta = 0 does nothing. */
int sd_bloch(const sd_bloch_cfg *cfg, const double *theta, long long ntheta, const double *t, int nt,
             double *B, double *lam, double *G, double *omega, void *stream);

#ifdef __cplusplus
}
#endif

#endif
