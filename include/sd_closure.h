/*
 * sd_closure.h - C ABI of the learned per-element closure of the SD
 * right-hand side (an MLP that corrects the coarse-grid residual) and of the
 * fine-to-coarse filter that builds its training data.
 *
 * Network: y = W3 g(W2 g(W1 x + b1) + b2) + b3, g the exact-erf GELU.
 * Parameters live in one flat FP32 vector P (the master copy), in the order
 * W1 [n_hidden][n_in], b1 [n_hidden], W2 [n_hidden][n_hidden], b2,
 * W3 [n_out][n_hidden], b3 [n_out]; weights row-major [out][in].  The
 * products use a BF16 copy of P (Wb, same length and offsets, weights only
 * read) on BF16 matrix cores with FP32 accumulation; every layer input is
 * rounded to BF16 (round to nearest even) before its product.  Sizes n_in,
 * n_hidden, n_out must be multiples of 16.
 *
 * All pointers are device pointers owned by the caller; every call is
 * enqueued on the given hipStream_t (NULL = default stream) and returns
 * SD_OK or a negative code of sd.h (message via sd_last_error()).
 */
#ifndef SD_CLOSURE_H
#define SD_CLOSURE_H

#include <stdint.h>

#include "sd.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int n_in, n_hidden, n_out;
} sd_mlp_shape;

/* Number of FP32 values of P (and of BF16 values of Wb). */
long long sd_mlp_param_count(const sd_mlp_shape *shape);

/* Bytes of the activation workspace for a batch of B samples (kept between
 * sd_mlp_forward and sd_mlp_backward). */
long long sd_mlp_work_bytes(const sd_mlp_shape *shape, int batch);

/* Wb = bf16(P), round to nearest even. */
int sd_mlp_round_weights(const sd_mlp_shape *shape, const float *P, uint16_t *Wb, void *stream);

/* Y [B][n_out] = net(X [B][n_in]); the activations go to work. */
int sd_mlp_forward(const sd_mlp_shape *shape, const float *P, const uint16_t *Wb, const float *X, int batch,
                   float *Y, void *work, void *stream);

/* The forward pass of sd_mlp_forward without the workspace argument and
 * without any device allocation, for callers that cannot allocate (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc).
 * The activations go to a static device array of the library (16 MiB, one
 * per GPU, held until the process ends); the caller still owns X and Y.
 * Every call on one GPU shares that array: calls that overlap on one GPU
 * (several streams or threads) race, and the activations are not kept for a
 * backward pass.  The activations of a batch B take five buffers, each
 * rounded up to 256 bytes: 2 B n_in, 2 B n_hidden twice (BF16 layer inputs)
 * and 4 B n_hidden twice (FP32 pre-activations), i.e. about
 * 2 n_in + 12 n_hidden bytes per sample (B <= 7 700 for 320-128-320).  A
 * batch that does not fit is rejected with SD_EINVAL and nothing is
 * launched. */
int sd_mlp_forward_noalloc(const sd_mlp_shape *shape, const float *P, const uint16_t *Wb, const float *X, int batch,
                           float *Y, void *stream);

/* Grad [param_count] = d(sum dY . Y)/dP for the forward pass whose
 * activations are in work (weights as their BF16 values, the roundings of
 * the forward pass treated as fixed); products in FP32 on the FP32 matrix
 * cores, every sum in a fixed order. */
int sd_mlp_backward(const sd_mlp_shape *shape, const uint16_t *Wb, void *work, const float *dY, int batch,
                    float *grad, void *stream);

/* Weighted mean square error of Y against T, both [rows][cols]:
 *     loss = sum_r w[r] sum_c (Y - T)^2 / (rows cols),  dY = 2 w[r] (Y - T) / (rows cols),
 * with w [rows] per-row weights (NULL = all ones); the loss goes to *loss
 * (device FP64 scalar), reduced in a fixed order, or is not computed when
 * loss is NULL (dY alone). */
int sd_mse(const float *Y, const float *T, const float *w, long long rows, int cols, float *dY, double *loss,
           void *stream);

/* One Adam step (Kingma & Ba, bias-corrected, step >= 1) on P with moments
 * m, v (FP32, same length), then Wb = bf16(P). */
int sd_mlp_adam(const sd_mlp_shape *shape, float *P, uint16_t *Wb, const float *grad, float *m, float *v,
                int step, float lr, float beta1, float beta2, float eps, void *stream);

/* L2 projection of a fine degree-p state on nel_fine[0..2] periodic-box
 * elements onto the degree-p space of each coarse element (ratio^3 fine
 * elements each), evaluated at the coarse solution points.  Layout of both
 * states as in sd.h (u[e][v][k][j][i]); nel_fine[d] must be divisible by
 * ratio; ratio * (p + 1) <= 16 and p + 1 <= 8. */
int sd_filter(const double *fine, const int *nel_fine, int ratio, int p, int nv, double *coarse, void *stream);

/* Closure of an SD context (3-D Navier-Stokes): every later right-hand side
 * (sd_rhs, and each stage of sd_rk_step) adds to element e
 *     C_e = out_scale[v] * net((u_e[v] - in_shift[v]) / in_scale[v])
 * unless C_e holds a non-finite value or, with max_ratio > 0,
 * max|C_e| > max_ratio * max|R_e| (then C_e = 0 for that element).
 * n_in = n_out = 5 (p+1)^3.  P and Wb stay owned by the caller and are read
 * at each evaluation.  P = NULL switches the closure off.  Inside the
 * solver the network's FP32 sums over K may be taken in another order than
 * in sd_mlp_forward (p = 3 with n_hidden = 128 or 256 runs as one launch
 * per RHS), so the two agree to the rounding of those sums,
 * which can move the BF16 rounding of an activation. */
int sd_closure_set(sd_ctx *ctx, const sd_mlp_shape *shape, const float *P, const uint16_t *Wb,
                   const float *in_shift, const float *in_scale, const float *out_scale, float max_ratio);

/* Number of element corrections discarded since the last sd_closure_set
 * (waits for the context's stream). */
int sd_closure_rejected(sd_ctx *ctx, long long *count);

#ifdef __cplusplus
}
#endif
#endif /* SD_CLOSURE_H */
