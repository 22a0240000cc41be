// Kernels of the learned closure: a dense MLP with exact-erf GELU, forward on
// BF16 matrix cores (v_mfma_f32_16x16x16bf16_1k, FP32 accumulation),
// backward products on FP32 matrix cores (v_mfma_f32_16x16x4f32), MSE, Adam;
// and the fine-to-coarse L2 projection filter.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sd {

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest even (NaN kept quiet)
__device__ __forceinline__ uint16_t to_bf16(float x) {
  uint32_t b = __float_as_uint(x);
  if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x0040u);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_prime_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// x (FP32) -> bf16
__global__ void k_to_bf16(const float *__restrict__ x, uint16_t *__restrict__ y, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// One dense layer Z = X W^T + b on matrix cores; X [M][K] bf16, W [N][K] bf16
// (row-major), b [N] FP32; K and N multiples of 16.  One wavefront per 16x16
// tile of Z.  Operand layout of the 16x16x16 BF16 instruction: lane l holds
// row l%16 of the A tile and column l%16 of the B tile at k = 4(l/16)+0..3,
// and D[4(l/16)+j][l%16] of the result.  ACT: also A_out = bf16(gelu(Z)).
template <bool ACT>
__global__ void __launch_bounds__(256) k_dense_fwd(const uint16_t *__restrict__ X, const uint16_t *__restrict__ W,
                                                   const float *__restrict__ bias, int M, int N, int K,
                                                   float *__restrict__ Z, uint16_t *__restrict__ Aout) {
  const int wave = (int)((blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  const int ntn = N / 16;
  const int mt = wave / ntn, nt = wave % ntn;
  if (mt * 16 >= M) return;                     // uniform for the wavefront
  const int r = lane & 15, kq = lane >> 4;
  const int row = mt * 16 + r, col = nt * 16 + r;
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  // chunks of KU steps: all operand reads of a chunk are issued before its
  // matrix instructions, from clamped addresses (rows past M read row M - 1
  // and steps past K the last step, replaced by zeros, so that they add
  // exact zeros); the products keep the order of k
  constexpr int KU = 10;
  const int rowc = row < M ? row : M - 1;
  const bf16x4_t zero = {0, 0, 0, 0};
  for (int k0 = 0; k0 < K; k0 += 16 * KU) {
    bf16x4_t a[KU], b[KU];
#pragma unroll
    for (int s = 0; s < KU; ++s) {
      const int k = min(k0 + 16 * s, K - 16);
      a[s] = *reinterpret_cast<const bf16x4_t *>(X + (long long)rowc * K + k + 4 * kq);
      b[s] = *reinterpret_cast<const bf16x4_t *>(W + (long long)col * K + k + 4 * kq);
    }
    // keeps the compiler from moving the reads down to their uses
    __asm__ __volatile__("" ::: "memory");
#pragma unroll
    for (int s = 0; s < KU; ++s) {
      // the lane's row of X and its column of W are separate operands
      const bool kin = k0 + 16 * s < K;
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(kin && row < M ? a[s] : zero, kin ? b[s] : zero, acc, 0, 0,
                                                       0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int m = mt * 16 + 4 * kq + j;
    if (m < M) {
      float z = acc[j] + bias[col];
      Z[(long long)m * N + col] = z;
      if constexpr (ACT) Aout[(long long)m * N + col] = to_bf16(gelu_f(z));
    }
  }
}

// C [M][N] = sum_k A(m, k) B(k, n) with strided operands on the FP32 matrix
// cores (v_mfma_f32_16x16x4f32: lane l supplies A(l%16, k0 + l/16) and
// B(k0 + l/16, l%16) and receives C[4(l/16)+j][l%16]), FP32 products and
// sums.  One 16x16 tile of C per block of KW wavefronts: wave w sums the
// w-th contiguous part of the k range (KW parts) and the partial tiles are
// added through LDS in wave order (a fixed order).  With GELU_BWD the tile is
// multiplied by gelu'(Z[m][n]) on the way out (the activation's backward).
// With Bsum non-null, the blocks of the first column of tiles also write
// Bsum[m] = sum_k A(m, k) (a layer's bias gradient when A is the output
// gradient transposed), summed per lane, then over the four lane groups and
// the waves in a fixed order.
template <typename TA>
__device__ __forceinline__ float as_f32(TA v) {
  if constexpr (sizeof(TA) == 2) return from_bf16((uint16_t)v);
  else return v;
}

template <int KW, typename TA, typename TB, bool GELU_BWD>
__global__ void __launch_bounds__(64 * KW) k_gemm_mfma(int M, int N, int K, const TA *__restrict__ A,
                                                               long long sam, long long sak,
                                                               const TB *__restrict__ B, long long sbk,
                                                               long long sbn, const float *__restrict__ Z,
                                                               float *__restrict__ C, float *__restrict__ Bsum) {
  __shared__ float red[KW - 1][4][64];
  __shared__ float bred[KW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = lane & 15, kq = lane >> 4;
  const long long m = (long long)blockIdx.y * 16 + r, n = (long long)blockIdx.x * 16 + r;
  const int kc = ((K + 4 * KW - 1) / (4 * KW)) * 4;
  const int kb = w * kc, ke = min(K, kb + kc);
  f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
  float asum = 0.f;
  // chunks of KU steps: all operand reads of a chunk are issued before its
  // matrix instructions, from clamped addresses (reads outside the operands
  // take the last row, column or k and are replaced by zeros, so steps past
  // the range add exact zeros); the products and sums keep the order of k
  constexpr int KU = KW >= 8 ? 16 : 10;
  const long long mc = m < M ? m : M - 1, nc = n < N ? n : N - 1;
  for (int k0 = kb; k0 < ke; k0 += 4 * KU) {
    TA a[KU];
    TB b[KU];
#pragma unroll
    for (int s = 0; s < KU; ++s) {
      const long long k = k0 + 4 * s + kq, kc = k < ke ? k : ke - 1;
      a[s] = A[mc * sam + kc * sak];
      b[s] = B[kc * sbk + nc * sbn];
    }
    // keeps the compiler from moving the reads down to their uses
    __asm__ __volatile__("" ::: "memory");
#pragma unroll
    for (int s = 0; s < KU; ++s) {
      const long long k = k0 + 4 * s + kq;
      const float av = (m < M && k < ke) ? as_f32(a[s]) : 0.f, bv = (n < N && k < ke) ? as_f32(b[s]) : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      asum += av;
    }
  }
  // the activation's pre-activations, read before the partial tiles are
  // summed so that their latency passes during the reduction
  float zv[4] = {0.f, 0.f, 0.f, 0.f};
  if constexpr (GELU_BWD) {
    if (w == 0)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const long long mo = (long long)blockIdx.y * 16 + 4 * kq + j;
        zv[j] = Z[(mo < M ? mo : M - 1) * N + nc];
      }
  }
  if (Bsum && blockIdx.x == 0) {
    // uniform over the block
    bred[w][lane] = asum;
    __syncthreads();
    if (w == 0 && kq == 0 && m < M) {
      float t = 0.f;
      for (int ww = 0; ww < KW; ++ww)
        for (int g = 0; g < 4; ++g) t += bred[ww][16 * g + r];
      Bsum[m] = t;
    }
  }
  if (w > 0)
#pragma unroll
    for (int j = 0; j < 4; ++j) red[w - 1][j][lane] = acc[j];
  __syncthreads();
  if (w != 0) return;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float v = acc[j];
    for (int ww = 0; ww < KW - 1; ++ww) v += red[ww][j][lane];
    const long long mo = (long long)blockIdx.y * 16 + 4 * kq + j;
    if (mo < M && n < N) {
      if constexpr (GELU_BWD) v *= gelu_prime_f(zv[j]);
      C[mo * N + n] = v;
    }
  }
}

// dY = 2 w_r (Y - T) / n, one thread per value (elementwise)
__global__ void __launch_bounds__(256) k_mse_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                  const float *__restrict__ w, long long n, int cols, float scale,
                                                  float *__restrict__ dY) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float wr = w ? w[i / cols] : 1.0f;
  dY[i] = scale * wr * (Y[i] - T[i]);
}

// loss = sum_r w_r sum_c (Y - T)^2 / n in FP64, one block, a fixed order:
// lane l takes the rows l, l + 1024, ... whole, then the 1024 partial sums
// are added pairwise
__global__ void __launch_bounds__(1024) k_mse_loss(const float *__restrict__ Y, const float *__restrict__ T,
                                                   const float *__restrict__ w, long long rows, int cols,
                                                   double inv_n, double *__restrict__ loss) {
  __shared__ double red[1024];
  double acc = 0.0;
  for (long long r = threadIdx.x; r < rows; r += blockDim.x) {
    const double wr = w ? (double)w[r] : 1.0;
    double rs = 0.0;
    for (int c = 0; c < cols; ++c) {
      const double d = (double)(Y[r * cols + c] - T[r * cols + c]);
      rs += d * d;
    }
    acc += wr * rs;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = red[0] * inv_n;
}

// Adam step with bias corrections c1 = 1/(1-b1^t), c2 = 1/(1-b2^t); Wb = bf16(P)
__global__ void k_adam(float *__restrict__ P, uint16_t *__restrict__ Wb, const float *__restrict__ g,
                       float *__restrict__ m, float *__restrict__ v, long long n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float p = P[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  P[i] = p;
  Wb[i] = to_bf16(p);
}

// Fine-to-coarse L2 projection: one block per (coarse element, variable).
constexpr int kFilterMaxRN = 16;
constexpr int kFilterMaxN = 8;
struct FilterArgs {
  int nelc[3];
  int nelf[3];
  int ratio, n, nv;
  double P[kFilterMaxN * kFilterMaxRN];   // [n][ratio*n], coarse coefficient from fine values
};

__global__ void __launch_bounds__(256) k_filter(const double *__restrict__ fine, double *__restrict__ coarse,
                                                FilterArgs a) {
  __shared__ double F[kFilterMaxRN * kFilterMaxRN * kFilterMaxRN];
  __shared__ double T1[kFilterMaxRN * kFilterMaxRN * kFilterMaxN];
  __shared__ double T2[kFilterMaxRN * kFilterMaxN * kFilterMaxN];
  const int n = a.n, r = a.ratio, rn = r * n, nv = a.nv;
  const int ec = blockIdx.x / nv, v = blockIdx.x % nv;
  const int cx = ec % a.nelc[0], cy = (ec / a.nelc[0]) % a.nelc[1], cz = ec / (a.nelc[0] * a.nelc[1]);
  const int n3 = n * n * n;
  // F[gz][gy][gx] over the r^3 fine elements of this coarse element
  for (int t = threadIdx.x; t < r * r * r * n3; t += blockDim.x) {
    int fe = t / n3, pt = t % n3;
    int fx = fe % r, fy = (fe / r) % r, fz = fe / (r * r);
    int i = pt % n, j = (pt / n) % n, k = pt / (n * n);
    long long ef = (long long)(cx * r + fx) + (long long)a.nelf[0] * ((cy * r + fy) + (long long)a.nelf[1] * (cz * r + fz));
    F[((fz * n + k) * rn + (fy * n + j)) * rn + (fx * n + i)] = fine[(ef * nv + v) * n3 + pt];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < rn * rn * n; t += blockDim.x) {       // along x
    int ic = t % n, gy = (t / n) % rn, gz = t / (n * rn);
    double s = 0.0;
    for (int g = 0; g < rn; ++g) s += a.P[ic * rn + g] * F[(gz * rn + gy) * rn + g];
    T1[(gz * rn + gy) * n + ic] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < rn * n * n; t += blockDim.x) {        // along y
    int ic = t % n, jc = (t / n) % n, gz = t / (n * n);
    double s = 0.0;
    for (int g = 0; g < rn; ++g) s += a.P[jc * rn + g] * T1[(gz * rn + g) * n + ic];
    T2[(gz * n + jc) * n + ic] = s;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < n3; t += blockDim.x) {               // along z
    int ic = t % n, jc = (t / n) % n, kc = t / (n * n);
    double s = 0.0;
    for (int g = 0; g < rn; ++g) s += a.P[kc * rn + g] * T2[(g * n + jc) * n + ic];
    coarse[((long long)ec * nv + v) * n3 + t] = s;
  }
}

// Closure input: X[e][v n^3 + pt] = (u[e][v][pt] - shift[v]) / scale[v]
struct ClosureNorm {
  float shift[5], scale[5], out_scale[5];
  float max_ratio;        // <= 0: no magnitude bound
};

// a[v] for a run-time v in [0, 5) by selects: the constant-index reads stay
// scalar loads of the kernel arguments (an indexed read would be a vector
// load from the argument segment per value)
__device__ __forceinline__ double pick5(const float (&a)[5], int v) {
  return (double)(v == 0 ? a[0] : v == 1 ? a[1] : v == 2 ? a[2] : v == 3 ? a[3] : a[4]);
}

__global__ void k_closure_input(const double *__restrict__ u, float *__restrict__ X, long long n, int np,
                                ClosureNorm cn) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int v = (int)((i / np) % 5);
  X[i] = (float)((u[i] - pick5(cn.shift, v)) / pick5(cn.scale, v));
}

}  // namespace sd
