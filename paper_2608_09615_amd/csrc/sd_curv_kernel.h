// SD diffusion right-hand side on curvilinear hexahedra (section 2.3 with a
// general adjoint S), scalar u_t = nu lap u, FP64.
//
// Geometry per element: S row d (S_d0, S_d1, S_d2) at the flux points of
// family d and 1/det J at the solution points, stored line-major: for
// family d the n^2 lines along d are numbered q by the two transverse
// indices (d = 0: q = j + n k; d = 1: q = i + n k; d = 2: q = i + n j) and
// the n + 1 flux points of a line by r.  Face arrays use the same q, so the
// two elements of a face index its points alike.
//
// Three kernels, one element per block (cv_threads<N>() lanes):
//   k_cv_traces  the solution at the six faces, T[e][f][q] (f = 2 d + s);
//   k_cv_grad    common solution at the faces, the continuous solution at
//                the flux points, the auxiliary variable v_m at the
//                solution points (J^-1 sum_d D_d(u^{Fd,C} S_dm)) and its
//                values at the faces: one-sided (compact: the family-d
//                solution keeps the own trace at the other face, which adds
//                J^-1 M[:, end] (T - u_hat) S_dm to v_m along the lines) or
//                standard (BR1);
//   k_cv_rhs     common gradient at the faces (average of the two sides,
//                plus the interior penalty when on: tau (u_R - u_L) along
//                n = S_d / |S_d|, stored as P = tau / |S_d| per face point),
//                v_m at the interior flux points, G_d = -nu sum_m S_dm v_m
//                and du/dt = -J^-1 sum_d D_d G_d.
#pragma once

namespace sd {

// one element per block: a single wavefront for n <= 4 (barriers stay
// cheap and many blocks fit a CU), more lanes for the larger elements
template <int N>
__host__ __device__ constexpr int cv_threads() { return N <= 4 ? 64 : (N <= 5 ? 128 : 256); }

template <int N>
__device__ __forceinline__ int cv_point(int d, int q, int c) {
  // solution point c along line q of direction d
  if (d == 0) return q * N + c;
  if (d == 1) return (q % N) + N * N * (q / N) + c * N;
  return q + c * N * N;
}

template <int N>
__device__ __forceinline__ void cv_line_of(int pt, int d, int &q, int &c) {
  const int i = pt % N, j = (pt / N) % N, k = pt / (N * N);
  if (d == 0) {
    q = j + N * k;
    c = i;
  } else if (d == 1) {
    q = i + N * k;
    c = j;
  } else {
    q = i + N * j;
    c = k;
  }
}

template <int N>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_traces(const double *__restrict__ U, double *__restrict__ T,
                                                          const double *__restrict__ ops, long long ne) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N;
  const long long e = blockIdx.x;
  if (e >= ne) return;
  const double *u = U + e * NP;
  for (int t = threadIdx.x; t < 6 * NF; t += blockDim.x) {
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    double acc = 0.0;
    for (int c = 0; c < N; ++c) acc += ops[O.Lend + s * N + c] * u[cv_point<N>(d, q, c)];
    T[e * 6 * NF + t] = acc;
  }
}

template <int N>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_grad(const double *__restrict__ U, const double *__restrict__ T,
                                                        const double *__restrict__ Sf, const double *__restrict__ Jinv,
                                                        const double *__restrict__ ops, KArgs a, int compact,
                                                        double *__restrict__ VF, double *__restrict__ VS) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF;
  // the element's metric rows ([d][q][r][m]) are read by every point of a
  // line: staged in LDS for n >= 5, where that beats the L2 (for n <= 4 the
  // extra LDS and load phase cost more than the misses they save)
  constexpr bool kStageS = N >= 5;
  __shared__ double su[NP], sT[6 * NF], sUh[6 * NF], sUF[3 * NL], sV[3 * NP], sS[kStageS ? 9 * NL : 1];
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x;
  const double *ji = Jinv + e * NP;
  const double *S = kStageS ? sS : Sf + e * 9 * NL;
  if constexpr (kStageS)
    for (int t = tid; t < 9 * NL; t += blockDim.x) sS[t] = Sf[e * 9 * NL + t];
  for (int t = tid; t < NP; t += blockDim.x) su[t] = U[e * NP + t];
  for (int t = tid; t < 6 * NF; t += blockDim.x) {
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    const double own = T[e * 6 * NF + t];
    const double oth = T[nbr(a, e, d, s) * 6 * NF + (2 * d + 1 - s) * NF + q];
    sT[t] = own;
    sUh[t] = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
  }
  __syncthreads();
  // continuous solution at the flux points of every family
  for (int t = tid; t < 3 * NL; t += blockDim.x) {
    const int d = t / NL, w = t % NL, q = w / (N + 1), r = w % (N + 1);
    double val;
    if (r == 0) {
      val = sUh[(2 * d) * NF + q];
    } else if (r == N) {
      val = sUh[(2 * d + 1) * NF + q];
    } else {
      val = 0.0;
      for (int c = 0; c < N; ++c) val += ops[O.Lint + (r - 1) * N + c] * su[cv_point<N>(d, q, c)];
    }
    sUF[t] = val;
  }
  __syncthreads();
  // auxiliary variable at the solution points
  for (int t = tid; t < 3 * NP; t += blockDim.x) {
    const int m = t / NP, pt = t % NP;
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      double dd = 0.0;
      for (int r = 0; r <= N; ++r)
        dd += ops[O.M + c * (N + 1) + r] * (sUF[d * NL + q * (N + 1) + r] * S[((d * NF + q) * (N + 1) + r) * 3 + m]);
      acc += dd;
    }
    const double v = ji[pt] * acc;
    sV[t] = v;
    VS[(e * 3 + m) * NP + pt] = v;
  }
  __syncthreads();
  // values at the faces
  for (int t = tid; t < 6 * 3 * NF; t += blockDim.x) {
    const int f = t / (3 * NF), w = t % (3 * NF), m = w / NF, q = w % NF, d = f >> 1, s = f & 1;
    double corr = 0.0;
    int rend = 0;
    if (compact) {
      // the family-d solution of face s keeps the own trace at the other face
      const int so = 1 - s;
      rend = so == 0 ? 0 : N;
      corr = (sT[(2 * d + so) * NF + q] - sUh[(2 * d + so) * NF + q]) * S[((d * NF + q) * (N + 1) + rend) * 3 + m];
    }
    double acc = 0.0;
    for (int c = 0; c < N; ++c) {
      const int pt = cv_point<N>(d, q, c);
      double v = sV[m * NP + pt];
      if (compact) v += ji[pt] * (ops[O.M + c * (N + 1) + rend] * corr);
      acc += ops[O.Lend + s * N + c] * v;
    }
    VF[((e * 6 + f) * 3 + m) * NF + q] = acc;
  }
}

template <int N>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_rhs(const double *__restrict__ VF, const double *__restrict__ VS,
                                                       const double *__restrict__ Sf, const double *__restrict__ Jinv,
                                                       const double *__restrict__ ops, KArgs a,
                                                       const double *__restrict__ T, const double *__restrict__ Pen,
                                                       double *__restrict__ dudt) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF;
  __shared__ double sV[3 * NP], sVh[6 * 3 * NF], sG[3 * NL];
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x;
  const double *S = Sf + e * 9 * NL;
  const double *ji = Jinv + e * NP;
  for (int t = tid; t < 3 * NP; t += blockDim.x) sV[t] = VS[e * 3 * NP + t];
  for (int t = tid; t < 6 * 3 * NF; t += blockDim.x) {
    const int f = t / (3 * NF), w = t % (3 * NF), d = f >> 1, s = f & 1;
    const long long en = nbr(a, e, d, s);
    const double own = VF[(e * 6 + f) * 3 * NF + w];
    const double oth = VF[(en * 6 + 2 * d + 1 - s) * 3 * NF + w];
    double vh = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
    if (Pen) {
      // interior penalty: P (u_R - u_L) S_dm, u_R on the +xi_d side
      const int m = w / NF, q = w % NF;
      const double to = T[(e * 6 + f) * NF + q], tn = T[(en * 6 + 2 * d + 1 - s) * NF + q];
      vh += Pen[(e * 6 + f) * NF + q] * (s == 0 ? to - tn : tn - to) *
            S[((d * NF + q) * (N + 1) + (s ? N : 0)) * 3 + m];
    }
    sVh[t] = vh;
  }
  __syncthreads();
  // G_d = -nu S_d . v at the flux points of family d
  for (int t = tid; t < 3 * NL; t += blockDim.x) {
    const int d = t / NL, w = t % NL, q = w / (N + 1), r = w % (N + 1);
    double g = 0.0;
    for (int m = 0; m < 3; ++m) {
      double v;
      if (r == 0) {
        v = sVh[((2 * d) * 3 + m) * NF + q];
      } else if (r == N) {
        v = sVh[((2 * d + 1) * 3 + m) * NF + q];
      } else {
        v = 0.0;
        for (int c = 0; c < N; ++c) v += ops[O.Lint + (r - 1) * N + c] * sV[m * NP + cv_point<N>(d, q, c)];
      }
      g += S[((d * NF + q) * (N + 1) + r) * 3 + m] * v;
    }
    sG[t] = -a.nu * g;
  }
  __syncthreads();
  for (int pt = tid; pt < NP; pt += blockDim.x) {
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      double dd = 0.0;
      for (int r = 0; r <= N; ++r) dd += ops[O.M + c * (N + 1) + r] * sG[d * NL + q * (N + 1) + r];
      acc += dd;
    }
    dudt[e * NP + pt] = -ji[pt] * acc;
  }
}

}  // namespace sd
