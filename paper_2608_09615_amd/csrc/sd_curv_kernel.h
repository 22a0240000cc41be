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

// ---------------------------------------------------------------------------
// Navier-Stokes on curvilinear hexahedra (section 2.3, eqs. ns:mapped and
// adj:f; fluxes of section 4.4), FP64.  The three kernels above for the five
// conservative variables: traces T[e][f][v][q]; the gradient of every
// variable at the solution points, VS[e][m*5 + v][pt], and at the faces,
// VF[e][f][m*5 + v][q] (one-sided for the compact scheme); then
// G_d = S_d . (F_c - F_v) at the interior flux points of family d, and at
// the faces |S_d| Roe(U_L, U_R; S_d / |S_d|) - S_d . F_v(u_hat, v_hat)
// (option (a)), and du/dt = -J^-1 sum_d D_d G_d.  One element per block,
// LDS sized per n (dynamic).
// ---------------------------------------------------------------------------
namespace sd {

constexpr int kCvnThreads = 256;

template <int N>
struct CvnGradSmem {
  static constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF;
  static constexpr int U = 0, T = U + 5 * NP, UH = T + 30 * NF, UF = UH + 30 * NF, V = UF + 15 * NL;
  static constexpr int TOTAL = V + 15 * NP;   // doubles
};
template <int N>
struct CvnRhsSmem {
  static constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF;
  static constexpr int V = 0, U = V + 15 * NP, TO = U + 5 * NP, TN = TO + 30 * NF, VH = TN + 30 * NF,
                       G = VH + 90 * NF;
  static constexpr int TOTAL = G + 15 * NL;
};

template <int N>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_traces(const double *__restrict__ U, double *__restrict__ T,
                                                            const double *__restrict__ ops, long long ne) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N;
  const long long e = blockIdx.x;
  if (e >= ne) return;
  for (int t = threadIdx.x; t < 30 * NF; t += blockDim.x) {
    const int f = t / (5 * NF), w = t % (5 * NF), v = w / NF, q = w % NF, d = f >> 1, s = f & 1;
    const double *u = U + (e * 5 + v) * NP;
    double acc = 0.0;
    for (int c = 0; c < N; ++c) acc += ops[O.Lend + s * N + c] * u[cv_point<N>(d, q, c)];
    T[e * 30 * NF + t] = acc;
  }
}

template <int N>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_grad(const double *__restrict__ U, const double *__restrict__ T,
                                                          const double *__restrict__ Sf,
                                                          const double *__restrict__ Jinv,
                                                          const double *__restrict__ ops, KArgs a, int compact,
                                                          double *__restrict__ VF, double *__restrict__ VS) {
  using SM = CvnGradSmem<N>;
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = SM::NP, NF = SM::NF, NL = SM::NL;
  extern __shared__ double smem_cvn[];
  double *su = smem_cvn + SM::U, *sT = smem_cvn + SM::T, *sUh = smem_cvn + SM::UH, *sUF = smem_cvn + SM::UF,
         *sV = smem_cvn + SM::V;
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const double *ji = Jinv + e * NP;
  const double *S = Sf + e * 9 * NL;
  for (int t = tid; t < 5 * NP; t += nth) su[t] = U[e * 5 * NP + t];
  for (int t = tid; t < 30 * NF; t += nth) {
    const int f = t / (5 * NF), w = t % (5 * NF), d = f >> 1, s = f & 1;
    const double own = T[e * 30 * NF + t];
    const double oth = T[nbr(a, e, d, s) * 30 * NF + (2 * d + 1 - s) * 5 * NF + w];
    sT[t] = own;
    sUh[t] = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
  }
  __syncthreads();
  // continuous solution of every variable at the flux points of every family
  for (int t = tid; t < 15 * NL; t += nth) {
    const int d = t / (5 * NL), w = t % (5 * NL), v = w / NL, l = w % NL, q = l / (N + 1), r = l % (N + 1);
    double val;
    if (r == 0) {
      val = sUh[((2 * d) * 5 + v) * NF + q];
    } else if (r == N) {
      val = sUh[((2 * d + 1) * 5 + v) * NF + q];
    } else {
      val = 0.0;
      for (int c = 0; c < N; ++c) val += ops[O.Lint + (r - 1) * N + c] * su[v * NP + cv_point<N>(d, q, c)];
    }
    sUF[t] = val;
  }
  __syncthreads();
  // gradient of every variable at the solution points
  for (int t = tid; t < 15 * NP; t += nth) {
    const int mv = t / NP, pt = t % NP, m = mv / 5, v = mv % 5;
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      double dd = 0.0;
      for (int r = 0; r <= N; ++r)
        dd += ops[O.M + c * (N + 1) + r] *
              (sUF[(d * 5 + v) * NL + q * (N + 1) + r] * S[((d * NF + q) * (N + 1) + r) * 3 + m]);
      acc += dd;
    }
    const double g = ji[pt] * acc;
    sV[t] = g;
    VS[e * 15 * NP + t] = g;
  }
  __syncthreads();
  // values at the faces: one-sided (compact: the family-d solution of face s
  // keeps the own trace at the other face) or standard
  for (int t = tid; t < 90 * NF; t += nth) {
    const int f = t / (15 * NF), w = t % (15 * NF), mv = w / NF, q = w % NF, m = mv / 5, v = mv % 5;
    const int d = f >> 1, s = f & 1;
    double corr = 0.0;
    int rend = 0;
    if (compact) {
      const int so = 1 - s;
      rend = so == 0 ? 0 : N;
      corr = (sT[((2 * d + so) * 5 + v) * NF + q] - sUh[((2 * d + so) * 5 + v) * NF + q]) *
             S[((d * NF + q) * (N + 1) + rend) * 3 + m];
    }
    double acc = 0.0;
    for (int c = 0; c < N; ++c) {
      const int pt = cv_point<N>(d, q, c);
      double g = sV[mv * NP + pt];
      if (compact) g += ji[pt] * (ops[O.M + c * (N + 1) + rend] * corr);
      acc += ops[O.Lend + s * N + c] * g;
    }
    VF[e * 90 * NF + t] = acc;
  }
}

template <int N>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_rhs(const double *__restrict__ U, const double *__restrict__ T,
                                                         const double *__restrict__ VF,
                                                         const double *__restrict__ VS,
                                                         const double *__restrict__ Sf,
                                                         const double *__restrict__ Jinv,
                                                         const double *__restrict__ ops, KArgs a,
                                                         double *__restrict__ dudt) {
  using SM = CvnRhsSmem<N>;
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = SM::NP, NF = SM::NF, NL = SM::NL;
  extern __shared__ double smem_cvn[];
  double *sV = smem_cvn + SM::V, *su = smem_cvn + SM::U, *sTo = smem_cvn + SM::TO, *sTn = smem_cvn + SM::TN,
         *sVh = smem_cvn + SM::VH, *sG = smem_cvn + SM::G;
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  const double *S = Sf + e * 9 * NL;
  const double *ji = Jinv + e * NP;
  for (int t = tid; t < 15 * NP; t += nth) sV[t] = VS[e * 15 * NP + t];
  for (int t = tid; t < 5 * NP; t += nth) su[t] = U[e * 5 * NP + t];
  for (int t = tid; t < 30 * NF; t += nth) {
    const int f = t / (5 * NF), w = t % (5 * NF), d = f >> 1, s = f & 1;
    sTo[t] = T[e * 30 * NF + t];
    sTn[t] = T[nbr(a, e, d, s) * 30 * NF + (2 * d + 1 - s) * 5 * NF + w];
  }
  for (int t = tid; t < 90 * NF; t += nth) {
    const int f = t / (15 * NF), w = t % (15 * NF), d = f >> 1, s = f & 1;
    const double own = VF[e * 90 * NF + t];
    const double oth = VF[nbr(a, e, d, s) * 90 * NF + (2 * d + 1 - s) * 15 * NF + w];
    sVh[t] = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
  }
  __syncthreads();
  // G_d at the flux points of family d: one item per (d, line, flux point)
  const NsConst<double> c(a);
  for (int t = tid; t < 3 * NL; t += nth) {
    const int d = t / NL, l = t % NL, q = l / (N + 1), r = l % (N + 1);
    const double *srow = S + ((d * NF + q) * (N + 1) + r) * 3;
    const double sv[3] = {srow[0], srow[1], srow[2]};
    double G[5];
    if (r == 0 || r == N) {
      const int s = r == 0 ? 0 : 1, f = 2 * d + s;
      double UL[5], UR[5], Uh[5], Vh[15];
      for (int v = 0; v < 5; ++v) {
        const double own = sTo[(f * 5 + v) * NF + q], oth = sTn[(f * 5 + v) * NF + q];
        UL[v] = s == 0 ? oth : own;
        UR[v] = s == 0 ? own : oth;
        Uh[v] = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
      }
      for (int mv = 0; mv < 15; ++mv) Vh[mv] = sVh[(f * 15 + mv) * NF + q];
      const double nrm = sqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
      const double nv[3] = {sv[0] / nrm, sv[1] / nrm, sv[2] / nrm};
      double Fr[5], Fv[5];
      ns_roe_dir(c, UL, UR, nv, Fr);
      Prim<double> st = ns_prim(c, Uh);
      ns_visc_dir(c, st, Vh, sv, Fv);
      for (int v = 0; v < 5; ++v) G[v] = nrm * Fr[v] - Fv[v];
    } else {
      double Uf[5], Vf[15];
      for (int v = 0; v < 5; ++v) {
        double acc = 0.0;
        for (int cc = 0; cc < N; ++cc) acc += ops[O.Lint + (r - 1) * N + cc] * su[v * NP + cv_point<N>(d, q, cc)];
        Uf[v] = acc;
      }
      for (int mv = 0; mv < 15; ++mv) {
        double acc = 0.0;
        for (int cc = 0; cc < N; ++cc) acc += ops[O.Lint + (r - 1) * N + cc] * sV[mv * NP + cv_point<N>(d, q, cc)];
        Vf[mv] = acc;
      }
      Prim<double> st = ns_prim(c, Uf);
      double Fc[5], Fv[5];
      ns_conv_dir(c, Uf, st, sv, Fc);
      ns_visc_dir(c, st, Vf, sv, Fv);
      for (int v = 0; v < 5; ++v) G[v] = Fc[v] - Fv[v];
    }
    for (int v = 0; v < 5; ++v) sG[(d * 5 + v) * NL + l] = G[v];
  }
  __syncthreads();
  for (int t = tid; t < 5 * NP; t += nth) {
    const int v = t / NP, pt = t % NP;
    double acc = 0.0;
    for (int d = 0; d < 3; ++d) {
      int q, cc;
      cv_line_of<N>(pt, d, q, cc);
      double dd = 0.0;
      for (int r = 0; r <= N; ++r) dd += ops[O.M + cc * (N + 1) + r] * sG[(d * 5 + v) * NL + q * (N + 1) + r];
      acc += dd;
    }
    dudt[e * 5 * NP + t] = -ji[pt] * acc;
  }
}

}  // namespace sd
