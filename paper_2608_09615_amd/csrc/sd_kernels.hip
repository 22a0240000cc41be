// HIP kernels of the SD right-hand side for gfx950 (generic path: any
// supported n, dimension, physics and precision).
//
// Data flow of one right-hand side evaluation:
//   k_traces      element-local: face traces T = c_s^T L u along each
//                 direction, the element-local part NN of the normal
//                 gradient trace, and the 12 edge traces (3-D);
//   k_br1_cross   BR1 only: adds to NN the opposite-face term of the
//                 standard gradient, which is what widens BR1's stencil;
//   k_rhs         fused per element: common solution at the faces, the
//                 auxiliary gradient at the solution points, the common
//                 gradient at the faces (own side and, rebuilt from the
//                 neighbour's traces, the neighbour side), fluxes at every
//                 flux point of the three families and their divergence.
// The gradient and face-gradient algebra is the one of sections 2.1-2.3,
// rearranged by linearity (no approximation):
//   grad_m u^S = (2/h_m) [ (M L)_m u + M c_L (u_hat_L - T_L) + M c_R (u_hat_R - T_R) ]
//   one-sided normal face value (compact) = (2/h_d) [ N_s + k_s (u_hat_s - T_s) ]
// with N_s = c_s^T L M L u and k_s = (L M)[s][s]; BR1 adds
// (L M)[s][s'] (u_hat_s' - T_s').  Transverse components are the standard
// gradient interpolated to the face (section 2.3: corrected fluxes are only
// differentiated along their own direction).
#include <hip/hip_runtime.h>

#include "sd_internal.h"
#include "sd_physics.h"

namespace sd {

// point index of coordinate c along direction d on the face-family line q
template <int DIM, int N>
__device__ __forceinline__ void line_of(int d, int q, int &base, int &stride) {
  if constexpr (DIM == 1) {
    base = 0; stride = 1;
  } else {
    if (d == 0) { base = q * N; stride = 1; }
    else if (d == 1) { base = (q % N) + N * N * (q / N); stride = N; }
    else { base = q; stride = N * N; }
  }
}

// coordinate along direction m and face-family index q of point pt
template <int DIM, int N>
__device__ __forceinline__ void coord_of(int pt, int m, int &a, int &q) {
  if constexpr (DIM == 1) {
    a = pt; q = 0;
  } else {
    int i = pt % N, j = (pt / N) % N, k = pt / (N * N);
    if (m == 0) { a = i; q = k * N + j; }
    else if (m == 1) { a = j; q = k * N + i; }
    else { a = k; q = j * N + i; }
  }
}

// neighbour of element e across face (d, s)
__device__ __forceinline__ long long nbr(const KArgs &a, long long e, int d, int s) {
  long long nx = a.nel[0], ny = a.nel[1];
  long long ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
  long long c[3] = {ex, ey, ez};
  int n = a.nel[d];
  c[d] = s ? (c[d] + 1 == n ? 0 : c[d] + 1) : (c[d] == 0 ? n - 1 : c[d] - 1);
  return c[0] + nx * (c[1] + ny * c[2]);
}

// edge id of the edge shared by faces (d1, s1) and (d2, s2), d1 != d2
__device__ __forceinline__ int edge_id(int d1, int s1, int d2, int s2) {
  int lo = d1 < d2 ? d1 : d2, hi = d1 < d2 ? d2 : d1;
  int slo = d1 < d2 ? s1 : s2, shi = d1 < d2 ? s2 : s1;
  int P = (lo == 0 && hi == 1) ? 0 : (lo == 0 ? 1 : 2);
  return 4 * P + 2 * slo + shi;
}

template <int DIM, int N, int NV, typename R>
__global__ void __launch_bounds__(256) k_traces(const double *__restrict__ U, R *__restrict__ X,
                                                const R *__restrict__ ops, KArgs a) {
  constexpr int NP = ipow_c(N, DIM), NF = ipow_c(N, DIM - 1);
  constexpr int XS = trace_stride(DIM, N, NV), FS = trace_face_stride(DIM, N, NV);
  constexpr int EO = trace_edge_off(DIM, N, NV);
  constexpr OpsLayout O = ops_layout(N);
  extern __shared__ char smem_raw[];
  R *sU = reinterpret_cast<R *>(smem_raw);
  const long long e0 = (long long)blockIdx.x * a.epb;
  const int nb = (int)min((long long)a.epb, a.ne - e0);
  for (int t = threadIdx.x; t < nb * NV * NP; t += blockDim.x) {
    int v = (t / NP) % NV;
    sU[t] = (R)(U[e0 * NV * NP + t] - a.U0[v]);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nb * 2 * DIM * NV * NF; t += blockDim.x) {
    int q = t % NF, r = t / NF;
    int v = r % NV; r /= NV;
    int f = r % (2 * DIM), el = r / (2 * DIM);
    int d = f >> 1, s = f & 1, base, stride;
    line_of<DIM, N>(d, q, base, stride);
    const R *u = sU + (el * NV + v) * NP;
    R tr = R(0), nn = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      R uv = u[base + c * stride];
      tr += ops[O.Lend + s * N + c] * uv;
      nn += ops[O.rrow + s * N + c] * uv;
    }
    R *xe = X + (e0 + el) * XS + f * FS;
    xe[v * NF + q] = tr;
    xe[NV * NF + v * NF + q] = nn;
  }
  if constexpr (DIM == 3) {
    for (int t = threadIdx.x; t < nb * 12 * NV * N; t += blockDim.x) {
      int at = t % N, r = t / N;
      int v = r % NV; r /= NV;
      int ed = r % 12, el = r / 12;
      int P = ed >> 2, slo = (ed >> 1) & 1, shi = ed & 1;
      int dlo = P == 2 ? 1 : 0, dhi = P == 0 ? 1 : 2, dt = 3 - dlo - dhi;
      const R *u = sU + (el * NV + v) * NP;
      R acc = R(0);
      for (int c2 = 0; c2 < N; ++c2) {
        R inner = R(0);
        for (int c1 = 0; c1 < N; ++c1) {
          int idx[3];
          idx[dlo] = c1; idx[dhi] = c2; idx[dt] = at;
          inner += ops[O.Lend + slo * N + c1] * u[(idx[2] * N + idx[1]) * N + idx[0]];
        }
        acc += ops[O.Lend + shi * N + c2] * inner;
      }
      X[(e0 + el) * XS + EO + (ed * NV + v) * N + at] = acc;
    }
  }
}

// BR1: NN_s += (L M)[s][s'] * u_hat_{s'}  (the common value at the opposite face)
template <int DIM, int N, int NV, typename R>
__global__ void __launch_bounds__(256) k_br1_cross(R *__restrict__ X, const R *__restrict__ ops, KArgs a) {
  constexpr int NF = ipow_c(N, DIM - 1);
  constexpr int XS = trace_stride(DIM, N, NV), FS = trace_face_stride(DIM, N, NV);
  constexpr OpsLayout O = ops_layout(N);
  long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long total = a.ne * 2 * DIM * NV * NF;
  if (t >= total) return;
  int q = (int)(t % NF);
  long long r = t / NF;
  int v = (int)(r % NV); r /= NV;
  int f = (int)(r % (2 * DIM));
  long long e = r / (2 * DIM);
  int d = f >> 1, s = f & 1, so = 1 - s;
  long long nb = nbr(a, e, d, so);
  R mine = X[e * XS + (2 * d + so) * FS + v * NF + q];
  R theirs = X[nb * XS + (2 * d + s) * FS + v * NF + q];
  R uh = so == 0 ? R(0.5) * (theirs + mine) : R(0.5) * (mine + theirs);
  X[e * XS + f * FS + NV * NF + v * NF + q] += ops[O.kapx + s] * uh;
}

template <int DIM, int N, int NV>
struct RhsSmem {
  static constexpr int NP = ipow_c(N, DIM), NF = ipow_c(N, DIM - 1), NFACE = 2 * DIM;
  static constexpr int U = 0;
  static constexpr int G = U + NV * NP;
  static constexpr int UH = G + DIM * NV * NP;
  static constexpr int TO = UH + NFACE * NV * NF;
  static constexpr int TN = TO + NFACE * NV * NF;
  static constexpr int VH = TN + NFACE * NV * NF;
  static constexpr int F = VH + NFACE * DIM * NV * NF;
  static constexpr int RR = F + NV * (N + 1) * NF;
  static constexpr int TOTAL = RR + NV * NP;   // values per element
};

template <int DIM, int N, int NV, int PHYS, typename R>
__global__ void __launch_bounds__(256) k_rhs(const double *__restrict__ U, const R *__restrict__ X,
                                             const R *__restrict__ ops, double *__restrict__ dudt,
                                             KArgs a) {
  using SM = RhsSmem<DIM, N, NV>;
  constexpr int NP = SM::NP, NF = SM::NF, NFACE = SM::NFACE;
  constexpr int XS = trace_stride(DIM, N, NV), FS = trace_face_stride(DIM, N, NV);
  constexpr int EO = trace_edge_off(DIM, N, NV);
  constexpr OpsLayout O = ops_layout(N);
  extern __shared__ char smem_raw[];
  R *sm = reinterpret_cast<R *>(smem_raw);
  const long long e0 = (long long)blockIdx.x * a.epb;
  const int nb = (int)min((long long)a.epb, a.ne - e0);
  auto S = [&](int el, int off) { return sm + el * SM::TOTAL + off; };

  // A: state (reference removed) and zeroed residual
  for (int t = threadIdx.x; t < nb * NV * NP; t += blockDim.x) {
    int el = t / (NV * NP), r = t % (NV * NP), v = r / NP;
    S(el, SM::U)[r] = (R)(U[e0 * NV * NP + t] - a.U0[v]);
    S(el, SM::RR)[r] = R(0);
  }
  // B: own and neighbour traces, common solution u_hat = (u_left + u_right)/2
  for (int t = threadIdx.x; t < nb * NFACE * NV * NF; t += blockDim.x) {
    int el = t / (NFACE * NV * NF), r = t % (NFACE * NV * NF);
    int f = r / (NV * NF), vq = r % (NV * NF);
    int d = f >> 1, s = f & 1;
    long long e = e0 + el, en = nbr(a, e, d, s);
    R own = X[e * XS + f * FS + vq];
    R oth = X[en * XS + (2 * d + (1 - s)) * FS + vq];
    S(el, SM::TO)[r] = own;
    S(el, SM::TN)[r] = oth;
    S(el, SM::UH)[r] = s == 0 ? R(0.5) * (oth + own) : R(0.5) * (own + oth);
  }
  __syncthreads();
  // C: auxiliary gradient at the solution points, [m][v][pt]
  for (int t = threadIdx.x; t < nb * DIM * NV * NP; t += blockDim.x) {
    int el = t / (DIM * NV * NP), r = t % (DIM * NV * NP);
    int m = r / (NV * NP), vp = r % (NV * NP), v = vp / NP, pt = vp % NP;
    int am, qm, base, stride;
    coord_of<DIM, N>(pt, m, am, qm);
    line_of<DIM, N>(m, qm, base, stride);
    const R *u = S(el, SM::U) + v * NP;
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) acc += ops[O.D + am * N + c] * u[base + c * stride];
    int fi0 = ((2 * m) * NV + v) * NF + qm, fi1 = ((2 * m + 1) * NV + v) * NF + qm;
    acc += ops[O.Mc + am] * (S(el, SM::UH)[fi0] - S(el, SM::TO)[fi0]);
    acc += ops[O.Mc + N + am] * (S(el, SM::UH)[fi1] - S(el, SM::TO)[fi1]);
    S(el, SM::G)[r] = (R)a.two_over_h[m] * acc;
  }
  __syncthreads();
  // D: common gradient at every face point, [f][m][v][q]
  for (int t = threadIdx.x; t < nb * NFACE * DIM * NV * NF; t += blockDim.x) {
    int el = t / (NFACE * DIM * NV * NF), r = t % (NFACE * DIM * NV * NF);
    int f = r / (DIM * NV * NF), r2 = r % (DIM * NV * NF);
    int m = r2 / (NV * NF), v = (r2 / NF) % NV, q = r2 % NF;
    int d = f >> 1, s = f & 1, so = 1 - s;
    long long e = e0 + el, en = nbr(a, e, d, s);
    int fv = (f * NV + v) * NF + q;
    R uh = S(el, SM::UH)[fv];
    R vown, voth;
    if (m == d) {
      R two_h = (R)a.two_over_h[d];
      vown = two_h * (X[e * XS + f * FS + NV * NF + v * NF + q] + ops[O.kap + s] * uh);
      voth = two_h * (X[en * XS + (2 * d + so) * FS + NV * NF + v * NF + q] + ops[O.kap + so] * uh);
    } else {
      // own side: the standard gradient interpolated to the face
      int base, stride;
      line_of<DIM, N>(d, q, base, stride);
      const R *g = S(el, SM::G) + (m * NV + v) * NP;
      R acc = R(0);
#pragma unroll
      for (int c = 0; c < N; ++c) acc += ops[O.Lend + s * N + c] * g[base + c * stride];
      vown = acc;
      if constexpr (DIM == 3) {
        // neighbour side: its standard gradient at its face (d, so), rebuilt
        // on the face from its trace and the edge traces of its neighbours
        // along m: (2/h_m) [ D_m T + M c_L (e_hat_L - e_L) + M c_R (e_hat_R - e_R) ]
        int t3 = 3 - d - m;
        int am, at;
        {  // coordinates of q along m and along the third axis t3
          int lo = m < t3 ? m : t3;
          int a_lo = q % N, a_hi = q / N;
          am = (lo == m) ? a_lo : a_hi;
          at = (lo == m) ? a_hi : a_lo;
        }
        const R *tn = S(el, SM::TN) + (f * NV + v) * NF;
        auto qidx = [&](int cm) { return (m < t3) ? (at * N + cm) : (cm * N + at); };
        R dT = R(0), eL = R(0), eR = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) {
          R tv = tn[qidx(c)];
          dT += ops[O.D + am * N + c] * tv;
          eL += ops[O.Lend + c] * tv;
          eR += ops[O.Lend + N + c] * tv;
        }
        long long nL = nbr(a, en, m, 0), nR = nbr(a, en, m, 1);
        R eLn = X[nL * XS + EO + (edge_id(d, so, m, 1) * NV + v) * N + at];
        R eRn = X[nR * XS + EO + (edge_id(d, so, m, 0) * NV + v) * N + at];
        R ehL = R(0.5) * (eLn + eL), ehR = R(0.5) * (eR + eRn);
        voth = (R)a.two_over_h[m] *
               (dT + ops[O.Mc + am] * (ehL - eL) + ops[O.Mc + N + am] * (ehR - eR));
      } else {
        voth = R(0);
      }
    }
    R vh = s == 0 ? R(0.5) * (voth + vown) : R(0.5) * (vown + voth);
    if (m == d) {
      // interior penalty on the normal component: tau_d (u_R - u_L)
      R own = S(el, SM::TO)[fv], oth = S(el, SM::TN)[fv];
      vh += (R)a.tau[d] * (s == 0 ? own - oth : oth - own);
    }
    S(el, SM::VH)[r] = vh;
  }
  __syncthreads();
  // E: per family d, fluxes at the n+1 flux points of every line, then the
  // divergence  du/dt -= (2/h_d) M F
  for (int d = 0; d < DIM; ++d) {
    for (int t = threadIdx.x; t < nb * (N + 1) * NF; t += blockDim.x) {
      int el = t / ((N + 1) * NF), r = t % ((N + 1) * NF);
      int rr = r / NF, q = r % NF;
      R Fv[NV];
      if (rr == 0 || rr == N) {
        int s = rr == 0 ? 0 : 1, f = 2 * d + s;
        R UL[NV], UR[NV], Uh[NV], Vh[DIM * NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          int fv = (f * NV + v) * NF + q;
          R own = S(el, SM::TO)[fv], oth = S(el, SM::TN)[fv];
          UL[v] = s == 0 ? oth : own;
          UR[v] = s == 0 ? own : oth;
          Uh[v] = S(el, SM::UH)[fv];
#pragma unroll
          for (int m = 0; m < DIM; ++m) Vh[m * NV + v] = S(el, SM::VH)[((f * DIM + m) * NV + v) * NF + q];
        }
        face_flux<PHYS, NV, R>(a, d, UL, UR, Uh, Vh, Fv);
      } else {
        int base, stride;
        line_of<DIM, N>(d, q, base, stride);
        const R *li = ops + O.Lint + (rr - 1) * N;
        R Uf[NV], Gf[DIM * NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const R *u = S(el, SM::U) + v * NP;
          R acc = R(0);
#pragma unroll
          for (int c = 0; c < N; ++c) acc += li[c] * u[base + c * stride];
          Uf[v] = acc;
#pragma unroll
          for (int m = 0; m < DIM; ++m) {
            const R *g = S(el, SM::G) + (m * NV + v) * NP;
            R ag = R(0);
#pragma unroll
            for (int c = 0; c < N; ++c) ag += li[c] * g[base + c * stride];
            Gf[m * NV + v] = ag;
          }
        }
        interior_flux<PHYS, NV, R>(a, d, Uf, Gf, Fv);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) S(el, SM::F)[(v * (N + 1) + rr) * NF + q] = Fv[v];
    }
    __syncthreads();
    for (int t = threadIdx.x; t < nb * NV * NP; t += blockDim.x) {
      int el = t / (NV * NP), r = t % (NV * NP), v = r / NP, pt = r % NP;
      int ad, qd;
      coord_of<DIM, N>(pt, d, ad, qd);
      const R *Fl = S(el, SM::F) + v * (N + 1) * NF;
      R acc = R(0);
#pragma unroll
      for (int c = 0; c <= N; ++c) acc += ops[O.M + ad * (N + 1) + c] * Fl[c * NF + qd];
      S(el, SM::RR)[r] -= (R)a.two_over_h[d] * acc;
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < nb * NV * NP; t += blockDim.x) {
    int el = t / (NV * NP), r = t % (NV * NP);
    dudt[e0 * NV * NP + t] = (double)S(el, SM::RR)[r];
  }
}

// ---------------------------------------------------------------------------
// Runge-Kutta (classical, four stages), FP64.
// ---------------------------------------------------------------------------
__global__ void k_rk_stage(const double *__restrict__ u, const double *__restrict__ k,
                           double *__restrict__ w, double *__restrict__ acc, double a, double c,
                           int first, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double ki = k[i];
  acc[i] = first ? ki : acc[i] + c * ki;
  w[i] = u[i] + a * ki;
}

__global__ void k_rk_final(double *__restrict__ u, const double *__restrict__ k4,
                           const double *__restrict__ acc, double dt6, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  u[i] = u[i] + dt6 * (acc[i] + k4[i]);
}

// SSP-RK(5,4) combinations (Shu-Osher form): out = a0 x0 + a1 x1 + b k
__global__ void k_lincomb(const double *__restrict__ x0, const double *__restrict__ x1,
                          const double *__restrict__ k, double *__restrict__ out, double a0, double a1, double b,
                          long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a0 * x0[i] + a1 * x1[i] + b * k[i];
}

// last SSP-RK(5,4) stage: out = a2 u2 + a3 u3 + b3 L3 + a4 u4 + b4 L4
__global__ void k_ssp_final(const double *__restrict__ u2, const double *__restrict__ u3,
                            const double *__restrict__ L3, const double *__restrict__ u4,
                            const double *__restrict__ L4, double *__restrict__ out, double a2, double a3,
                            double b3, double a4, double b4, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  out[i] = a2 * u2[i] + a3 * u3[i] + b3 * L3[i] + a4 * u4[i] + b4 * L4[i];
}

// ---------------------------------------------------------------------------
// Diagnostics (FP64): per block partial sums of the Gauss-quadrature
// integrals, then one block sums the partials in a fixed order.
// ---------------------------------------------------------------------------
constexpr int kDiagVals = 10;  // ke, ens, mass, mom0..2, energy, umax, bad, smax
__host__ __device__ constexpr bool diag_is_max(int c) { return c >= 7; }

template <int N>
__global__ void __launch_bounds__(256) k_diag(const double *__restrict__ U, const double *__restrict__ X,
                                              const double *__restrict__ ops, double *__restrict__ part,
                                              KArgs a, double J) {
  constexpr int DIM = 3, NV = 5, NP = N * N * N, NF = N * N;
  constexpr int XS = trace_stride(DIM, N, NV), FS = trace_face_stride(DIM, N, NV);
  constexpr OpsLayout O = ops_layout(N);
  extern __shared__ char smem_raw[];
  double *sU = reinterpret_cast<double *>(smem_raw);           // epb * NV * NP
  double *sG = sU + a.epb * NV * NP;                            // epb * 3 * NV * NP
  double *red = sG + a.epb * 3 * NV * NP;                       // blockDim * kDiagVals
  const long long e0 = (long long)blockIdx.x * a.epb;
  const int nb = (int)min((long long)a.epb, a.ne - e0);
  for (int t = threadIdx.x; t < nb * NV * NP; t += blockDim.x) sU[t] = U[e0 * NV * NP + t];
  __syncthreads();
  for (int t = threadIdx.x; t < nb * 3 * NV * NP; t += blockDim.x) {
    int el = t / (3 * NV * NP), r = t % (3 * NV * NP);
    int m = r / (NV * NP), vp = r % (NV * NP), v = vp / NP, pt = vp % NP;
    int am, qm, base, stride;
    coord_of<DIM, N>(pt, m, am, qm);
    line_of<DIM, N>(m, qm, base, stride);
    const double *u = sU + (el * NV + v) * NP;
    double acc = 0.0;
    for (int c = 0; c < N; ++c) acc += ops[O.D + am * N + c] * u[base + c * stride];
    long long e = e0 + el;
    for (int s = 0; s < 2; ++s) {
      long long en = nbr(a, e, m, s);
      double own = X[e * XS + (2 * m + s) * FS + v * NF + qm];
      double oth = X[en * XS + (2 * m + 1 - s) * FS + v * NF + qm];
      double uh = s == 0 ? 0.5 * (oth + own) : 0.5 * (own + oth);
      acc += ops[O.Mc + s * N + am] * (uh - own);
    }
    sG[t] = a.two_over_h[m] * acc;
  }
  __syncthreads();
  double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int t = threadIdx.x; t < nb * NP; t += blockDim.x) {
    int el = t / NP, pt = t % NP;
    int i = pt % N, j = (pt / N) % N, k = pt / (N * N);
    double wq = J * ops[O.ws + i] * ops[O.ws + j] * ops[O.ws + k];
    double Uq[5];
    for (int v = 0; v < 5; ++v) {
      Uq[v] = sU[(el * NV + v) * NP + pt];
      if (!isfinite(Uq[v])) acc[8] = 1.0;
    }
    double vel[3] = {Uq[1] / Uq[0], Uq[2] / Uq[0], Uq[3] / Uq[0]};
    double du[3][3];
    for (int c = 0; c < 3; ++c)
      for (int m = 0; m < 3; ++m) {
        const double *g = sG + ((el * 3 + m) * NV) * NP;
        du[c][m] = (g[(1 + c) * NP + pt] - vel[c] * g[pt]) / Uq[0];
      }
    double om0 = du[2][1] - du[1][2], om1 = du[0][2] - du[2][0], om2 = du[1][0] - du[0][1];
    double v2 = vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2];
    acc[0] += wq * 0.5 * v2;
    acc[1] += wq * (om0 * om0 + om1 * om1 + om2 * om2);
    acc[2] += wq * Uq[0];
    acc[3] += wq * Uq[1];
    acc[4] += wq * Uq[2];
    acc[5] += wq * Uq[3];
    acc[6] += wq * Uq[4];
    acc[7] = fmax(acc[7], sqrt(v2));
    // fastest acoustic signal |u| + c, c^2 = gamma P / rho
    // (infinite where the state is inadmissible: rho <= 0 or P < 0)
    const double P = a.gm1 * (Uq[4] - 0.5 * Uq[0] * v2);
    const double sp = (Uq[0] > 0.0 && P >= 0.0) ? sqrt(v2) + sqrt((a.gm1 + 1.0) * P / Uq[0]) : HUGE_VAL;
    acc[9] = fmax(acc[9], sp);
  }
  for (int c = 0; c < kDiagVals; ++c) red[threadIdx.x * kDiagVals + c] = acc[c];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < kDiagVals; ++c) {
        double o = red[(threadIdx.x + w) * kDiagVals + c];
        double &m = red[threadIdx.x * kDiagVals + c];
        m = diag_is_max(c) ? fmax(m, o) : m + o;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < kDiagVals; ++c) part[blockIdx.x * kDiagVals + c] = red[c];
}

__global__ void k_diag_final(const double *__restrict__ part, int nparts, double *__restrict__ out) {
  __shared__ double red[256 * kDiagVals];
  double acc[kDiagVals] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int c = 0; c < kDiagVals; ++c) {
      double o = part[b * kDiagVals + c];
      acc[c] = diag_is_max(c) ? fmax(acc[c], o) : acc[c] + o;
    }
  for (int c = 0; c < kDiagVals; ++c) red[threadIdx.x * kDiagVals + c] = acc[c];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int c = 0; c < kDiagVals; ++c) {
        double o = red[(threadIdx.x + w) * kDiagVals + c];
        double &m = red[threadIdx.x * kDiagVals + c];
        m = diag_is_max(c) ? fmax(m, o) : m + o;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < kDiagVals; ++c) out[c] = red[c];
}

}  // namespace sd

#include "sd_ns_kernel.h"
#include "sd_mlp.h"
#include "sd_bloch_kernel.h"
#include "sd_curv_kernel.h"
#include "sd_dispatch.inc"
#include "sd_closure.inc"
#include "sd_bloch.inc"
#include "sd_run1d.inc"
#include "sd_curv.inc"
