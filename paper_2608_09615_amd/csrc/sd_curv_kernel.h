// SD diffusion right-hand side on curvilinear hexahedra (section 2.3 with a
// general adjoint S), scalar u_t = nu lap u, in FP64 or FP32 (the compute
// type R of the metric terms, the work buffers and the arithmetic; the state
// is read and the RHS written in FP64).
//
// Geometry per element: S row d (S_d0, S_d1, S_d2) at the flux points of
// family d and 1/det J at the solution points, stored line-major: for
// family d the n^2 lines along d are numbered q by the two transverse
// indices (d = 0: q = j + n k; d = 1: q = i + n k; d = 2: q = i + n j) and
// the n + 1 flux points of a line by r.  Face arrays use the same q, so the
// two elements of a face index its points alike.  The two elements of a
// face also hold the same S_d there: the row is built from the tangential
// derivatives of the mapping, which only the face's nodes set.
//
// Three kernels, one element per block (cv_threads<N>() lanes):
//   k_cv_traces  the solution at the six faces, T[e][f][q] (f = 2 d + s);
//   k_cv_grad    everything that needs the element alone and its
//                neighbours' traces, with the metric rows read once into
//                LDS: common solution at the faces, the continuous solution
//                at the flux points, the auxiliary variable v_m at the
//                solution points (J^-1 sum_d D_d(u^{Fd,C} S_dm)); its values
//                at the faces, one-sided (compact: the family-d solution
//                keeps the own trace at the other face, which adds
//                J^-1 M[:, end] (T - u_hat) S_dm to v_m along the lines) or
//                standard (BR1), stored projected on the face's S row,
//                W = S_d . v (the common flux only needs that component);
//                the fluxes G_d = -nu S_d . v at the interior flux points and
//                their part of the divergence, sum_d sum_{0<r<n} M[c][r] G_d;
//   k_cv_face    the common flux at the faces, -nu (W_L + W_R) / 2 (plus the
//                interior penalty when on: -nu P' (u_R - u_L), P' = tau |S_d|
//                stored per face point), and du/dt = -J^-1 (that part + the
//                face columns of M times the face fluxes).
// Per element the path moves the state, the metric rows and 1/det J once,
// plus the traces, W and the partial divergence: no gradient round trip.
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

// trace at point q of face f = 2 d + s from the n values v[c] of its line
// (already in the compute type): k_cv_traces and k_cv_grad evaluate an
// element's traces with this same sequence of operations on the same
// rounded values, so both see the same traces
template <int N, typename R>
__device__ __forceinline__ R cv_dot_end(const R *__restrict__ ops, const R *v, int s) {
  constexpr OpsLayout O = ops_layout(N);
  R acc = R(0);
#pragma unroll
  for (int c = 0; c < N; ++c) acc += ops[O.Lend + s * N + c] * v[c];
  return acc;
}

// the state in the compute type, minus the subtracted constant (the
// reference state of the Navier-Stokes variables; 0 otherwise)
template <typename R>
__device__ __forceinline__ R cv_in(double u, double shift) {
  return (R)(u - shift);
}

template <int N, typename R>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_traces(const double *__restrict__ U, R *__restrict__ T,
                                                          const R *__restrict__ ops, long long ne) {
  constexpr int NP = N * N * N, NF = N * N;
  const long long e = blockIdx.x;
  if (e >= ne) return;
  const double *u = U + e * NP;
  // every read of a lane issued before the first trace (clamped indices)
  constexpr int NTH = cv_threads<N>(), IT = (6 * NF + NTH - 1) / NTH;
  const int tid = threadIdx.x;
  double x[IT][N];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = min(tid + i * NTH, 6 * NF - 1), f = t / NF, q = t % NF, d = f >> 1;
#pragma unroll
    for (int c = 0; c < N; ++c) x[i][c] = u[cv_point<N>(d, q, c)];
  }
  // keeps the compiler from moving the reads down to their uses
  __asm__ __volatile__("" ::: "memory");
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = tid + i * NTH;
    if (t >= 6 * NF) break;
    R v[N];
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = cv_in<R>(x[i][c], 0.0);
    T[e * 6 * NF + t] = cv_dot_end<N>(ops, v, (t / NF) & 1);
  }
}

template <int N, typename R>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_grad(const double *__restrict__ U, const R *__restrict__ T,
                                                        const R *__restrict__ Sf, const R *__restrict__ Jinv,
                                                        const R *__restrict__ ops, KArgs a, int compact,
                                                        R *__restrict__ W, R *__restrict__ Part) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF, NI = (N - 1) * NF;
  __shared__ R sS[9 * NL], su[NP], sJ[NP], sT[6 * NF], sUh[6 * NF], sUF[3 * NL], sV[3 * NP];
  // the interior fluxes [d][q][r - 1] take the place of the flux-point
  // solution once the gradient is formed
  R *sG = sUF;
  static_assert(3 * NI <= 3 * NL, "interior fluxes fit the flux-point solution's place");
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x;
  const R nu = (R)a.nu;
  // the element's metric rows, state and 1/det J and its neighbours' traces:
  // every read of a lane issued before the first store (clamped indices, so
  // that no read sits behind a branch)
  constexpr int NTH = cv_threads<N>();
  constexpr int IS = (9 * NL + NTH - 1) / NTH, IP = (NP + NTH - 1) / NTH, IF = (6 * NF + NTH - 1) / NTH;
  R oth[IF];
  {
    R vs[IS], vj[IP];
    double vu[IP];
#pragma unroll
    for (int i = 0; i < IS; ++i) vs[i] = Sf[e * 9 * NL + min(tid + i * NTH, 9 * NL - 1)];
#pragma unroll
    for (int i = 0; i < IP; ++i) {
      const int t = min(tid + i * NTH, NP - 1);
      vu[i] = U[e * NP + t];
      vj[i] = Jinv[e * NP + t];
    }
#pragma unroll
    for (int i = 0; i < IF; ++i) {
      const int t = min(tid + i * NTH, 6 * NF - 1);
      const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
      oth[i] = T[nbr(a, e, d, s) * 6 * NF + (2 * d + 1 - s) * NF + q];
    }
    // keeps the compiler from moving the reads down to their uses
    __asm__ __volatile__("" ::: "memory");
#pragma unroll
    for (int i = 0; i < IS; ++i)
      if (tid + i * NTH < 9 * NL) sS[tid + i * NTH] = vs[i];
#pragma unroll
    for (int i = 0; i < IP; ++i) {
      const int t = tid + i * NTH;
      if (t < NP) {
        su[t] = cv_in<R>(vu[i], 0.0);
        sJ[t] = vj[i];
      }
    }
  }
  __syncthreads();
  // own traces and the common solution at the faces
#pragma unroll
  for (int i = 0; i < IF; ++i) {
    const int t = tid + i * NTH;
    if (t >= 6 * NF) break;
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    R v[N];
#pragma unroll
    for (int c = 0; c < N; ++c) v[c] = su[cv_point<N>(d, q, c)];
    const R own = cv_dot_end<N>(ops, v, s);
    sT[t] = own;
    sUh[t] = s == 0 ? R(0.5) * (oth[i] + own) : R(0.5) * (own + oth[i]);
  }
  __syncthreads();
  // continuous solution at the flux points of every family
  for (int t = tid; t < 3 * NL; t += blockDim.x) {
    const int d = t / NL, w = t % NL, q = w / (N + 1), r = w % (N + 1);
    R val;
    if (r == 0) {
      val = sUh[(2 * d) * NF + q];
    } else if (r == N) {
      val = sUh[(2 * d + 1) * NF + q];
    } else {
      val = R(0);
      for (int c = 0; c < N; ++c) val += ops[O.Lint + (r - 1) * N + c] * su[cv_point<N>(d, q, c)];
    }
    sUF[t] = val;
  }
  __syncthreads();
  // auxiliary variable at the solution points
  for (int t = tid; t < 3 * NP; t += blockDim.x) {
    const int m = t / NP, pt = t % NP;
    R acc = R(0);
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      R dd = R(0);
      for (int r = 0; r <= N; ++r)
        dd += ops[O.M + c * (N + 1) + r] * (sUF[d * NL + q * (N + 1) + r] * sS[((d * NF + q) * (N + 1) + r) * 3 + m]);
      acc += dd;
    }
    sV[t] = sJ[pt] * acc;
  }
  __syncthreads();
  // values at the faces, projected on the face's S row
  for (int t = tid; t < 6 * NF; t += blockDim.x) {
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    const R *srow = sS + ((d * NF + q) * (N + 1) + (s ? N : 0)) * 3;
    int rend = 0;
    R jump = R(0);
    if (compact) {
      // the family-d solution of face s keeps the own trace at the other face
      const int so = 1 - s;
      rend = so == 0 ? 0 : N;
      jump = sT[(2 * d + so) * NF + q] - sUh[(2 * d + so) * NF + q];
    }
    R w = R(0);
    for (int m = 0; m < 3; ++m) {
      const R corr = compact ? jump * sS[((d * NF + q) * (N + 1) + rend) * 3 + m] : R(0);
      R acc = R(0);
      for (int c = 0; c < N; ++c) {
        const int pt = cv_point<N>(d, q, c);
        R v = sV[m * NP + pt];
        if (compact) v += sJ[pt] * (ops[O.M + c * (N + 1) + rend] * corr);
        acc += ops[O.Lend + s * N + c] * v;
      }
      w += srow[m] * acc;
    }
    W[e * 6 * NF + t] = w;
  }
  // G_d = -nu S_d . v at the interior flux points of family d
  for (int t = tid; t < 3 * NI; t += blockDim.x) {
    const int d = t / NI, w = t % NI, q = w / (N - 1), r = 1 + w % (N - 1);
    R g = R(0);
    for (int m = 0; m < 3; ++m) {
      R v = R(0);
      for (int c = 0; c < N; ++c) v += ops[O.Lint + (r - 1) * N + c] * sV[m * NP + cv_point<N>(d, q, c)];
      g += sS[((d * NF + q) * (N + 1) + r) * 3 + m] * v;
    }
    sG[t] = -nu * g;
  }
  __syncthreads();
  // their part of the divergence
  for (int pt = tid; pt < NP; pt += blockDim.x) {
    R acc = R(0);
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      R dd = R(0);
      for (int r = 1; r < N; ++r) dd += ops[O.M + c * (N + 1) + r] * sG[d * NI + q * (N - 1) + r - 1];
      acc += dd;
    }
    Part[e * NP + pt] = acc;
  }
}

template <int N, typename R>
__global__ void __launch_bounds__(cv_threads<N>()) k_cv_face(const R *__restrict__ W, const R *__restrict__ Part,
                                                        const R *__restrict__ Jinv, const R *__restrict__ ops,
                                                        KArgs a, const R *__restrict__ T, const R *__restrict__ Pen,
                                                        double *__restrict__ dudt) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N;
  __shared__ R sGf[6 * NF];
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x;
  const R nu = (R)a.nu;
  // every read of a lane issued before the first use (clamped indices)
  constexpr int NTH = cv_threads<N>();
  constexpr int IF = (6 * NF + NTH - 1) / NTH, IP = (NP + NTH - 1) / NTH;
  R own[IF], oth[IF], to[IF], tn[IF], pen[IF], part[IP], jin[IP];
#pragma unroll
  for (int i = 0; i < IF; ++i) {
    const int t = min(tid + i * NTH, 6 * NF - 1);
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    const long long en = nbr(a, e, d, s);
    own[i] = W[e * 6 * NF + t];
    oth[i] = W[en * 6 * NF + (2 * d + 1 - s) * NF + q];
    if (Pen) {
      to[i] = T[e * 6 * NF + t];
      tn[i] = T[en * 6 * NF + (2 * d + 1 - s) * NF + q];
      pen[i] = Pen[e * 6 * NF + t];
    }
  }
#pragma unroll
  for (int i = 0; i < IP; ++i) {
    const int pt = min(tid + i * NTH, NP - 1);
    part[i] = Part[e * NP + pt];
    jin[i] = Jinv[e * NP + pt];
  }
  // keeps the compiler from moving the reads down to their uses
  __asm__ __volatile__("" ::: "memory");
#pragma unroll
  for (int i = 0; i < IF; ++i) {
    const int t = tid + i * NTH;
    if (t >= 6 * NF) break;
    const int s = (t / NF) & 1;
    R g = s == 0 ? R(0.5) * (oth[i] + own[i]) : R(0.5) * (own[i] + oth[i]);
    // interior penalty: P' (u_R - u_L), u_R on the +xi_d side
    if (Pen) g += pen[i] * (s == 0 ? to[i] - tn[i] : tn[i] - to[i]);
    sGf[t] = -nu * g;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IP; ++i) {
    const int pt = tid + i * NTH;
    if (pt >= NP) break;
    R acc = part[i];
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      acc += ops[O.M + c * (N + 1)] * sGf[(2 * d) * NF + q] + ops[O.M + c * (N + 1) + N] * sGf[(2 * d + 1) * NF + q];
    }
    dudt[e * NP + pt] = (double)(-jin[i] * acc);
  }
}

}  // namespace sd

// ---------------------------------------------------------------------------
// Navier-Stokes on curvilinear hexahedra (section 2.3, eqs. ns:mapped and
// adj:f; fluxes of section 4.4), FP64 or FP32 as above, the constant
// reference state removed before the rounding to the compute type (as on
// Cartesian meshes).  The same three steps for the five conservative
// variables (traces T[e][f][v][q]):
//   k_cvn_grad  the gradient of every variable at the solution points (kept
//               in LDS), its one-sided (compact) or standard face values,
//               the fluxes G_d = S_d . (F_c - F_v) at the interior flux
//               points of family d and their part of the divergence; and at
//               each face point the element's half of the common flux,
//                 X = |S_d| Roe(U_L, U_R; S_d / |S_d|) / 2 - S_d . F_v(u_hat, v_own) / 2,
//               since F_v is linear in the gradient at a fixed state: the
//               common flux of option (a), |S_d| Roe - S_d . F_v(u_hat,
//               (v_L + v_R) / 2), is X_L + X_R (both sides evaluate the same
//               Roe flux from the same traces and the same S_d);
//   k_cvn_face  G at the faces = X_L + X_R and du/dt = -J^-1 (the interior
//               part + the face columns of M times the face fluxes).
// One element per block, LDS sized per n (dynamic).
// ---------------------------------------------------------------------------
namespace sd {

// Fluxes along a direction vector s (curvilinear elements: the flux through
// the rows of the adjugate S): F . s = sum_m s_m F e_m, with F_c(U0) . s
// removed as above.
template <typename R>
__device__ __forceinline__ void ns_conv_dir(const NsConst<R> &c, const R *U, const Prim<R> &st, const R *sv, R *F) {
  const R us = st.u[0] * sv[0] + st.u[1] * sv[1] + st.u[2] * sv[2];
  F[0] = U[1] * sv[0] + U[2] * sv[1] + U[3] * sv[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) F[1 + i] = U[1 + i] * us + st.dp * sv[i];
  F[4] = (st.rhoE + st.p) * us;
}

// F_v . s from the state and the conservative gradient G[m*5 + v]
template <typename R>
__device__ __forceinline__ void ns_visc_dir(const NsConst<R> &c, const Prim<R> &st, const R *G, const R *sv, R *F) {
  R E = st.rhoE * st.inv;
  R du[3][3], dT[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    R drho = G[m * 5 + 0];
#pragma unroll
    for (int i = 0; i < 3; ++i) du[i][m] = (G[m * 5 + 1 + i] - st.u[i] * drho) * st.inv;
    R dE = (G[m * 5 + 4] - E * drho) * st.inv;
    dT[m] = c.gm1 * (dE - (st.u[0] * du[0][m] + st.u[1] * du[1][m] + st.u[2] * du[2][m]));
  }
  R T = st.p * st.inv;
  R mu = c.mu0;
  if (c.suth) {
    R th = T * c.T0inv;
    mu = c.mu0 * th * fsqrt(th) * c.onepS * frcp(th + c.S);
  }
  const R lam = c.lam_over_mu * mu, kappa = c.cp_over_pr * mu;
  const R div = du[0][0] + du[1][1] + du[2][2];
  R ts[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    R acc = lam * div * sv[i];
#pragma unroll
    for (int m = 0; m < 3; ++m) acc += mu * (du[i][m] + du[m][i]) * sv[m];
    ts[i] = acc;
  }
  F[0] = R(0);
  F[1] = ts[0];
  F[2] = ts[1];
  F[3] = ts[2];
  F[4] = st.u[0] * ts[0] + st.u[1] * ts[1] + st.u[2] * ts[2] + kappa * (dT[0] * sv[0] + dT[1] * sv[1] + dT[2] * sv[2]);
}

// Roe flux along the unit normal n with Harten's fix on the acoustic waves
// (the axis version above with u_d -> u . n and the tangential velocity jump
// du - (du . n) n), minus F_c(U0) . n.
template <typename R>
__device__ __forceinline__ void ns_roe_dir(const NsConst<R> &c, const R *UL, const R *UR, const R *n, R *F) {
  Prim<R> L = ns_prim(c, UL), Rr = ns_prim(c, UR);
  R FL[5], FR[5];
  ns_conv_dir(c, UL, L, n, FL);
  ns_conv_dir(c, UR, Rr, n, FR);
  R sL = fsqrt(L.rho), sR = fsqrt(Rr.rho);
  R wsum = frcp(sL + sR);
  R HL = (L.rhoE + L.p) * L.inv, HR = (Rr.rhoE + Rr.p) * Rr.inv;
  R ut[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) ut[i] = (sL * L.u[i] + sR * Rr.u[i]) * wsum;
  R Ht = (sL * HL + sR * HR) * wsum;
  R rt = sL * sR;
  R q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
  R c2 = c.gm1 * (Ht - R(0.5) * q2);
  R cs = fsqrt(c2);
  R un = ut[0] * n[0] + ut[1] * n[1] + ut[2] * n[2];
  R du[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) du[i] = Rr.u[i] - L.u[i];
  R drho = Rr.rho - L.rho, dpj = Rr.dp - L.dp, dun = du[0] * n[0] + du[1] * n[1] + du[2] * n[2];
  R ic2 = frcp(c2);
  R inv2c2 = R(0.5) * ic2;
  R a1 = (dpj - rt * cs * dun) * inv2c2;
  R a5 = (dpj + rt * cs * dun) * inv2c2;
  R a2 = drho - dpj * ic2;
  R l1 = fabs(un - cs), l2 = fabs(un), l5 = fabs(un + cs);
  R delta = c.efix * (l2 + cs);
  if (delta > R(0)) {
    R i2d = R(0.5) * frcp(delta);
    if (l1 < delta) l1 = (l1 * l1 + delta * delta) * i2d;
    if (l5 < delta) l5 = (l5 * l5 + delta * delta) * i2d;
  }
  R dut[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) dut[i] = du[i] - dun * n[i];
  R w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2, ws = l2 * rt;
  R D[5];
  D[0] = w1 + w2 + w5;
#pragma unroll
  for (int i = 0; i < 3; ++i) D[1 + i] = (w1 + w5 + w2) * ut[i] + ws * dut[i] + (w5 - w1) * cs * n[i];
  D[4] = w1 * (Ht - cs * un) + w5 * (Ht + cs * un) + w2 * R(0.5) * q2 +
         ws * (ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2]);
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = R(0.5) * (FL[k] + FR[k]) - R(0.5) * D[k];
}

constexpr int kCvnThreads = 256;

// LDS of k_cvn_grad in elements of the compute type
template <int N>
struct CvnGradSmem {
  static constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF, NI = (N - 1) * NF;
  static constexpr int S = 0, U = S + 9 * NL, J = U + 5 * NP, T = J + NP, TN = T + 30 * NF, UF = TN + 30 * NF,
                       V = UF + 15 * NL, G = V + 15 * NP, VF = G + 15 * NI;
  static constexpr int TOTAL = VF + 90 * NF;
};

template <int N, typename R>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_traces(const double *__restrict__ U, R *__restrict__ T,
                                                            const R *__restrict__ ops, KArgs a) {
  constexpr int NP = N * N * N, NF = N * N;
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  // every read of a lane issued before the first trace (clamped indices)
  constexpr int IT = (30 * NF + kCvnThreads - 1) / kCvnThreads;
  const int tid = threadIdx.x;
  double y[IT][N];
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = min(tid + i * kCvnThreads, 30 * NF - 1);
    const int f = t / (5 * NF), w = t % (5 * NF), v = w / NF, q = w % NF, d = f >> 1;
    const double *u = U + (e * 5 + v) * NP;
#pragma unroll
    for (int c = 0; c < N; ++c) y[i][c] = u[cv_point<N>(d, q, c)];
  }
  // keeps the compiler from moving the reads down to their uses
  __asm__ __volatile__("" ::: "memory");
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int t = tid + i * kCvnThreads;
    if (t >= 30 * NF) break;
    const int f = t / (5 * NF), v = (t % (5 * NF)) / NF;
    R x[N];
#pragma unroll
    for (int c = 0; c < N; ++c) x[c] = cv_in<R>(y[i][c], a.U0[v]);
    T[e * 30 * NF + t] = cv_dot_end<N>(ops, x, f & 1);
  }
}

// common solution at point q of face f for variable v, from the own and the
// neighbour's trace (the same expression on both sides of the face)
template <typename R>
__device__ __forceinline__ R cvn_hat(const R *sT, const R *sTn, int f, int idx) {
  const R own = sT[idx], oth = sTn[idx];
  return (f & 1) == 0 ? R(0.5) * (oth + own) : R(0.5) * (own + oth);
}

// G_d = S_d . (F_c - F_v) at interior flux point w of family d (item t)
template <int N, typename R>
__device__ __forceinline__ void cvn_interior_item(const NsConst<R> &c, const R *__restrict__ ops, const R *sS,
                                                  const R *sUF, const R *sV, R *sG, int t) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N, NL = (N + 1) * NF, NI = (N - 1) * NF;
  const int d = t / NI, w = t % NI, q = w / (N - 1), r = 1 + w % (N - 1);
  const R *srow = sS + ((d * NF + q) * (N + 1) + r) * 3;
  const R sv[3] = {srow[0], srow[1], srow[2]};
  R Uf[5], Vf[15];
  for (int v = 0; v < 5; ++v) Uf[v] = sUF[(d * 5 + v) * NL + q * (N + 1) + r];
  for (int mv = 0; mv < 15; ++mv) {
    R acc = R(0);
    for (int cc = 0; cc < N; ++cc) acc += ops[O.Lint + (r - 1) * N + cc] * sV[mv * NP + cv_point<N>(d, q, cc)];
    Vf[mv] = acc;
  }
  Prim<R> st = ns_prim(c, Uf);
  R Fc[5], Fv[5];
  ns_conv_dir(c, Uf, st, sv, Fc);
  ns_visc_dir(c, st, Vf, sv, Fv);
  for (int v = 0; v < 5; ++v) sG[(d * 5 + v) * NI + w] = Fc[v] - Fv[v];
}

template <int N, typename R>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_grad(const double *__restrict__ U, const R *__restrict__ T,
                                                          const R *__restrict__ Sf, const R *__restrict__ Jinv,
                                                          const R *__restrict__ ops, KArgs a, int compact,
                                                          R *__restrict__ X, R *__restrict__ Part) {
  using SM = CvnGradSmem<N>;
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = SM::NP, NF = SM::NF, NL = SM::NL, NI = SM::NI;
  extern __shared__ double smem_cvn[];
  R *base = reinterpret_cast<R *>(smem_cvn);
  R *sS = base + SM::S, *su = base + SM::U, *sJ = base + SM::J, *sT = base + SM::T, *sTn = base + SM::TN,
    *sUF = base + SM::UF, *sV = base + SM::V, *sG = base + SM::G, *sVf = base + SM::VF;
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x, nth = blockDim.x;
  // the element's metric rows, state and 1/det J and its neighbours' traces:
  // every read of a lane issued before the first store (clamped indices, so
  // that no read sits behind a branch; kCvnThreads lanes)
  {
    constexpr int IS = (9 * NL + kCvnThreads - 1) / kCvnThreads, IU = (5 * NP + kCvnThreads - 1) / kCvnThreads,
                  IJ = (NP + kCvnThreads - 1) / kCvnThreads, IT = (30 * NF + kCvnThreads - 1) / kCvnThreads;
    R vs[IS], vj[IJ], vt[IT];
    double vu[IU];
#pragma unroll
    for (int i = 0; i < IS; ++i) vs[i] = Sf[e * 9 * NL + min(tid + i * kCvnThreads, 9 * NL - 1)];
#pragma unroll
    for (int i = 0; i < IU; ++i) vu[i] = U[e * 5 * NP + min(tid + i * kCvnThreads, 5 * NP - 1)];
#pragma unroll
    for (int i = 0; i < IJ; ++i) vj[i] = Jinv[e * NP + min(tid + i * kCvnThreads, NP - 1)];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int t = min(tid + i * kCvnThreads, 30 * NF - 1);
      const int f = t / (5 * NF), w = t % (5 * NF), d = f >> 1, s = f & 1;
      vt[i] = T[nbr(a, e, d, s) * 30 * NF + (2 * d + 1 - s) * 5 * NF + w];
    }
    // keeps the compiler from moving the reads down to their uses
    __asm__ __volatile__("" ::: "memory");
#pragma unroll
    for (int i = 0; i < IS; ++i)
      if (tid + i * kCvnThreads < 9 * NL) sS[tid + i * kCvnThreads] = vs[i];
#pragma unroll
    for (int i = 0; i < IU; ++i) {
      const int t = tid + i * kCvnThreads;
      if (t < 5 * NP) su[t] = cv_in<R>(vu[i], a.U0[t / NP]);
    }
#pragma unroll
    for (int i = 0; i < IJ; ++i)
      if (tid + i * kCvnThreads < NP) sJ[tid + i * kCvnThreads] = vj[i];
#pragma unroll
    for (int i = 0; i < IT; ++i)
      if (tid + i * kCvnThreads < 30 * NF) sTn[tid + i * kCvnThreads] = vt[i];
  }
  __syncthreads();
  // own traces (from the state)
  for (int t = tid; t < 30 * NF; t += nth) {
    const int f = t / (5 * NF), w = t % (5 * NF), v = w / NF, q = w % NF, d = f >> 1, s = f & 1;
    R x[N];
#pragma unroll
    for (int cc = 0; cc < N; ++cc) x[cc] = su[v * NP + cv_point<N>(d, q, cc)];
    sT[t] = cv_dot_end<N>(ops, x, s);
  }
  __syncthreads();
  // continuous solution of every variable at the flux points of every family
  for (int t = tid; t < 15 * NL; t += nth) {
    const int d = t / (5 * NL), w = t % (5 * NL), v = w / NL, l = w % NL, q = l / (N + 1), r = l % (N + 1);
    R val;
    if (r == 0 || r == N) {
      const int f = 2 * d + (r == N ? 1 : 0);
      val = cvn_hat(sT, sTn, f, (f * 5 + v) * NF + q);
    } else {
      val = R(0);
      for (int c = 0; c < N; ++c) val += ops[O.Lint + (r - 1) * N + c] * su[v * NP + cv_point<N>(d, q, c)];
    }
    sUF[t] = val;
  }
  __syncthreads();
  // gradient of every variable at the solution points
  for (int t = tid; t < 15 * NP; t += nth) {
    const int mv = t / NP, pt = t % NP, m = mv / 5, v = mv % 5;
    R acc = R(0);
    for (int d = 0; d < 3; ++d) {
      int q, c;
      cv_line_of<N>(pt, d, q, c);
      R dd = R(0);
      for (int r = 0; r <= N; ++r)
        dd += ops[O.M + c * (N + 1) + r] *
              (sUF[(d * 5 + v) * NL + q * (N + 1) + r] * sS[((d * NF + q) * (N + 1) + r) * 3 + m]);
      acc += dd;
    }
    sV[t] = sJ[pt] * acc;
  }
  __syncthreads();
  // one-sided (compact: the family-d solution of face s keeps the own trace
  // at the other face) or standard face values of every gradient component,
  // sVf[f][mv][q], one item per value
  for (int t = tid; t < 90 * NF; t += nth) {
    const int f = t / (15 * NF), w = t % (15 * NF), mv = w / NF, q = w % NF, d = f >> 1, s = f & 1;
    const int m = mv / 5, v = mv % 5, so = 1 - s, rend = so == 0 ? 0 : N;
    R corr = R(0);
    if (compact) {
      const int idx = ((2 * d + so) * 5 + v) * NF + q;
      corr = (sT[idx] - cvn_hat(sT, sTn, 2 * d + so, idx)) * sS[((d * NF + q) * (N + 1) + rend) * 3 + m];
    }
    R acc = R(0);
    for (int cc = 0; cc < N; ++cc) {
      const int pt = cv_point<N>(d, q, cc);
      R g = sV[mv * NP + pt];
      if (compact) g += sJ[pt] * (ops[O.M + cc * (N + 1) + rend] * corr);
      acc += ops[O.Lend + s * N + cc] * g;
    }
    sVf[t] = acc;
  }
  __syncthreads();
  const NsConst<R> c(a);
  // one list of work items: the element's half of the common flux at every
  // face point, then G_d at the interior flux points of family d
  for (int t = tid; t < 6 * NF + 3 * NI; t += nth) {
    if (t >= 6 * NF) {
      cvn_interior_item<N>(c, ops, sS, sUF, sV, sG, t - 6 * NF);
      continue;
    }
    const int f = t / NF, q = t % NF, d = f >> 1, s = f & 1;
    const R *srow = sS + ((d * NF + q) * (N + 1) + (s ? N : 0)) * 3;
    const R sv[3] = {srow[0], srow[1], srow[2]};
    R Vf[15];
    for (int mv = 0; mv < 15; ++mv) Vf[mv] = sVf[(f * 15 + mv) * NF + q];
    R UL[5], UR[5], Uh[5];
    for (int v = 0; v < 5; ++v) {
      const int idx = (f * 5 + v) * NF + q;
      UL[v] = s == 0 ? sTn[idx] : sT[idx];
      UR[v] = s == 0 ? sT[idx] : sTn[idx];
      Uh[v] = cvn_hat(sT, sTn, f, idx);
    }
    const R nrm = fsqrt(sv[0] * sv[0] + sv[1] * sv[1] + sv[2] * sv[2]);
    const R nv[3] = {sv[0] / nrm, sv[1] / nrm, sv[2] / nrm};
    R Fr[5], Fv[5];
    ns_roe_dir(c, UL, UR, nv, Fr);
    Prim<R> st = ns_prim(c, Uh);
    ns_visc_dir(c, st, Vf, sv, Fv);
    for (int v = 0; v < 5; ++v) X[(e * 6 + f) * 5 * NF + v * NF + q] = R(0.5) * (nrm * Fr[v]) - R(0.5) * Fv[v];
  }
  __syncthreads();
  // their part of the divergence
  for (int t = tid; t < 5 * NP; t += nth) {
    const int v = t / NP, pt = t % NP;
    R acc = R(0);
    for (int d = 0; d < 3; ++d) {
      int q, cc;
      cv_line_of<N>(pt, d, q, cc);
      R dd = R(0);
      for (int r = 1; r < N; ++r) dd += ops[O.M + cc * (N + 1) + r] * sG[(d * 5 + v) * NI + q * (N - 1) + r - 1];
      acc += dd;
    }
    Part[e * 5 * NP + t] = acc;
  }
}

// With the reference state removed, the momentum fluxes carry P - p0 and
// P0div holds -J^-1 sum_d D_d (p0 S_dm) per element (three n^3 blocks, the
// divergence of the removed constant flux F_c(U0) . S_d, zero wherever the
// metric identities hold discretely); adding it back keeps the equations of
// the full-pressure discretisation on every mesh.
template <int N, typename R>
__global__ void __launch_bounds__(kCvnThreads) k_cvn_face(const R *__restrict__ X, const R *__restrict__ Part,
                                                          const R *__restrict__ Jinv, const R *__restrict__ ops,
                                                          KArgs a, const R *__restrict__ P0div,
                                                          double *__restrict__ dudt) {
  constexpr OpsLayout O = ops_layout(N);
  constexpr int NP = N * N * N, NF = N * N;
  __shared__ R sGf[30 * NF];
  const long long e = blockIdx.x;
  if (e >= a.ne) return;
  const int tid = threadIdx.x;
  // every read of a lane issued before the first use (clamped indices)
  constexpr int IF = (30 * NF + kCvnThreads - 1) / kCvnThreads, IP = (5 * NP + kCvnThreads - 1) / kCvnThreads;
  R own[IF], oth[IF], part[IP], jin[IP], p0[IP];
#pragma unroll
  for (int i = 0; i < IF; ++i) {
    const int t = min(tid + i * kCvnThreads, 30 * NF - 1);
    const int f = t / (5 * NF), w = t % (5 * NF), d = f >> 1, s = f & 1;
    own[i] = X[e * 30 * NF + t];
    oth[i] = X[nbr(a, e, d, s) * 30 * NF + (2 * d + 1 - s) * 5 * NF + w];
  }
#pragma unroll
  for (int i = 0; i < IP; ++i) {
    const int t = min(tid + i * kCvnThreads, 5 * NP - 1), v = t / NP, pt = t % NP;
    part[i] = Part[e * 5 * NP + t];
    jin[i] = Jinv[e * NP + pt];
    if (P0div) p0[i] = P0div[(e * 3 + min(max(v - 1, 0), 2)) * NP + pt];
  }
  // keeps the compiler from moving the reads down to their uses
  __asm__ __volatile__("" ::: "memory");
#pragma unroll
  for (int i = 0; i < IF; ++i) {
    const int t = tid + i * kCvnThreads;
    if (t >= 30 * NF) break;
    const int s = (t / (5 * NF)) & 1;
    sGf[t] = s == 0 ? oth[i] + own[i] : own[i] + oth[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < IP; ++i) {
    const int t = tid + i * kCvnThreads;
    if (t >= 5 * NP) break;
    const int v = t / NP, pt = t % NP;
    R acc = part[i];
    for (int d = 0; d < 3; ++d) {
      int q, cc;
      cv_line_of<N>(pt, d, q, cc);
      acc += ops[O.M + cc * (N + 1)] * sGf[((2 * d) * 5 + v) * NF + q] +
             ops[O.M + cc * (N + 1) + N] * sGf[((2 * d + 1) * 5 + v) * NF + q];
    }
    double r = (double)(-jin[i] * acc);
    if (P0div && v >= 1 && v <= 3) r += (double)p0[i];
    dudt[e * 5 * NP + t] = r;
  }
}

}  // namespace sd
