// Fused Navier-Stokes right-hand side kernel for gfx950 (3-D, any n <= 7).
//
// Same algebra as the generic k_rhs (see sd_kernels.hip), organised for the
// five-variable system:
//   P0  per element: neighbour indices once (6 face + 12 edge neighbours,
//       32-bit arithmetic); the state (reference removed) and the
//       neighbours' face traces T, normal-gradient traces NN and edge traces
//       staged in LDS with coalesced loads;
//   P1  own face traces (and, compact, own normal-gradient traces) from the
//       LDS state: no re-read of the trace buffer;
//   P2  auxiliary gradient at the solution points (15 components);
//   P3  one work item per face point: the common gradient (own side from the
//       gradient, neighbour side rebuilt from its traces and the edge traces)
//       and the interface flux (Roe minus viscous), kept in LDS;
//   P4  one work item per line of a flux-point family: the line's state and
//       gradient in registers, the n-1 interior fluxes, the two interface
//       fluxes, and the divergence along the line (-2/h_d M F);
//   P5  the three directional contributions summed and stored in FP64.
#pragma once

#include "sd_internal.h"
#include "sd_physics.h"

namespace sd {

constexpr int kNsMaxEpb = 8;

template <int N, typename R>
struct NsOps {
  R Lend[2][N];
  R Lint[N - 1][N];
  R D[N][N];
  R M[N][N + 1];
  R Mc[2][N];
  R rrow[2][N];
  R kap[2];
};

template <int N>
struct NsSmem {
  static constexpr int NP = N * N * N, NF = N * N;
  static constexpr int U = 0;                  // [5][NP]
  static constexpr int G = U + 5 * NP;         // [3][5][NP]
  static constexpr int TO = G + 15 * NP;       // [6][5][NF] own traces
  static constexpr int TN = TO + 30 * NF;      // [6][5][NF] neighbour traces
  static constexpr int NO = TN + 30 * NF;      // [6][5][NF] own normal-gradient traces
  static constexpr int NN = NO + 30 * NF;      // [6][5][NF] neighbour normal-gradient traces
  static constexpr int E = NN + 30 * NF;       // [12][5][N] edge-neighbour edge traces
  static constexpr int FH = E + 60 * N;        // [6][5][NF] interface fluxes
  static constexpr int RS = TO;                // [3][5][NP] aliases TO..E after P3
  static constexpr int TOTAL = FH + 30 * NF;
  static_assert(RS + 15 * NP <= FH, "partial residuals overlap the interface fluxes");
};

template <int N, typename R, bool COMPACT>
__global__ void __launch_bounds__(256) k_rhs_ns(const double *__restrict__ U, const R *__restrict__ X,
                                                double *__restrict__ dudt, KArgs a, NsOps<N, R> op) {
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF;
  constexpr int XS = trace_stride(3, N, 5), FS = trace_face_stride(3, N, 5), EO = trace_edge_off(3, N, 5);
  extern __shared__ char smem_raw[];
  R *sm = reinterpret_cast<R *>(smem_raw);
  __shared__ int snb[kNsMaxEpb][18];
  const int tid = threadIdx.x, nth = blockDim.x;
  const int epb = a.epb;
  const int e0 = blockIdx.x * epb;
  const int nb = min(epb, (int)(a.ne - e0));

  // P0: neighbour table, state, neighbour traces
  for (int t = tid; t < nb * 18; t += nth) {
    int el = t / 18, k = t % 18;
    int e = e0 + el;
    int nx = a.nel[0], ny = a.nel[1], nz = a.nel[2];
    int c[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
    const int ext[3] = {nx, ny, nz};
    auto step = [&](int d, int s) { c[d] = s ? (c[d] + 1 == ext[d] ? 0 : c[d] + 1) : (c[d] == 0 ? ext[d] - 1 : c[d] - 1); };
    if (k < 6) {
      step(k >> 1, k & 1);
    } else {
      int ed = k - 6, P = ed >> 2;
      int lo = P == 2 ? 1 : 0, hi = P == 0 ? 1 : 2;
      step(lo, (ed >> 1) & 1);
      step(hi, ed & 1);
    }
    snb[el][k] = c[0] + nx * (c[1] + ny * c[2]);
  }
  for (int t = tid; t < nb * 5 * NP; t += nth) {
    int el = t / (5 * NP), r = t % (5 * NP);
    sm[el * SM::TOTAL + SM::U + r] = (R)(U[(long long)e0 * 5 * NP + t] - a.U0[r / NP]);
  }
  __syncthreads();
  for (int t = tid; t < nb * 60 * NF; t += nth) {
    int el = t / (60 * NF), r = t % (60 * NF);
    int f = r / (10 * NF), w = r % (10 * NF);
    int d = f >> 1, s = f & 1;
    R val = X[(long long)snb[el][f] * XS + (2 * d + 1 - s) * FS + w];
    if (w < 5 * NF) sm[el * SM::TOTAL + SM::TN + f * 5 * NF + w] = val;
    else sm[el * SM::TOTAL + SM::NN + f * 5 * NF + (w - 5 * NF)] = val;
  }
  for (int t = tid; t < nb * 60 * N; t += nth) {
    int el = t / (60 * N), r = t % (60 * N);
    int ed = r / (5 * N), w = r % (5 * N);
    int opp = (ed & ~3) + 2 * (1 - ((ed >> 1) & 1)) + (1 - (ed & 1));
    sm[el * SM::TOTAL + SM::E + ed * 5 * N + w] = X[(long long)snb[el][6 + ed] * XS + EO + opp * 5 * N + w];
  }
  // P1: own traces from the staged state
  for (int t = tid; t < nb * 6 * NF; t += nth) {
    int el = t / (6 * NF), r = t % (6 * NF);
    int f = r / NF, q = r % NF, d = f >> 1, s = f & 1, base, stride;
    line_of<3, N>(d, q, base, stride);
    R *E = sm + el * SM::TOTAL;
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R *u = E + SM::U + v * NP + base;
      R tr = R(0), nn = R(0);
#pragma unroll
      for (int c = 0; c < N; ++c) {
        R uv = u[c * stride];
        tr += op.Lend[s][c] * uv;
        if constexpr (COMPACT) nn += op.rrow[s][c] * uv;
      }
      E[SM::TO + (f * 5 + v) * NF + q] = tr;
      if constexpr (COMPACT) E[SM::NO + (f * 5 + v) * NF + q] = nn;
    }
  }
  __syncthreads();
  // P2: gradient at the solution points
  for (int t = tid; t < nb * NP; t += nth) {
    int el = t / NP, pt = t % NP;
    R *E = sm + el * SM::TOTAL;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int am, qm, base, stride;
      coord_of<3, N>(pt, m, am, qm);
      line_of<3, N>(m, qm, base, stride);
      R th = (R)a.two_over_h[m];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const R *u = E + SM::U + v * NP + base;
        R acc = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) acc += op.D[am][c] * u[c * stride];
        int i0 = ((2 * m) * 5 + v) * NF + qm, i1 = ((2 * m + 1) * 5 + v) * NF + qm;
        R to0 = E[SM::TO + i0], tn0 = E[SM::TN + i0], to1 = E[SM::TO + i1], tn1 = E[SM::TN + i1];
        R uh0 = R(0.5) * (tn0 + to0), uh1 = R(0.5) * (to1 + tn1);
        acc += op.Mc[0][am] * (uh0 - to0);
        acc += op.Mc[1][am] * (uh1 - to1);
        E[SM::G + (m * 5 + v) * NP + pt] = th * acc;
      }
    }
  }
  __syncthreads();
  // P3: interface fluxes, one work item per face point
  for (int t = tid; t < nb * 6 * NF; t += nth) {
    int el = t / (6 * NF), r = t % (6 * NF);
    int f = r / NF, q = r % NF, d = f >> 1, s = f & 1, so = 1 - s;
    const R *E = sm + el * SM::TOTAL;
    R UL[5], UR[5], Uh[5], Vh[15];
    const R thd = (R)a.two_over_h[d];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      int fv = (f * 5 + v) * NF + q;
      R own = E[SM::TO + fv], oth = E[SM::TN + fv];
      UL[v] = s == 0 ? oth : own;
      UR[v] = s == 0 ? own : oth;
      Uh[v] = s == 0 ? R(0.5) * (oth + own) : R(0.5) * (own + oth);
    }
    int base, stride;
    line_of<3, N>(d, q, base, stride);
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      if (m == d) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          int fv = (f * 5 + v) * NF + q;
          R vown;
          if constexpr (COMPACT) {
            vown = thd * (E[SM::NO + fv] + op.kap[s] * Uh[v]);
          } else {
            const R *g = E + SM::G + (m * 5 + v) * NP + base;
            R acc = R(0);
#pragma unroll
            for (int c = 0; c < N; ++c) acc += op.Lend[s][c] * g[c * stride];
            vown = acc;
          }
          R voth = thd * (E[SM::NN + fv] + op.kap[so] * Uh[v]);
          Vh[m * 5 + v] = s == 0 ? R(0.5) * (voth + vown) : R(0.5) * (vown + voth);
        }
      } else {
        int t3 = 3 - d - m;
        int a_lo = q % N, a_hi = q / N;
        int am = (m < t3) ? a_lo : a_hi, at = (m < t3) ? a_hi : a_lo;
        int qs = (m < t3) ? at * N : at, qstep = (m < t3) ? 1 : N;
        R thm = (R)a.two_over_h[m];
        int e0i = edge_id(d, s, m, 0), e1i = edge_id(d, s, m, 1);
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          const R *g = E + SM::G + (m * 5 + v) * NP + base;
          R vown = R(0);
#pragma unroll
          for (int c = 0; c < N; ++c) vown += op.Lend[s][c] * g[c * stride];
          const R *tn = E + SM::TN + (f * 5 + v) * NF + qs;
          R dT = R(0), eL = R(0), eR = R(0);
#pragma unroll
          for (int c = 0; c < N; ++c) {
            R tv = tn[c * qstep];
            dT += op.D[am][c] * tv;
            eL += op.Lend[0][c] * tv;
            eR += op.Lend[1][c] * tv;
          }
          R eLn = E[SM::E + (e0i * 5 + v) * N + at];
          R eRn = E[SM::E + (e1i * 5 + v) * N + at];
          R ehL = R(0.5) * (eLn + eL), ehR = R(0.5) * (eR + eRn);
          R voth = thm * (dT + op.Mc[0][am] * (ehL - eL) + op.Mc[1][am] * (ehR - eR));
          Vh[m * 5 + v] = s == 0 ? R(0.5) * (voth + vown) : R(0.5) * (vown + voth);
        }
      }
    }
    R F[5];
    face_flux<PHYS_NS, 5, R>(a, d, UL, UR, Uh, Vh, F);
    R *Ew = sm + el * SM::TOTAL;
#pragma unroll
    for (int v = 0; v < 5; ++v) Ew[SM::FH + (f * 5 + v) * NF + q] = F[v];
  }
  __syncthreads();
  // P4: one work item per line of each flux-point family
  for (int t = tid; t < nb * 3 * NF; t += nth) {
    int el = t / (3 * NF), r = t % (3 * NF);
    int d = r / NF, q = r % NF, base, stride;
    line_of<3, N>(d, q, base, stride);
    R *E = sm + el * SM::TOTAL;
    R ul[5][N], gl[15][N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
#pragma unroll
      for (int v = 0; v < 5; ++v) ul[v][c] = E[SM::U + v * NP + base + c * stride];
#pragma unroll
      for (int w = 0; w < 15; ++w) gl[w][c] = E[SM::G + w * NP + base + c * stride];
    }
    R Fl[N + 1][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Fl[0][v] = E[SM::FH + ((2 * d) * 5 + v) * NF + q];
      Fl[N][v] = E[SM::FH + ((2 * d + 1) * 5 + v) * NF + q];
    }
#pragma unroll
    for (int rr = 1; rr < N; ++rr) {
      R Uf[5], Gf[15];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        R acc = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) acc += op.Lint[rr - 1][c] * ul[v][c];
        Uf[v] = acc;
      }
#pragma unroll
      for (int w = 0; w < 15; ++w) {
        R acc = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) acc += op.Lint[rr - 1][c] * gl[w][c];
        Gf[w] = acc;
      }
      interior_flux<PHYS_NS, 5, R>(a, d, Uf, Gf, Fl[rr]);
    }
    const R thd = (R)a.two_over_h[d];
#pragma unroll
    for (int ai = 0; ai < N; ++ai)
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        R acc = R(0);
#pragma unroll
        for (int c = 0; c <= N; ++c) acc += op.M[ai][c] * Fl[c][v];
        E[SM::RS + (d * 5 + v) * NP + base + ai * stride] = -thd * acc;
      }
  }
  __syncthreads();
  // P5: sum of the three directional contributions
  for (int t = tid; t < nb * 5 * NP; t += nth) {
    int el = t / (5 * NP), r = t % (5 * NP);
    const R *E = sm + el * SM::TOTAL + SM::RS;
    dudt[(long long)e0 * 5 * NP + t] = (double)E[r] + (double)E[5 * NP + r] + (double)E[10 * NP + r];
  }
}

template <int N, typename R>
NsOps<N, R> make_ns_ops(const double *t) {
  const OpsLayout O = ops_layout(N);
  NsOps<N, R> op{};
  for (int s = 0; s < 2; ++s)
    for (int c = 0; c < N; ++c) {
      op.Lend[s][c] = (R)t[O.Lend + s * N + c];
      op.Mc[s][c] = (R)t[O.Mc + s * N + c];
      op.rrow[s][c] = (R)t[O.rrow + s * N + c];
    }
  for (int r = 0; r < N - 1; ++r)
    for (int c = 0; c < N; ++c) op.Lint[r][c] = (R)t[O.Lint + r * N + c];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) op.D[i][j] = (R)t[O.D + i * N + j];
  for (int i = 0; i < N; ++i)
    for (int j = 0; j <= N; ++j) op.M[i][j] = (R)t[O.M + i * (N + 1) + j];
  op.kap[0] = (R)t[O.kap];
  op.kap[1] = (R)t[O.kap + 1];
  return op;
}

}  // namespace sd
