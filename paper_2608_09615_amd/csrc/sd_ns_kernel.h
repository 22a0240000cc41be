// Fused Navier-Stokes right-hand side kernel for gfx950 (3-D, any n <= 7).
//
// Same algebra as the generic k_rhs (see sd_kernels.hip), organised for the
// five-variable system:
//   P0  per element: neighbour indices once (6 face + 12 edge neighbours,
//       32-bit arithmetic); the state (reference removed), the neighbours'
//       face traces T and normal-gradient traces NN, and the edge traces
//       staged in LDS with vector loads;
//   P2  auxiliary gradient at the solution points (15 components); the own
//       face traces it needs come from the same state values;
//   P3  one work item per face point, two passes: own trace (and, compact,
//       normal-gradient trace) from the state, the common gradient (own side
//       from the gradient, neighbour side rebuilt from its traces and the
//       edge traces) and minus the viscous flux; then the Roe flux of the two
//       traces added; kept in LDS;
//   P4  one work item per interior flux point of a family: the 20 state and
//       gradient values interpolated along its line and the interior flux,
//       kept in LDS over the dead neighbour traces;
//   P5  one work item per line and variable: the divergence along the line
//       (-2/h_d M F over the n+1 fluxes), kept in LDS over the dead gradient;
//       then per value the three directional contributions summed in FP64
//       (and the RK stage applied).
// Work items of P2-P4 are ordered direction-major (face-major for P3) so
// that, with epb * n^2 = 64 (p = 3, four elements per block), every
// wavefront works on a single direction (and, in P4, a single flux point of
// the line): the bodies are compiled per direction and the branches are
// uniform.  Small work items keep the register footprint low, so that more
// wavefronts share a compute unit.
#pragma once

#include <cstring>
#include <type_traits>

#include "sd_internal.h"
#include "sd_physics.h"

namespace sd {

constexpr int kNsMaxEpb = 8;

// Largest block of k_rhs_ns (four wavefronts).
template <int N, typename R>
__host__ __device__ constexpr int ns_max_threads() {
  return 256;
}


template <int N, typename R>
struct NsOps {
  R Lend[2][N];
  R Lint[N - 1][N];
  R D[N][N];
  R M[N][N + 1];
  R Mc[2][N];
  R rrow[2][N];
  R kap[2];
  R kapx[2];    // (L M)[end_s][end_other]: BR1's opposite-face term
  // auxiliary gradient along a line regrouped by linearity:
  // D u + Mc0 (uh0 - Lend0 u) + Mc1 (uh1 - Lend1 u) with uh = (t + Lend u)/2
  // = A u + hMc0 t0 + hMc1 t1, A = D - (Mc0 Lend0^T + Mc1 Lend1^T)/2
  R A[N][N];
  R hMc[2][N];
};

__host__ __device__ constexpr int pad4(int x) { return (x + 3) / 4 * 4; }

// BF16x3 split precision (precision SD_BF16X3): the gradient and divergence
// line contractions run on the 16-block 4x4x4 BF16 matrix-core instruction.
// Each lane owns one column (a line of one variable): its K inputs go in the
// B operand, lane l % 4 of every block supplies row l % 4 of the operator in
// the A operand, and the lane receives its column's four outputs.  Operator
// and data are split into hi + lo BF16 parts; hi*hi + hi*lo + lo*hi is
// accumulated in FP32 (the lo*lo term, ~2^-18 relative, is dropped).  Both
// operators annihilate constants (with the neighbour-trace term of the
// gradient), so each column is shifted by its first value before the split:
// exact algebra that leaves the split error proportional to the variation
// along the line rather than to its level.  Operators are padded to
// multiples of 4 in rows and in K.
template <int N>
struct alignas(16) NsSplitOps {
  static constexpr int RC = (N + 3) / 4;       // 4-row chunks of the outputs
  static constexpr int KA = (N + 3) / 4;       // K chunks of the gradient operator (K = N)
  static constexpr int KM = (N + 4) / 4;       // K chunks of the divergence operator (K = N + 1)
  uint16_t Ahi[4 * RC][4 * KA], Alo[4 * RC][4 * KA];
  uint16_t Mhi[4 * RC][4 * KM], Mlo[4 * RC][4 * KM];
};

typedef short mf_bf16x4 __attribute__((ext_vector_type(4)));
typedef float mf_f32x4 __attribute__((ext_vector_type(4)));

// x = hi + lo + O(2^-18 |x|), both BF16 rounded to nearest even (finite x)
__device__ __forceinline__ uint32_t bf16_rne_bits(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b + 0x7fffu + ((b >> 16) & 1u)) & 0xffff0000u;
}
__device__ __forceinline__ void split_bf16(float x, short &h, short &l) {
  const uint32_t hb = bf16_rne_bits(x);
  h = (short)(hb >> 16);
  l = (short)(bf16_rne_bits(x - __uint_as_float(hb)) >> 16);
}

// y[0 .. 4 RC) = Op x for this lane's column x[0 .. K); Ohi/Olo rows in LDS
template <int K, int RC, int KC, int W>
__device__ __forceinline__ void split_matvec(const uint16_t (*Ohi)[W], const uint16_t (*Olo)[W], const float *x,
                                             float *y, int lane) {
  mf_bf16x4 xh[KC], xl[KC];
#pragma unroll
  for (int kc = 0; kc < KC; ++kc)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      short h, l;
      split_bf16(4 * kc + k < K ? x[4 * kc + k] : 0.0f, h, l);
      xh[kc][k] = h;
      xl[kc][k] = l;
    }
  const int i = lane & 3;
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    mf_f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      const mf_bf16x4 ah = *reinterpret_cast<const mf_bf16x4 *>(&Ohi[4 * r + i][4 * kc]);
      const mf_bf16x4 al = *reinterpret_cast<const mf_bf16x4 *>(&Olo[4 * r + i][4 * kc]);
      acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah, xh[kc], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(ah, xl[kc], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(al, xh[kc], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) y[4 * r + j] = acc[j];
  }
}

// FP32 matrix-core variant (precision SD_FP32_MFMA): the same column
// organisation on the 16-block 4x4x1 FP32 matrix instruction, one
// instruction per K step and 4-row chunk.  The gradient operator is extended
// by the neighbour-trace columns, [A | Mc0/2 | Mc1/2] acting on
// [x; tn0; tn1], so the whole line contraction is on the matrix core; the
// divergence uses M.  Rows padded to multiples of 4.
template <int N>
struct alignas(16) NsF32Ops {
  static constexpr int RC = (N + 3) / 4;
  static constexpr int KG = N + 2, KD = N + 1;
  float G[4 * RC][KG];
  float D[4 * RC][KD];
};

typedef float mf_f32x4v __attribute__((ext_vector_type(4)));

// y[0 .. 4 RC) = Op x for this lane's column x[0 .. K); Op rows in LDS
template <int K, int RC, int W>
__device__ __forceinline__ void f32_matvec(const float (*Op)[W], const float *x, float *y, int lane) {
  const int i = lane & 3;
#pragma unroll
  for (int r = 0; r < RC; ++r) {
    mf_f32x4v acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < K; ++k) acc = __builtin_amdgcn_mfma_f32_4x4x1f32(Op[4 * r + i][k], x[k], acc, 0, 0, 0);
#pragma unroll
    for (int j = 0; j < 4; ++j) y[4 * r + j] = acc[j];
  }
}

// Point values of an element in LDS: x-lines of N values at pitch PT
// (PT = N + 1 in k_rhs_ns, so that the lines read by one wavefront spread
// over the LDS banks; PT = N in k_traces_ns).  Point (i, j, k) sits at
// i + PT (j + N k); line q of direction d as in the face-point numbering
// (d = 0: q = j + N k; d = 1: q = i + N k; d = 2: q = i + N j).
template <int N, int PT>
__device__ __forceinline__ void ns_line(int d, int q, int &base, int &stride) {
  if (d == 0) { base = q * PT; stride = 1; }
  else if (d == 1) { base = (q % N) + PT * N * (q / N); stride = PT; }
  else { base = (q % N) + PT * (q / N); stride = PT * N; }
}
template <int N, int PT>
__device__ __forceinline__ int ns_pidx(int pt) { return (pt % N) + PT * (pt / N); }

template <int N>
struct NsSmem {
  static constexpr int NP = N * N * N, NF = N * N;
  static constexpr int PT = N + 1, NPP = N * N * PT;   // padded point count per variable
  static constexpr int U = 0;                        // [5][NPP]
  static constexpr int G = pad4(U + 5 * NPP);        // [3][5][NPP]; P5: directional residuals
  static constexpr int TNN = pad4(G + 15 * NPP);     // [6][10][NF] neighbour T (v < 5) and NN (v >= 5)
  static constexpr int E = pad4(TNN + 60 * NF);      // [12][5][N] edge-neighbour edge traces
  static constexpr int FH = pad4(E + 60 * N);        // [6][5][NF] interface fluxes
  static constexpr int END = pad4(FH + 30 * NF);
  // [3][N-1][NF][5] interior fluxes: alias TNN..E (dead after P3) when they fit
  static constexpr int FIN = 15 * NF * (N - 1);
  static constexpr int FI = (TNN + FIN <= FH) ? TNN : END;
  static constexpr int TOTAL = (FI == TNN) ? END : pad4(END + FIN);
};

// Launch shape of k_rhs_ns, fixed per instantiation so that the work-item
// index arithmetic divides by compile-time constants: as many elements per
// block as fit a 64 KB LDS target (at most one full block of solution points
// and kNsMaxEpb), and ns_lanes threads per element, at most 256 per block.
// Work items are ordered face-major (P3), direction-major (P2, P4, P5), so
// that with epb * n^2 = 64 (p = 3: four elements) every wavefront works on a
// single face or direction and runs one specialised body.
template <int N, typename R>
__host__ __device__ constexpr int ns_epb() {
  constexpr long long per = (long long)NsSmem<N>::TOTAL * (long long)sizeof(R);
  long long e = (64LL * 1024) / per;
  const long long cap = (256 / (N * N * N)) > 1 ? (256 / (N * N * N)) : 1;
  if (e > cap) e = cap;
  if (e > kNsMaxEpb) e = kNsMaxEpb;
  return e < 1 ? 1 : (int)e;
}
// Lanes per element, measured per degree and precision (TGV workloads of
// 1.9-17 M solution points).
template <int N, typename R>
__host__ __device__ constexpr int ns_lanes() {
  constexpr bool f64 = sizeof(R) == 8;
  return N == 2 ? 32 : N == 3 ? (f64 ? 36 : 72) : N == 4 ? 128 : N == 5 ? 100 : N == 6 ? 256 : 4 * N * N;
}
template <int N, typename R>
__host__ __device__ constexpr int ns_threads() {
  const int t = (ns_epb<N, R>() * ns_lanes<N, R>() + 63) / 64 * 64;
  return t < ns_max_threads<N, R>() ? t : ns_max_threads<N, R>();
}

// Number of neighbours whose state an element reads: 6 across the faces and
// 12 across the edges; BR1 adds the 6 at distance two along the axes (the
// common solution at a face neighbour's far face enters its standard normal
// gradient).
template <bool COMPACT>
__host__ __device__ constexpr int ns_nnb() { return COMPACT ? 18 : 24; }

// Element of block b: blocks are dealt to the eight XCDs of the chip in turn
// (b % 8), so each XCD is given a contiguous range of elements and walks it
// in order; the neighbours an element reads were then read shortly before by
// blocks of the same XCD and are found in its L2.
__device__ __forceinline__ long long ns_block_elem(long long b, long long nblocks, int epb) {
  const long long q = nblocks / 8, r = nblocks % 8;
  const long long x = b % 8, k = b / 8;
  return (x * q + (x < r ? x : r) + k) * epb;
}

// When every direction has an even element count and half the x count is
// a multiple of the block's run, XCD x takes brick x of the 2 x 2 x 2 split
// of the box instead, walking its x-runs row by row and plane by plane: the
// planes of neighbour states it reuses are those of one brick, a quarter of
// the box's.
__device__ __forceinline__ bool ns_bricks(const KArgs &a, int epb) {
  return ((a.nel[0] | a.nel[1] | a.nel[2]) & 1) == 0 && (a.nel[0] / 2) % epb == 0;
}
__device__ __forceinline__ long long ns_block_elem_brick(long long b, const KArgs &a, int epb) {
  const int hx = a.nel[0] / 2, hy = a.nel[1] / 2, hz = a.nel[2] / 2;
  const int x = (int)(b % 8);
  const long long s = b / 8;
  const int bpr = hx / epb;
  const long long row = s / bpr;
  const int col = (int)(s - row * bpr);
  const int ly = (int)(row % hy), lz = (int)(row / hy);
  const int ox = (x & 1) * hx, oy = ((x >> 1) & 1) * hy, oz = (x >> 2) * hz;
  return (long long)(ox + col * epb) + (long long)a.nel[0] * ((oy + ly) + (long long)a.nel[1] * (oz + lz));
}

// number of values moved per vector load for a contiguous run of CNT values
template <typename R, int CNT>
__host__ __device__ constexpr int vec_width() {
  return sizeof(R) == 4 ? (CNT % 4 == 0 ? 4 : (CNT % 2 == 0 ? 2 : 1)) : (CNT % 2 == 0 ? 2 : 1);
}

template <typename R, int W>
struct VecT;
template <> struct VecT<float, 4> { using T = float4; };
template <> struct VecT<float, 2> { using T = float2; };
template <> struct VecT<float, 1> { using T = float; };
template <> struct VecT<double, 2> { using T = double2; };
template <> struct VecT<double, 1> { using T = double; };

// interface flux at face point q of face (D, S), in two passes over the face
// points: PART 0 stores minus the viscous flux of the common solution and
// gradient, PART 1 adds the Roe flux of the two traces.  Each pass keeps only
// its own operands live.
template <int N, typename R, bool COMPACT, int D, int S, int PART>
__device__ __forceinline__ void ns_face_item(const KArgs &a, const NsOps<N, R> &op, R *E, int q) {
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF, f = 2 * D + S, SO = 1 - S;
  R UL[5], UR[5], Uh[5], Vh[15], NNo[5];
  const R thd = (R)a.two_over_h[D];
  int base, stride;
  ns_line<N, SM::PT>(D, q, base, stride);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    // own face trace (and, compact, own normal-gradient trace) from the state
    const R *u = E + SM::U + v * SM::NPP + base;
    R own = R(0), nn = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) {
      R uv = u[c * stride];
      own += op.Lend[S][c] * uv;
      if constexpr (COMPACT) nn += op.rrow[S][c] * uv;
    }
    NNo[v] = nn;
    R oth = E[SM::TNN + (f * 10 + v) * NF + q];
    UL[v] = S == 0 ? oth : own;
    UR[v] = S == 0 ? own : oth;
    Uh[v] = S == 0 ? R(0.5) * (oth + own) : R(0.5) * (own + oth);
  }
  NsConst<R> c(a);
  R F[5];
  if constexpr (PART == 1) {
    ns_roe(c, UL, UR, D, F);
    if (a.tau[D] != 0.0) {
      // interior penalty on the normal component of the common gradient,
      // tau_D (U_R - U_L): the viscous flux is linear in the gradient for a
      // given state, so its share is F_v(U_hat, penalty) (added here, where
      // few registers are live, rather than in the viscous pass)
      R Gp[15];
#pragma unroll
      for (int w = 0; w < 15; ++w) Gp[w] = R(0);
#pragma unroll
      for (int v = 0; v < 5; ++v) Gp[D * 5 + v] = (R)a.tau[D] * (UR[v] - UL[v]);
      Prim<R> sp = ns_prim(c, Uh);
      R Fp[5];
      ns_visc(c, sp, Gp, D, Fp);
#pragma unroll
      for (int v = 0; v < 5; ++v) F[v] -= Fp[v];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) E[SM::FH + (f * 5 + v) * NF + q] += F[v];
    return;
  }
  // normal component: one-sided (compact) or standard (BR1) on each side
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    R vown;
    if constexpr (COMPACT) {
      vown = thd * (NNo[v] + op.kap[S] * Uh[v]);
    } else {
      const R *g = E + SM::G + (D * 5 + v) * SM::NPP + base;
      R acc = R(0);
#pragma unroll
      for (int c = 0; c < N; ++c) acc += op.Lend[S][c] * g[c * stride];
      vown = acc;
    }
    R voth = thd * (E[SM::TNN + (f * 10 + 5 + v) * NF + q] + op.kap[SO] * Uh[v]);
    Vh[D * 5 + v] = S == 0 ? R(0.5) * (voth + vown) : R(0.5) * (vown + voth);
  }
  // transverse components: the standard gradient on both sides
#pragma unroll
  for (int mm = 0; mm < 2; ++mm) {
    const int m = (D + 1 + mm) % 3;        // compile-time after unrolling
    const int t3 = 3 - D - m;
    const int a_lo = q % N, a_hi = q / N;
    const int am = (m < t3) ? a_lo : a_hi, at = (m < t3) ? a_hi : a_lo;
    const int qs = (m < t3) ? at * N : at, qstep = (m < t3) ? 1 : N;
    const R thm = (R)a.two_over_h[m];
    const int e0i = edge_id(D, S, m, 0), e1i = edge_id(D, S, m, 1);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const R *g = E + SM::G + (m * 5 + v) * SM::NPP + base;
      R vown = R(0);
#pragma unroll
      for (int c = 0; c < N; ++c) vown += op.Lend[S][c] * g[c * stride];
      const R *tn = E + SM::TNN + (f * 10 + v) * NF + qs;
      // neighbour's gradient along m at this point, from its face trace
      // along the line and the edge traces of its neighbours (regrouped A)
      R acc = R(0);
#pragma unroll
      for (int c = 0; c < N; ++c) acc += op.A[am][c] * tn[c * qstep];
      R eLn = E[SM::E + (e0i * 5 + v) * N + at];
      R eRn = E[SM::E + (e1i * 5 + v) * N + at];
      R voth = thm * (acc + op.hMc[0][am] * eLn + op.hMc[1][am] * eRn);
      Vh[m * 5 + v] = S == 0 ? R(0.5) * (voth + vown) : R(0.5) * (vown + voth);
    }
  }
  Prim<R> s = ns_prim(c, Uh);
  ns_visc(c, s, Vh, D, F);
#pragma unroll
  for (int v = 0; v < 5; ++v) E[SM::FH + (f * 5 + v) * NF + q] = -F[v];
}

// interior flux at flux point r (1 <= r <= N-1) of line q of family D
template <int N, typename R, int D>
__device__ __forceinline__ void ns_iflux_item(const KArgs &a, const NsOps<N, R> &op, R *E, int q, int r) {
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF;
  int base, stride;
  ns_line<N, SM::PT>(D, q, base, stride);
  R w[N];
#pragma unroll
  for (int c = 0; c < N; ++c) {
    R x = op.Lint[0][c];
#pragma unroll
    for (int k = 1; k < N - 1; ++k) x = (r == k + 1) ? op.Lint[k][c] : x;
    w[c] = x;
  }
  R Uf[5], Gf[15];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const R *u = E + SM::U + v * SM::NPP + base;
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) acc += w[c] * u[c * stride];
    Uf[v] = acc;
  }
#pragma unroll
  for (int m = 0; m < 15; ++m) {
    const R *g = E + SM::G + m * SM::NPP + base;
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) acc += w[c] * g[c * stride];
    Gf[m] = acc;
  }
  R F[5];
  interior_flux<PHYS_NS, 5, R>(a, D, Uf, Gf, F);
  R *fo = E + SM::FI + ((D * (N - 1) + r - 1) * NF + q) * 5;
#pragma unroll
  for (int v = 0; v < 5; ++v) fo[v] = F[v];
}

// divergence of variable v along line q of family D: -2/h_D M F over the
// two interface fluxes and the N-1 interior ones, stored over the gradient
template <int N, typename R, int D>
__device__ __forceinline__ void ns_div_item(const KArgs &a, const NsOps<N, R> &op, R *E, int q, int v) {
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF;
  int base, stride;
  ns_line<N, SM::PT>(D, q, base, stride);
  R F[N + 1];
  F[0] = E[SM::FH + ((2 * D) * 5 + v) * NF + q];
  F[N] = E[SM::FH + ((2 * D + 1) * 5 + v) * NF + q];
#pragma unroll
  for (int c = 1; c < N; ++c) F[c] = E[SM::FI + ((D * (N - 1) + c - 1) * NF + q) * 5 + v];
  const R thd = (R)a.two_over_h[D];
#pragma unroll
  for (int ai = 0; ai < N; ++ai) {
    R acc = R(0);
#pragma unroll
    for (int c = 0; c <= N; ++c) acc += op.M[ai][c] * F[c];
    E[SM::G + (D * 5 + v) * SM::NPP + base + ai * stride] = -thd * acc;
  }
}

// What the right-hand-side kernel does with R at the solution points:
// mode 0 stores it; mode 1 applies one classical RK4 stage in FP64,
//   acc <- first ? R : acc + c R,  out <- u0 + a R      (stages 1-3)
//   out <- u0 + dt6 (acc + R)                          (last stage, out = u0)
// Every block reads its own elements' state before writing them, and other
// blocks only read the trace buffer, so out may alias the input state.
struct RkEpi {
  int mode, first, last;
  double a, c, dt6;
  const double *u0;
  double *acc;
  double *out;
};

// Trace records of a block's elements, assembled in LDS: element el's state
// [5][NP] (reference removed) sits at sm + el * PER + UO and its record (face
// traces T, normal-gradient traces NN, edge traces) goes to sm + el * PER + XO.
// Ends with a barrier.
template <int N, int PT, typename R>
__device__ __forceinline__ void ns_trace_record(R *sm, int PER, int UO, int XO, int epb, int nb,
                                                const NsOps<N, R> &op, int tid, int nth) {
  constexpr int NPV = N * N * PT;                  // values per variable in the state layout
  constexpr int NF = N * N;
  constexpr int FS = trace_face_stride(3, N, 5), EO = trace_edge_off(3, N, 5);
  // face traces and normal-gradient traces, face-major work items
  for (int t = tid; t < 6 * epb * NF; t += nth) {
    int f = t / (epb * NF), r = t % (epb * NF), el = r / NF, q = r % NF;
    if (el >= nb) continue;
    const R *u = sm + el * PER + UO;
    R *x = sm + el * PER + XO;
    auto item = [&](auto Dc, auto Sc) {
      constexpr int D = decltype(Dc)::value, S = decltype(Sc)::value, ff = 2 * D + S;
      int base, stride;
      ns_line<N, PT>(D, q, base, stride);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        R tr = R(0), nn = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) {
          R uv = u[v * NPV + base + c * stride];
          tr += op.Lend[S][c] * uv;
          nn += op.rrow[S][c] * uv;
        }
        x[ff * FS + v * NF + q] = tr;
        x[ff * FS + 5 * NF + v * NF + q] = nn;
      }
    };
    using Z = std::integral_constant<int, 0>;
    using O = std::integral_constant<int, 1>;
    using T2 = std::integral_constant<int, 2>;
    switch (f) {
      case 0: item(Z{}, Z{}); break;
      case 1: item(Z{}, O{}); break;
      case 2: item(O{}, Z{}); break;
      case 3: item(O{}, O{}); break;
      case 4: item(T2{}, Z{}); break;
      default: item(T2{}, O{}); break;
    }
  }
  __syncthreads();
  // edge traces from the face traces: edge (lo, s_lo; hi, s_hi) is the face
  // trace of (lo, s_lo) interpolated along hi to side s_hi
  for (int t = tid; t < nb * 12 * 5 * N; t += nth) {
    int el = t / (60 * N), r = t % (60 * N);
    int ed = r / (5 * N), w = r % (5 * N), v = w / N, at = w % N;
    int P = ed >> 2, slo = (ed >> 1) & 1, shi = ed & 1;
    int lo = P == 2 ? 1 : 0, hi = P == 0 ? 1 : 2, t3 = 3 - lo - hi;
    R *x = sm + el * PER + XO;
    const R *tf = x + (2 * lo + slo) * FS + v * NF;
    R acc = R(0);
#pragma unroll
    for (int c = 0; c < N; ++c) acc += op.Lend[shi][c] * tf[(hi < t3) ? (at * N + c) : (c * N + at)];
    x[EO + (ed * 5 + v) * N + at] = acc;
  }
  __syncthreads();
}

// contiguous vector store of the block's trace records to X
template <int N, typename R>
__device__ __forceinline__ void ns_store_records(const R *sm, int PER, int XO, R *X, long long e0, int nb, int tid,
                                                 int nth) {
  constexpr int XS = trace_stride(3, N, 5);
  constexpr int W = vec_width<R, XS>();
  using V = typename VecT<R, W>::T;
  V *dst = reinterpret_cast<V *>(X + e0 * XS);
  for (int t = tid; t < nb * XS / W; t += nth) {
    int el = (t * W) / XS, r = (t * W) % XS;
    dst[t] = *reinterpret_cast<const V *>(sm + el * PER + XO + r);
  }
}

// Element-local trace kernel for the Navier-Stokes system: the full trace
// record of every element is assembled in LDS and stored with contiguous
// vector stores.
template <int N, typename R>
__global__ void __launch_bounds__(256) k_traces_ns(const double *__restrict__ U, R *__restrict__ X, KArgs a,
                                                   NsOps<N, R> op) {
  constexpr int NP = N * N * N;
  constexpr int XS = trace_stride(3, N, 5);
  constexpr int PER = pad4(5 * NP) + pad4(XS);
  extern __shared__ double2 smem_tr[];
  R *sm = reinterpret_cast<R *>(smem_tr);
  const int tid = threadIdx.x, nth = blockDim.x;
  const int epb = a.epb;
  const int e0 = blockIdx.x * epb;
  const int nb = min(epb, (int)(a.ne - e0));
  {
    constexpr int W = (NP % 2 == 0) ? 2 : 1;
    using V = typename VecT<double, W>::T;
    const V *src = reinterpret_cast<const V *>(U + (long long)e0 * 5 * NP);
    for (int t = tid; t < nb * 5 * NP / W; t += nth) {
      int r = (t * W) % (5 * NP), el = (t * W) / (5 * NP);
      double u0 = a.U0[r / NP];
      R *dst = sm + el * PER + r;
      if constexpr (W == 2) {
        V x = src[t];
        dst[0] = (R)(x.x - u0);
        dst[1] = (R)(x.y - u0);
      } else {
        dst[0] = (R)(src[t] - u0);
      }
    }
  }
  __syncthreads();
  ns_trace_record<N, N, R>(sm, PER, 0, pad4(5 * NP), epb, nb, op, tid, nth);
  ns_store_records<N, R>(sm, PER, pad4(5 * NP), X, e0, nb, tid, nth);
}

// Chained RK stages (fused path without a closure): the stage state between
// stages is kept in compute precision with the reference state removed (the
// value the kernel would round the FP64 state to).  in_r: stage state to
// read instead of U (nullptr: U); out_r: where the stage epilogue writes the
// next stage state (nullptr: FP64 epilogue of RkEpi).  Every block reads the
// states of its elements' neighbours, so out_r must not alias in_r.
template <typename R>
struct NsChain {
  const R *in_r;
  R *out_r;
};

// Readers of the stage state for the prologue of k_rhs_ns: compute-precision
// stage state (reference already removed), or the FP64 state U with the
// reference state (U0[0] on rho, U0[4] on rho E; zero on the momenta) removed
// before rounding.
template <typename R>
struct NsSrcR {
  const R *__restrict__ p;
  __device__ __forceinline__ R operator()(long long i, int) const { return p[i]; }
  template <int W>
  __device__ __forceinline__ void vec(long long i, int, R *x, std::integral_constant<int, W>) const {
    using V = typename VecT<R, W>::T;
    const V v = *reinterpret_cast<const V *>(p + i);
    const R *xv = reinterpret_cast<const R *>(&v);
#pragma unroll
    for (int w = 0; w < W; ++w) x[w] = xv[w];
  }
};
template <typename R>
struct NsSrcU {
  const double *__restrict__ p;
  double r0, e0;
  __device__ __forceinline__ R operator()(long long i, int v) const {
    return (R)(p[i] - (v == 0 ? r0 : (v == 4 ? e0 : 0.0)));
  }
  // W consecutive values of one variable v (W divides the per-variable count)
  template <int W>
  __device__ __forceinline__ void vec(long long i, int v, R *x, std::integral_constant<int, W>) const {
    const double u0 = v == 0 ? r0 : (v == 4 ? e0 : 0.0);
    if constexpr (W % 2 == 0) {
#pragma unroll
      for (int w = 0; w < W; w += 2) {
        const double2 d = *reinterpret_cast<const double2 *>(p + i + w);
        x[w] = (R)(d.x - u0);
        x[w + 1] = (R)(d.y - u0);
      }
    } else {
#pragma unroll
      for (int w = 0; w < W; ++w) x[w] = (R)(p[i + w] - u0);
    }
  }
};

// Neighbour k of element e: k < 6 across face (k >> 1, k & 1); 6 <= k < 18
// across edge k - 6 (a step along lo to side slo and along hi to side shi,
// the edge numbering of the trace records); 18 <= k < 24 two steps across
// face k - 18 (BR1 only).  Periodic box.
__device__ __forceinline__ int ns_neighbour(const KArgs &a, int e, int k) {
  const int nx = a.nel[0], ny = a.nel[1], nz = a.nel[2];
  int c[3] = {e % nx, (e / nx) % ny, e / (nx * ny)};
  const int ext[3] = {nx, ny, nz};
  auto step = [&](int d, int s, int dist) {
    int x = pick(d, c[0], c[1], c[2]);
    const int n = pick(d, ext[0], ext[1], ext[2]);
    x = s ? (x + dist) % n : (x - dist % n + n) % n;
    if (d == 0) c[0] = x;
    else if (d == 1) c[1] = x;
    else c[2] = x;
  };
  if (k < 6) {
    step(k >> 1, k & 1, 1);
  } else if (k < 18) {
    const int ed = k - 6, P = ed >> 2;
    step(P == 2 ? 1 : 0, (ed >> 1) & 1, 1);
    step(P == 0 ? 1 : 2, ed & 1, 1);
  } else {
    step((k - 18) >> 1, (k - 18) & 1, 2);
  }
  return c[0] + nx * (c[1] + ny * c[2]);
}

// Prologue of k_rhs_ns for a block: the state of its elements into LDS, the
// neighbours' face traces T and normal-gradient traces NN of the shared faces
// and the edge neighbours' edge traces, computed from the neighbours' states
// read through the source src (NsSrcR or NsSrcU).  Every global read is
// unrolled with a compile-time trip count and issued in chunks of about 64
// registers before any of them is used, so that an element waits for the
// latency of its neighbour reads once or twice, not once per work item.
template <int N, typename R>
struct NsTraceOps {
  R Lend[2][N];
  R rrow[2][N];
  R kapx[2];
};

template <int N, typename R, bool COMPACT, int NNB, class Src>
__device__ __forceinline__ void ns_prologue(const Src &src, const NsTraceOps<N, R> op, R *sm,
                                            const int (*snb)[NNB], int e0, int nb, int tid) {
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF;
  constexpr int nth = ns_threads<N, R>();
  constexpr int epb = ns_epb<N, R>();
  // own state into LDS (x-lines at pitch PT)
  auto own_state = [&]() __attribute__((always_inline)) {
    constexpr int W = vec_width<R, 5 * NP>();
    constexpr int RND = (epb * 5 * NP / W + nth - 1) / nth;
#pragma unroll
    for (int it = 0; it < RND; ++it) {
      const int t = tid + it * nth;
      if (t < nb * 5 * NP / W) {
        const int r = (t * W) % (5 * NP), el = (t * W) / (5 * NP);
        R xv[W];
        src.vec((long long)e0 * 5 * NP + (long long)t * W, r / NP, xv, std::integral_constant<int, W>{});
#pragma unroll
        for (int w = 0; w < W; ++w) {
          const int rw = r + w;
          sm[el * SM::TOTAL + SM::U + (rw / NP) * SM::NPP + ns_pidx<N, SM::PT>(rw % NP)] = xv[w];
        }
      }
    }
  };
  // face neighbours: T and NN of the shared face.  The directions are
  // unrolled at compile time, so the reads of a line sit at constant offsets
  // from one address; work items past the end read valid data of the first
  // item and store nothing, so the reads need no branches.
  // values per vector read of a contiguous x-run of N values (aligned: every
  // run starts at a multiple of N within an element of 5 N^3 values)
  constexpr int WN = sizeof(R) == 4 ? (N % 4 == 0 ? 4 : (N % 2 == 0 ? 2 : 1)) : (N % 2 == 0 ? 2 : 1);
  constexpr int FCNT = epb * 2 * 5 * NF, FRND = (FCNT + nth - 1) / nth;
  constexpr int NL = COMPACT ? N : 2 * N;
  struct FaceBuf {
    R x[FRND][NL];
  };
  auto faces_load = [&](auto Dc, FaceBuf &b) __attribute__((always_inline)) {
    constexpr int D = decltype(Dc)::value;
    constexpr int ST = D == 0 ? 1 : (D == 1 ? N : N * N);
#pragma unroll
    for (int it = 0; it < FRND; ++it) {
      const int t = tid + it * nth, tc = t < FCNT ? t : 0;
      const int S = tc / (epb * 5 * NF), r = tc % (epb * 5 * NF), el = r / (5 * NF), w = r % (5 * NF);
      const int v = w / NF, q = w % NF;
      int base, stride;
      ns_line<N, N>(D, q, base, stride);
      const int elc = el < nb ? el : 0;
      const long long o = (long long)snb[elc][2 * D + S] * 5 * NP + v * NP + base;
      auto line = [&](long long oo, R *x) __attribute__((always_inline)) {
        if constexpr (ST == 1) {
          // an x-line is contiguous: vector reads
#pragma unroll
          for (int c = 0; c < N; c += WN) src.vec(oo + c, v, x + c, std::integral_constant<int, WN>{});
        } else {
#pragma unroll
          for (int c = 0; c < N; ++c) x[c] = src(oo + c * ST, v);
        }
      };
      line(o, b.x[it]);
      if constexpr (!COMPACT) {
        const long long o2 = (long long)snb[elc][18 + 2 * D + S] * 5 * NP + v * NP + base;
        line(o2, b.x[it] + N);
      }
    }
  };
  auto faces_compute = [&](auto Dc, const FaceBuf &b) __attribute__((always_inline)) {
    constexpr int D = decltype(Dc)::value;
#pragma unroll
    for (int it = 0; it < FRND; ++it) {
      const int t = tid + it * nth;
      const int S = t / (epb * 5 * NF), r = t % (epb * 5 * NF), el = r / (5 * NF), w = r % (5 * NF);
      const int v = w / NF, q = w % NF;
      // the neighbour's side of the shared face is 1 - S; the operator rows
      // stay at compile-time indices (SC: side S known at compile time)
      auto side = [&](auto SC, R &tr, R &nn) __attribute__((always_inline)) {
        constexpr int SS = decltype(SC)::value, SO = 1 - SS;
        tr = R(0);
        nn = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) {
          tr += op.Lend[SO][c] * b.x[it][c];
          nn += op.rrow[SO][c] * b.x[it][c];
        }
        if constexpr (!COMPACT) {
          // BR1: common solution at the neighbour's far face (side S)
          R mine = R(0), theirs = R(0);
#pragma unroll
          for (int c = 0; c < N; ++c) {
            mine += op.Lend[SS][c] * b.x[it][c];
            theirs += op.Lend[SO][c] * b.x[it][N + c];
          }
          const R uh = SS ? R(0.5) * (mine + theirs) : R(0.5) * (theirs + mine);
          nn += op.kapx[SO] * uh;
        }
      };
      R tr, nn;
      if constexpr ((epb * 5 * NF) % 64 == 0) {
        // S is the same across the wavefront: one side's sums
        if (__builtin_amdgcn_readfirstlane(S)) side(std::integral_constant<int, 1>{}, tr, nn);
        else side(std::integral_constant<int, 0>{}, tr, nn);
      } else {
        // both sides' sums formed, one selected
        R ta, na, tb, nb2;
        side(std::integral_constant<int, 1>{}, ta, na);
        side(std::integral_constant<int, 0>{}, tb, nb2);
        tr = S ? ta : tb;
        nn = S ? na : nb2;
      }
      if (t < FCNT && el < nb) {
        R *E = sm + el * SM::TOTAL;
        const int f = 2 * D + S;
        E[SM::TNN + (f * 10 + v) * NF + q] = tr;
        E[SM::TNN + (f * 10 + 5 + v) * NF + q] = nn;
      }
    }
  };
  // edge neighbours, one edge family P (edges along t3, spanned by lo < hi)
  // at a time: the trace of the neighbour across edge ed at the shared edge,
  // i.e. its face trace on face (lo, 1 - slo) interpolated along hi to side
  // 1 - shi
  constexpr int ECNT = epb * 4 * 5 * N, ERND = (ECNT + nth - 1) / nth;
  struct EdgeBuf {
    R x[ERND][N * N];
  };
  auto edges_load = [&](auto Pc, EdgeBuf &b) __attribute__((always_inline)) {
    constexpr int P = decltype(Pc)::value;
    constexpr int lo = P == 2 ? 1 : 0, hi = P == 0 ? 1 : 2, t3 = 3 - lo - hi;
    constexpr int SL = lo == 0 ? 1 : N, SH = hi == 1 ? N : N * N, ST = t3 == 2 ? N * N : (t3 == 1 ? N : 1);
#pragma unroll
    for (int it = 0; it < ERND; ++it) {
      const int t = tid + it * nth, tc = t < ECNT ? t : 0;
      const int el = tc / (20 * N), r = tc % (20 * N), e4 = r / (5 * N), w = r % (5 * N), v = w / N, at = w % N;
      const int elc = el < nb ? el : 0;
      const long long o = (long long)snb[elc][6 + 4 * P + e4] * 5 * NP + v * NP + at * ST;
#pragma unroll
      for (int c2 = 0; c2 < N; ++c2) {
        if constexpr (SL == 1) {
          // the lo direction is x: each run of N values is contiguous
#pragma unroll
          for (int c1 = 0; c1 < N; c1 += WN)
            src.vec(o + c1 + c2 * SH, v, b.x[it] + c2 * N + c1, std::integral_constant<int, WN>{});
        } else {
#pragma unroll
          for (int c1 = 0; c1 < N; ++c1) b.x[it][c2 * N + c1] = src(o + c1 * SL + c2 * SH, v);
        }
      }
    }
  };
  auto edges_compute = [&](auto Pc, const EdgeBuf &b) __attribute__((always_inline)) {
    constexpr int P = decltype(Pc)::value;
#pragma unroll
    for (int it = 0; it < ERND; ++it) {
      const int t = tid + it * nth;
      const int el = t / (20 * N), r = t % (20 * N), e4 = r / (5 * N), w = r % (5 * N), v = w / N, at = w % N;
      const bool slo = (e4 >> 1) != 0, shi = (e4 & 1) != 0;
      // the rows of the two interpolations, selected per lane (the neighbour
      // sides are 1 - slo and 1 - shi); the rows are register values here
      R rl[N], rh[N];
#pragma unroll
      for (int c = 0; c < N; ++c) {
        rl[c] = slo ? op.Lend[0][c] : op.Lend[1][c];
        rh[c] = shi ? op.Lend[0][c] : op.Lend[1][c];
      }
      R acc = R(0);
#pragma unroll
      for (int c2 = 0; c2 < N; ++c2) {
        R inner = R(0);
#pragma unroll
        for (int c1 = 0; c1 < N; ++c1) inner += rl[c1] * b.x[it][c2 * N + c1];
        acc += rh[c2] * inner;
      }
      if (t < ECNT && el < nb) sm[el * SM::TOTAL + SM::E + ((4 * P + e4) * 5 + v) * N + at] = acc;
    }
  };
  using I0 = std::integral_constant<int, 0>;
  using I1 = std::integral_constant<int, 1>;
  using I2 = std::integral_constant<int, 2>;
  // reads issued ahead of the arithmetic that uses them, as far as about 48
  // registers of read data allow
  constexpr int FACE_REGS = 3 * FRND * NL * (int)(sizeof(R) / 4);
  if constexpr (FACE_REGS <= 48) {
    FaceBuf f0, f1, f2;
    faces_load(I0{}, f0);
    faces_load(I1{}, f1);
    faces_load(I2{}, f2);
    own_state();
    faces_compute(I0{}, f0);
    faces_compute(I1{}, f1);
    faces_compute(I2{}, f2);
  } else {
    own_state();
    FaceBuf f0;
    faces_load(I0{}, f0);
    faces_compute(I0{}, f0);
    FaceBuf f1;
    faces_load(I1{}, f1);
    faces_compute(I1{}, f1);
    FaceBuf f2;
    faces_load(I2{}, f2);
    faces_compute(I2{}, f2);
  }
  EdgeBuf g0;
  edges_load(I0{}, g0);
  edges_compute(I0{}, g0);
  EdgeBuf g1;
  edges_load(I1{}, g1);
  edges_compute(I1{}, g1);
  EdgeBuf g2;
  edges_load(I2{}, g2);
  edges_compute(I2{}, g2);
}

// Wavefronts per SIMD that the LDS of k_rhs_ns allows (160 KB per compute
// unit, four SIMDs): the register budget the kernel is compiled for, so that
// registers do not limit the occupancy below what the LDS gives (rounded
// down, except that 1.5 counts as 2).
template <int N, typename R>
__host__ __device__ constexpr int ns_waves_per_simd() {
  const int blocks = (160 * 1024) / ((int)sizeof(R) * NsSmem<N>::TOTAL * ns_epb<N, R>() + 1024);
  const int tot = blocks * (ns_threads<N, R>() / 64);
  const int w = (tot >= 6 && tot < 8) ? 2 : tot / 4;
  // at most four (128 registers or more); FP64 at most two (its values take
  // register pairs, and the face pass then needs about 250 registers)
  const int cap = sizeof(R) == 8 ? 2 : 4;
  return w < 1 ? 1 : (w > cap ? cap : w);
}

// MM: 0 vector units; 1 BF16x3 split precision on the BF16 matrix cores;
// 2 FP32 on the FP32 matrix cores (gradient and divergence contractions)
template <int N, typename R, bool COMPACT, int MM = 0>
__global__ void __launch_bounds__((ns_threads<N, R>()))
__attribute__((amdgpu_waves_per_eu(ns_waves_per_simd<N, R>(), 8))) k_rhs_ns(const double *__restrict__ U,
                                                                 double *__restrict__ dudt, KArgs a,
                                                                 NsOps<N, R> op, RkEpi ep, NsSplitOps<N> spo, NsF32Ops<N> fpo,
                                                                 NsChain<R> ch) {
  constexpr bool SPLIT = MM == 1, MF32 = MM == 2;
  static_assert(MM == 0 || sizeof(R) == 4, "BF16x3 and FP32 matrix-core variants work on the FP32 kernel");
  using SM = NsSmem<N>;
  constexpr int NP = SM::NP, NF = SM::NF;
  constexpr int NNB = ns_nnb<COMPACT>();
  extern __shared__ double2 smem_ns[];          // 16-byte aligned dynamic LDS
  R *sm = reinterpret_cast<R *>(smem_ns);
  __shared__ int snb[ns_epb<N, R>()][NNB];
  __shared__ NsSplitOps<SPLIT ? N : 1> ssp;
  __shared__ NsF32Ops<MF32 ? N : 1> sfp;
  constexpr int nth = ns_threads<N, R>();          // == blockDim.x
  const int tid = threadIdx.x;
  if constexpr (SPLIT) {
    constexpr int WORDS = sizeof(NsSplitOps<N>) / 4;
    for (int t = tid; t < WORDS; t += nth)
      reinterpret_cast<uint32_t *>(&ssp)[t] = reinterpret_cast<const uint32_t *>(&spo)[t];
  }
  if constexpr (MF32) {
    constexpr int WORDS = sizeof(NsF32Ops<N>) / 4;
    for (int t = tid; t < WORDS; t += nth)
      reinterpret_cast<uint32_t *>(&sfp)[t] = reinterpret_cast<const uint32_t *>(&fpo)[t];
  }
  constexpr int epb = ns_epb<N, R>();              // == a.epb
  const long long nblocks = (a.ne + epb - 1) / epb;
  const int e0 = (int)(ns_bricks(a, epb) ? ns_block_elem_brick(blockIdx.x, a, epb)
                                          : ns_block_elem(blockIdx.x, nblocks, epb));
  const int nb = min(epb, (int)(a.ne - e0));
  const R *__restrict__ in_r = ch.in_r;

  // the waves of blocks in the prologue, the phase that reads the
  // neighbours' states, issue ahead of those computing (32^3 p = 3: FP64
  // 504 -> 479 us per stage, FP32 204 -> 199 us)
  __builtin_amdgcn_s_setprio(3);
  // P0: neighbour table; then the state and the neighbours' traces computed
  // from their states (read through L2)
  for (int t = tid; t < nb * NNB; t += nth) snb[t / NNB][t % NNB] = ns_neighbour(a, e0 + t / NNB, t % NNB);
  __syncthreads();
  {
    // the operator rows of the prologue, copied with compile-time indices
    // (each of the two inlined prologues then keeps them in registers)
    NsTraceOps<N, R> to;
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        to.Lend[s2][c] = op.Lend[s2][c];
        to.rrow[s2][c] = op.rrow[s2][c];
      }
      to.kapx[s2] = op.kapx[s2];
    }
    if (in_r) ns_prologue<N, R, COMPACT, NNB>(NsSrcR<R>{in_r}, to, sm, snb, e0, nb, tid);
    else ns_prologue<N, R, COMPACT, NNB>(NsSrcU<R>{U, a.U0[0], a.U0[4]}, to, sm, snb, e0, nb, tid);
  }
  __syncthreads();
  __builtin_amdgcn_s_setprio(0);
  // P2: gradient at the solution points
  if constexpr (SPLIT) {
    // one column per (direction, element, variable, line):
    // g = (2/h_m) [A x + (Mc0 tn0 + Mc1 tn1) / 2],  A = D - (Mc0 Lend0^T + Mc1 Lend1^T) / 2
    using SO = NsSplitOps<N>;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
    const int ncol = 3 * epb * 5 * NF;
    for (int b0 = wave * 64; b0 < ncol; b0 += nwaves * 64) {
      const int col = b0 + lane;
      const int m = col / (epb * 5 * NF), r0 = col % (epb * 5 * NF);
      const int el = r0 / (5 * NF), w = r0 % (5 * NF), v = w / NF, q = w % NF;
      const bool ok = col < ncol && el < nb;
      R x[N];
      R tn0 = R(0), tn1 = R(0);
      int base = 0, stride = 0;
      R *E = sm + (ok ? el : 0) * SM::TOTAL;
#pragma unroll
      for (int c = 0; c < N; ++c) x[c] = R(0);
      if (ok) {
        ns_line<N, SM::PT>(m, q, base, stride);
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] = E[SM::U + v * SM::NPP + base + c * stride];
        tn0 = E[SM::TNN + ((2 * m) * 10 + v) * NF + q];
        tn1 = E[SM::TNN + ((2 * m + 1) * 10 + v) * NF + q];
        const R x0 = x[0];
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] -= x0;
        tn0 -= x0;
        tn1 -= x0;
      }
      float y[4 * SO::RC];
      split_matvec<N, SO::RC, SO::KA>(ssp.Ahi, ssp.Alo, x, y, lane);
      if (ok) {
        const R th = (R)pick(m, a.two_over_h[0], a.two_over_h[1], a.two_over_h[2]);
#pragma unroll
        for (int ai = 0; ai < N; ++ai)
          E[SM::G + (m * 5 + v) * SM::NPP + base + ai * stride] =
              th * (y[ai] + R(0.5) * (op.Mc[0][ai] * tn0 + op.Mc[1][ai] * tn1));
      }
    }
  } else if constexpr (MF32) {
    // one column per (direction, element, variable, line):
    // g = (2/h_m) [A x + (Mc0 tn0 + Mc1 tn1) / 2] as one contraction over
    // [x; tn0; tn1] on the FP32 matrix instruction
    using FO = NsF32Ops<N>;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
    const int ncol = 3 * epb * 5 * NF;
    for (int b0 = wave * 64; b0 < ncol; b0 += nwaves * 64) {
      const int col = b0 + lane;
      const int m = col / (epb * 5 * NF), r0 = col % (epb * 5 * NF);
      const int el = r0 / (5 * NF), w = r0 % (5 * NF), v = w / NF, q = w % NF;
      const bool ok = col < ncol && el < nb;
      float x[FO::KG];
      int base = 0, stride = 0;
      R *E = sm + (ok ? el : 0) * SM::TOTAL;
#pragma unroll
      for (int c = 0; c < FO::KG; ++c) x[c] = 0.0f;
      if (ok) {
        ns_line<N, SM::PT>(m, q, base, stride);
#pragma unroll
        for (int c = 0; c < N; ++c) x[c] = E[SM::U + v * SM::NPP + base + c * stride];
        x[N] = E[SM::TNN + ((2 * m) * 10 + v) * NF + q];
        x[N + 1] = E[SM::TNN + ((2 * m + 1) * 10 + v) * NF + q];
      }
      float y[4 * FO::RC];
      f32_matvec<FO::KG, FO::RC>(sfp.G, x, y, lane);
      if (ok) {
        const R th = (R)pick(m, a.two_over_h[0], a.two_over_h[1], a.two_over_h[2]);
#pragma unroll
        for (int ai = 0; ai < N; ++ai) E[SM::G + (m * 5 + v) * SM::NPP + base + ai * stride] = th * y[ai];
      }
    }
  } else
  for (int t = tid; t < nb * NP; t += nth) {
    int el = t / NP, pt = t % NP;
    R *E = sm + el * SM::TOTAL;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
      int am, qm, base, stride;
      coord_of<3, N>(pt, m, am, qm);
      ns_line<N, SM::PT>(m, qm, base, stride);
      R th = (R)a.two_over_h[m];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        const R *u = E + SM::U + v * SM::NPP + base;
        R acc = R(0);
#pragma unroll
        for (int c = 0; c < N; ++c) acc += op.A[am][c] * u[c * stride];
        R tn0 = E[SM::TNN + ((2 * m) * 10 + v) * NF + qm];
        R tn1 = E[SM::TNN + ((2 * m + 1) * 10 + v) * NF + qm];
        acc += op.hMc[0][am] * tn0 + op.hMc[1][am] * tn1;
        E[SM::G + (m * 5 + v) * SM::NPP + ns_pidx<N, SM::PT>(pt)] = th * acc;
      }
    }
  }
  __syncthreads();
  // P3: interface fluxes, face-major work items, in two passes (minus the
  // viscous flux, then plus the Roe flux) over the face points
  auto p3item = [&](auto Pc, int t) {
    constexpr int PART = decltype(Pc)::value;
    const int f = t / (epb * NF), r = t % (epb * NF), el = r / NF, q = r % NF;
    if (el >= nb) return;
    R *E = sm + el * SM::TOTAL;
    switch (f) {
      case 0: ns_face_item<N, R, COMPACT, 0, 0, PART>(a, op, E, q); break;
      case 1: ns_face_item<N, R, COMPACT, 0, 1, PART>(a, op, E, q); break;
      case 2: ns_face_item<N, R, COMPACT, 1, 0, PART>(a, op, E, q); break;
      case 3: ns_face_item<N, R, COMPACT, 1, 1, PART>(a, op, E, q); break;
      case 4: ns_face_item<N, R, COMPACT, 2, 0, PART>(a, op, E, q); break;
      default: ns_face_item<N, R, COMPACT, 2, 1, PART>(a, op, E, q); break;
    }
  };
  constexpr int PI = 6 * epb * NF;   // face points of the block: items per pass
  if constexpr (PI >= nth) {
    // both passes as one list of 2 PI items in rounds of nth separated by
    // barriers: a face point's second pass falls in a later round than its
    // first (PI >= nth), and no wavefront idles while the others finish a
    // pass (at p = 3, 6 x 64 + 6 x 64 items are three rounds of four
    // wavefronts, each on one face and pass)
    constexpr int RND = (2 * PI + nth - 1) / nth;
    for (int rr = 0; rr < RND; ++rr) {
      const int t = tid + rr * nth;
      if (t < PI) p3item(std::integral_constant<int, 0>{}, t);
      else if (t < 2 * PI) p3item(std::integral_constant<int, 1>{}, t - PI);
      __syncthreads();
    }
  } else {
    // the same thread takes the same face point in both passes, so the
    // second reads its own LDS writes
    for (int t = tid; t < PI; t += nth) p3item(std::integral_constant<int, 0>{}, t);
    for (int t = tid; t < PI; t += nth) p3item(std::integral_constant<int, 1>{}, t);
    __syncthreads();
  }
  // P4: interior fluxes, items ordered (direction, flux point, element, line)
  for (int t = tid; t < 3 * (N - 1) * epb * NF; t += nth) {
    int d = t / ((N - 1) * epb * NF), r0 = t % ((N - 1) * epb * NF);
    int r = 1 + r0 / (epb * NF), w = r0 % (epb * NF), el = w / NF, q = w % NF;
    if (el >= nb) continue;
    R *E = sm + el * SM::TOTAL;
    switch (d) {
      case 0: ns_iflux_item<N, R, 0>(a, op, E, q, r); break;
      case 1: ns_iflux_item<N, R, 1>(a, op, E, q, r); break;
      default: ns_iflux_item<N, R, 2>(a, op, E, q, r); break;
    }
  }
  __syncthreads();
  // RK stage inputs of this thread's values, requested now so that their
  // latency passes during the divergence
  constexpr int ERK = (epb * 5 * NP + nth - 1) / nth;
  constexpr bool PREF = ERK * 4 <= 24;     // registers of the prefetched values
  double pu0[ERK], pac[ERK];
  if (PREF && ep.mode != 0) {
#pragma unroll
    for (int k = 0; k < ERK; ++k) {
      const int t = tid + k * nth;
      const long long i = (long long)e0 * 5 * NP + (t < nb * 5 * NP ? t : 0);
      pu0[k] = __builtin_nontemporal_load(ep.u0 + i);
      pac[k] = ep.first ? 0.0 : __builtin_nontemporal_load(ep.acc + i);
    }
  }
  // P5: divergence per line and variable, items ordered (direction, element,
  // variable, line); then the three contributions summed in FP64
  if constexpr (SPLIT) {
    using SO = NsSplitOps<N>;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
    const int ncol = 3 * epb * 5 * NF;
    for (int b0 = wave * 64; b0 < ncol; b0 += nwaves * 64) {
      const int col = b0 + lane;
      const int d = col / (epb * 5 * NF), r0 = col % (epb * 5 * NF);
      const int el = r0 / (5 * NF), w = r0 % (5 * NF), v = w / NF, q = w % NF;
      const bool ok = col < ncol && el < nb;
      R F[N + 1];
      int base = 0, stride = 0;
      R *E = sm + (ok ? el : 0) * SM::TOTAL;
#pragma unroll
      for (int c = 0; c <= N; ++c) F[c] = R(0);
      if (ok) {
        ns_line<N, SM::PT>(d, q, base, stride);
        F[0] = E[SM::FH + ((2 * d) * 5 + v) * NF + q];
        F[N] = E[SM::FH + ((2 * d + 1) * 5 + v) * NF + q];
#pragma unroll
        for (int c = 1; c < N; ++c) F[c] = E[SM::FI + ((d * (N - 1) + c - 1) * NF + q) * 5 + v];
        const R f0 = F[0];
#pragma unroll
        for (int c = 0; c <= N; ++c) F[c] -= f0;
      }
      float y[4 * SO::RC];
      split_matvec<N + 1, SO::RC, SO::KM>(ssp.Mhi, ssp.Mlo, F, y, lane);
      if (ok) {
        const R thd = (R)pick(d, a.two_over_h[0], a.two_over_h[1], a.two_over_h[2]);
#pragma unroll
        for (int ai = 0; ai < N; ++ai) E[SM::G + (d * 5 + v) * SM::NPP + base + ai * stride] = -thd * y[ai];
      }
    }
  } else if constexpr (MF32) {
    using FO = NsF32Ops<N>;
    const int lane = tid & 63, wave = tid >> 6, nwaves = nth >> 6;
    const int ncol = 3 * epb * 5 * NF;
    for (int b0 = wave * 64; b0 < ncol; b0 += nwaves * 64) {
      const int col = b0 + lane;
      const int d = col / (epb * 5 * NF), r0 = col % (epb * 5 * NF);
      const int el = r0 / (5 * NF), w = r0 % (5 * NF), v = w / NF, q = w % NF;
      const bool ok = col < ncol && el < nb;
      float F[N + 1];
      int base = 0, stride = 0;
      R *E = sm + (ok ? el : 0) * SM::TOTAL;
#pragma unroll
      for (int c = 0; c <= N; ++c) F[c] = 0.0f;
      if (ok) {
        ns_line<N, SM::PT>(d, q, base, stride);
        F[0] = E[SM::FH + ((2 * d) * 5 + v) * NF + q];
        F[N] = E[SM::FH + ((2 * d + 1) * 5 + v) * NF + q];
#pragma unroll
        for (int c = 1; c < N; ++c) F[c] = E[SM::FI + ((d * (N - 1) + c - 1) * NF + q) * 5 + v];
      }
      float y[4 * FO::RC];
      f32_matvec<N + 1, FO::RC>(sfp.D, F, y, lane);
      if (ok) {
        const R thd = (R)pick(d, a.two_over_h[0], a.two_over_h[1], a.two_over_h[2]);
#pragma unroll
        for (int ai = 0; ai < N; ++ai) E[SM::G + (d * 5 + v) * SM::NPP + base + ai * stride] = -thd * y[ai];
      }
    }
  } else
  for (int t = tid; t < 3 * epb * 5 * NF; t += nth) {
    int d = t / (epb * 5 * NF), r0 = t % (epb * 5 * NF);
    int el = r0 / (5 * NF), w = r0 % (5 * NF), v = w / NF, q = w % NF;
    if (el >= nb) continue;
    R *E = sm + el * SM::TOTAL;
    switch (d) {
      case 0: ns_div_item<N, R, 0>(a, op, E, q, v); break;
      case 1: ns_div_item<N, R, 1>(a, op, E, q, v); break;
      default: ns_div_item<N, R, 2>(a, op, E, q, v); break;
    }
  }
  __syncthreads();
  // the values of the RK stage (step start u0, accumulator) were requested
  // before the divergence; the RK streams are read and written once per
  // stage: non-temporal, so that they do not push the neighbour states out of
  // L2
#pragma unroll
  for (int k = 0; k < ERK; ++k) {
    const int t = tid + k * nth;
    if (t >= nb * 5 * NP) break;
    const int el = t / (5 * NP), r = t % (5 * NP);
    const int pr = (r / NP) * SM::NPP + ns_pidx<N, SM::PT>(r % NP);
    const R *E = sm + el * SM::TOTAL + SM::G + pr;
    double Rv = (double)E[0] + (double)E[5 * SM::NPP] + (double)E[10 * SM::NPP];
    long long i = (long long)e0 * 5 * NP + t;
    if (ep.mode == 0) {
      __builtin_nontemporal_store(Rv, dudt + i);
    } else {
      const double u0v = PREF ? pu0[k] : __builtin_nontemporal_load(ep.u0 + i);
      double accv = ep.first ? Rv : (PREF ? pac[k] : __builtin_nontemporal_load(ep.acc + i)) + ep.c * Rv;
      if (ep.last) {
        __builtin_nontemporal_store(u0v + ep.dt6 * accv, ep.out + i);
      } else {
        __builtin_nontemporal_store(accv, ep.acc + i);
        const double w = u0v + ep.a * Rv;
        if (ch.out_r) {
          // next stage state, as the next kernel would round it
          ch.out_r[i] = (R)(w - (r < NP ? a.U0[0] : (r >= 4 * NP ? a.U0[4] : 0.0)));
        } else {
          __builtin_nontemporal_store(w, ep.out + i);
        }
      }
    }
  }
}

// BF16 bits of a float, round to nearest even (host)
inline uint16_t host_bf16(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  b += 0x7fffu + ((b >> 16) & 1u);
  return (uint16_t)(b >> 16);
}
inline float host_from_bf16(uint16_t h) {
  uint32_t b = (uint32_t)h << 16;
  float x;
  std::memcpy(&x, &b, 4);
  return x;
}

// Split operators of the BF16x3 path from the operator table: the gradient
// operator D - (Mc0 Lend0^T + Mc1 Lend1^T) / 2 (the correction of the
// auxiliary gradient by the common solution, regrouped) and the divergence
// operator M, each rounded to FP32 and split into hi + lo BF16.
template <int N>
NsSplitOps<N> make_split_ops(const double *t) {
  const OpsLayout O = ops_layout(N);
  NsSplitOps<N> s{};
  auto put = [](uint16_t *hi, uint16_t *lo, double v) {
    float f = (float)v;
    *hi = host_bf16(f);
    *lo = host_bf16(f - host_from_bf16(*hi));
  };
  for (int i = 0; i < N; ++i) {
    for (int c = 0; c < N; ++c) {
      double a = t[O.D + i * N + c] - 0.5 * (t[O.Mc + i] * t[O.Lend + c] + t[O.Mc + N + i] * t[O.Lend + N + c]);
      put(&s.Ahi[i][c], &s.Alo[i][c], a);
    }
    for (int c = 0; c <= N; ++c) put(&s.Mhi[i][c], &s.Mlo[i][c], t[O.M + i * (N + 1) + c]);
  }
  return s;
}

// Operators of the FP32 matrix-core variant: the gradient operator
// A = D - (Mc0 Lend0^T + Mc1 Lend1^T)/2 with the neighbour-trace columns
// Mc0/2, Mc1/2 appended, and the divergence operator M, rounded to FP32.
template <int N>
NsF32Ops<N> make_f32_ops(const double *t) {
  const OpsLayout O = ops_layout(N);
  NsF32Ops<N> f{};
  for (int i = 0; i < N; ++i) {
    for (int c = 0; c < N; ++c)
      f.G[i][c] = (float)(t[O.D + i * N + c] - 0.5 * (t[O.Mc + i] * t[O.Lend + c] + t[O.Mc + N + i] * t[O.Lend + N + c]));
    f.G[i][N] = (float)(0.5 * t[O.Mc + i]);
    f.G[i][N + 1] = (float)(0.5 * t[O.Mc + N + i]);
    for (int c = 0; c <= N; ++c) f.D[i][c] = (float)t[O.M + i * (N + 1) + c];
  }
  return f;
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
  op.kapx[0] = (R)t[O.kapx];
  op.kapx[1] = (R)t[O.kapx + 1];
  for (int i = 0; i < N; ++i) {
    for (int c = 0; c < N; ++c)
      op.A[i][c] = (R)(t[O.D + i * N + c] - 0.5 * (t[O.Mc + i] * t[O.Lend + c] + t[O.Mc + N + i] * t[O.Lend + N + c]));
    op.hMc[0][i] = (R)(0.5 * t[O.Mc + i]);
    op.hMc[1][i] = (R)(0.5 * t[O.Mc + N + i]);
  }
  return op;
}

}  // namespace sd
