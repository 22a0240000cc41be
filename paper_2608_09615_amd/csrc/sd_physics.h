// Pointwise flux laws evaluated on the device (section 4.4 and eq. pme).
//
// States may carry a subtracted constant reference state U0 = (rho0, 0, 0, 0,
// p0/(gamma-1)); every Navier-Stokes flux returned here has the constant flux
// F_c(U0) = (0, p0 e_d, 0) removed, which leaves the divergence unchanged (M
// annihilates constants) and keeps FP32 evaluation away from the large
// constant part of the pressure at low Mach number.
#pragma once

#include "sd_internal.h"

namespace sd {

template <typename R>
struct NsConst {
  R gm1, rho0, rE0, p0, mu0, T0inv, S, onepS, lam_over_mu, cp_over_pr, efix;
  int suth;
  __device__ explicit NsConst(const KArgs &a)
      : gm1((R)a.gm1), rho0((R)a.rho0_ref), rE0((R)a.rE0_ref), p0((R)a.p0_ref), mu0((R)a.mu0),
        T0inv((R)a.T0inv), S((R)a.suth_s), onepS((R)(1.0 + a.suth_s)),
        lam_over_mu((R)a.lam_over_mu), cp_over_pr((R)a.cp_over_pr), efix((R)a.efix), suth(a.suth) {}
};

// Reciprocal and square root: exact in FP64; the single-instruction
// v_rcp_f32 / v_sqrt_f32 (about 1 ulp) in FP32, whose error sits far below
// the FP32 path's tolerance.
template <typename R>
__device__ __forceinline__ R frcp(R x) { return R(1) / x; }
template <>
__device__ __forceinline__ float frcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <typename R>
__device__ __forceinline__ R fsqrt(R x) { return sqrt(x); }
template <>
__device__ __forceinline__ float fsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }

// Component d of a 3-vector without runtime indexing of a private array
// (which would put the array in scratch memory).
template <typename R>
__device__ __forceinline__ R pick(int d, R a0, R a1, R a2) {
  return d == 0 ? a0 : (d == 1 ? a1 : a2);
}

// Primitive quantities of a (reference-shifted) conservative state.
template <typename R>
struct Prim {
  R rho, inv, u[3], dp, p, rhoE;
};

template <typename R>
__device__ __forceinline__ Prim<R> ns_prim(const NsConst<R> &c, const R *U) {
  Prim<R> s;
  s.rho = c.rho0 + U[0];
  s.inv = frcp(s.rho);
  s.u[0] = U[1] * s.inv;
  s.u[1] = U[2] * s.inv;
  s.u[2] = U[3] * s.inv;
  R q2 = s.u[0] * s.u[0] + s.u[1] * s.u[1] + s.u[2] * s.u[2];
  s.dp = c.gm1 * (U[4] - R(0.5) * s.rho * q2);
  s.p = c.p0 + s.dp;
  s.rhoE = c.rE0 + U[4];
  return s;
}

// F_c e_d - F_c(U0) e_d
template <typename R>
__device__ __forceinline__ void ns_conv(const NsConst<R> &c, const R *U, const Prim<R> &s, int d, R *F) {
  R ud = pick(d, s.u[0], s.u[1], s.u[2]);
  F[0] = pick(d, U[1], U[2], U[3]);
#pragma unroll
  for (int i = 0; i < 3; ++i) F[1 + i] = U[1 + i] * ud + (i == d ? s.dp : R(0));
  F[4] = (s.rhoE + s.p) * ud;
}

// F_v e_d from the state and the conservative gradient G[m*5 + v]
template <typename R>
__device__ __forceinline__ void ns_visc(const NsConst<R> &c, const Prim<R> &s, const R *G, int d, R *F) {
  R E = s.rhoE * s.inv;
  R du[3][3], dT[3];
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    R drho = G[m * 5 + 0];
#pragma unroll
    for (int i = 0; i < 3; ++i) du[i][m] = (G[m * 5 + 1 + i] - s.u[i] * drho) * s.inv;
    R dE = (G[m * 5 + 4] - E * drho) * s.inv;
    dT[m] = c.gm1 * (dE - (s.u[0] * du[0][m] + s.u[1] * du[1][m] + s.u[2] * du[2][m]));
  }
  R T = s.p * s.inv;
  R mu = c.mu0;
  if (c.suth) {
    R th = T * c.T0inv;
    mu = c.mu0 * th * fsqrt(th) * c.onepS * frcp(th + c.S);
  }
  R lam = c.lam_over_mu * mu;
  R kappa = c.cp_over_pr * mu;
  R div = du[0][0] + du[1][1] + du[2][2];
  R tau[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    R dud = pick(d, du[i][0], du[i][1], du[i][2]);   // d u_i / d x_d
    R ddu = pick(d, du[0][i], du[1][i], du[2][i]);   // d u_d / d x_i
    tau[i] = mu * (dud + ddu) + (i == d ? lam * div : R(0));
  }
  F[0] = R(0);
  F[1] = tau[0];
  F[2] = tau[1];
  F[3] = tau[2];
  F[4] = s.u[0] * tau[0] + s.u[1] * tau[1] + s.u[2] * tau[2] + kappa * pick(d, dT[0], dT[1], dT[2]);
}

// Roe flux along e_d with Harten's fix on the acoustic waves, minus F_c(U0).
template <typename R>
__device__ __forceinline__ void ns_roe(const NsConst<R> &c, const R *UL, const R *UR, int d, R *F) {
  Prim<R> L = ns_prim(c, UL), Rr = ns_prim(c, UR);
  R FL[5], FR[5];
  ns_conv(c, UL, L, d, FL);
  ns_conv(c, UR, Rr, d, FR);
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
  R un = pick(d, ut[0], ut[1], ut[2]);
  R du[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) du[i] = Rr.u[i] - L.u[i];
  R drho = Rr.rho - L.rho, dpj = Rr.dp - L.dp, dun = pick(d, du[0], du[1], du[2]);
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
  for (int i = 0; i < 3; ++i) dut[i] = i == d ? R(0) : du[i];
  R w1 = l1 * a1, w5 = l5 * a5, w2 = l2 * a2, ws = l2 * rt;
  R D[5];
  D[0] = w1 + w2 + w5;
#pragma unroll
  for (int i = 0; i < 3; ++i) D[1 + i] = (w1 + w5 + w2) * ut[i] + ws * dut[i] + (i == d ? (w5 - w1) * cs : R(0));
  D[4] = w1 * (Ht - cs * un) + w5 * (Ht + cs * un) + w2 * R(0.5) * q2 +
         ws * (ut[0] * dut[0] + ut[1] * dut[1] + ut[2] * dut[2]);
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = R(0.5) * (FL[k] + FR[k]) - R(0.5) * D[k];
}

// u^k for a small non-negative integer k
template <typename R>
__device__ __forceinline__ R ipow_r(R u, int k) {
  R r = R(1);
  for (int i = 0; i < k; ++i) r *= u;
  return r;
}

// Physical flux along d at an interior flux point: U[NV], G[m*NV + v].
template <int PHYS, int NV, typename R>
__device__ __forceinline__ void interior_flux(const KArgs &a, int d, const R *U, const R *G, R *F) {
  if constexpr (PHYS == PHYS_NS) {
    NsConst<R> c(a);
    Prim<R> s = ns_prim(c, U);
    R Fc[5], Fv[5];
    ns_conv(c, U, s, d, Fc);
    ns_visc(c, s, G, d, Fv);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = Fc[k] - Fv[k];
  } else if constexpr (PHYS == PHYS_PME) {
    F[0] = -(R)a.pme_m * ipow_r(U[0], a.pme_m - 1) * G[d];
  } else {
    F[0] = -(R)a.nu * G[d];
  }
  (void)NV;
}

// Interface flux along d: Roe on the two traces minus the viscous flux of
// the averaged solution and gradient (option (a)), or the scalar law on
// (u_hat, v_hat).
template <int PHYS, int NV, typename R>
__device__ __forceinline__ void face_flux(const KArgs &a, int d, const R *UL, const R *UR, const R *Uh,
                                          const R *Vh, R *F) {
  if constexpr (PHYS == PHYS_NS) {
    NsConst<R> c(a);
    R Fr[5], Fv[5];
    ns_roe(c, UL, UR, d, Fr);
    Prim<R> s = ns_prim(c, Uh);
    ns_visc(c, s, Vh, d, Fv);
#pragma unroll
    for (int k = 0; k < 5; ++k) F[k] = Fr[k] - Fv[k];
  } else {
    interior_flux<PHYS, NV, R>(a, d, Uh, Vh, F);
  }
}

}  // namespace sd
