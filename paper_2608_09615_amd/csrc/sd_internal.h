// Internal declarations of the SD library (host and device).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace sd {

constexpr int kMaxN = 9;           // n = p + 1 <= 9

// Reference-element operators in FP64 (host), section 2.1.
struct HostOps {
  int n;
  double xs[kMaxN], ws[kMaxN], xf[kMaxN + 1];
  double L[(kMaxN + 1) * kMaxN];   // (n+1) x n, L_ij = l_j(xf_i)
  double M[kMaxN * (kMaxN + 1)];   // n x (n+1), M_ij = l'_{j-1/2}(xs_i)
};

// Builds HostOps for degree p; returns 0 on success.
int build_host_ops(int p, HostOps *o);

// Offsets of the device operator table (one table per precision).
struct OpsLayout {
  int Lend;   // [2][n]      rows 0 and n of L (face interpolation)
  int Lint;   // [n-1][n]    interior rows 1..n-1 of L
  int D;      // [n][n]      M L: derivative at the solution points
  int M;      // [n][n+1]    flux-point to solution-point derivative
  int Mc;     // [2][n]      columns 0 and n of M (interface lifting)
  int rrow;   // [2][n]      normal-gradient face row (scheme dependent)
  int kap;    // [2]         (L M)[end_s][end_s]
  int kapx;   // [2]         (L M)[end_s][end_other]
  int ws;     // [n]         Gauss weights
  int total;
};

__host__ __device__ constexpr OpsLayout ops_layout(int n) {
  OpsLayout o{};
  int c = 0;
  o.Lend = c; c += 2 * n;
  o.Lint = c; c += (n - 1) * n;
  o.D = c; c += n * n;
  o.M = c; c += n * (n + 1);
  o.Mc = c; c += 2 * n;
  o.rrow = c; c += 2 * n;
  o.kap = c; c += 2;
  o.kapx = c; c += 2;
  o.ws = c; c += n;
  o.total = c;
  return o;
}

enum Phys { PHYS_DIFF = 0, PHYS_PME = 1, PHYS_NS = 2 };

// Kernel arguments shared by every launch of a context.
struct KArgs {
  long long ne;          // number of elements
  int nel[3];            // elements per direction (1 for unused directions)
  int epb;               // elements per block
  double two_over_h[3];  // 2 / h_d  (= J^-1 S_dd for the affine hexahedron)
  double nu;             // diffusion coefficient
  int pme_m;             // porous-medium exponent
  // Navier-Stokes constants (reference state removed when ref_state is on)
  double gm1;            // gamma - 1
  double rho0_ref;       // rho of the subtracted state (0 when off)
  double rE0_ref;        // rho E of the subtracted state
  double p0_ref;         // pressure of the subtracted state
  double mu0, T0inv, suth_s;
  int suth;              // 1: Sutherland, 0: constant mu
  double lam_over_mu;
  double cp_over_pr;     // kappa / mu = gamma / ((gamma - 1) Pr), R = 1
  double efix;           // Harten coefficient
  double U0[5];          // subtracted constant state per variable
  double tau[3];         // interior penalty eta_ip (p+1)^2 / h_d (0: off)
};

// Face / edge bookkeeping of the trace buffer (per element, in elements of
// the compute type): faces f = 2 d + s each hold T[nv][n^(dim-1)] and
// NN[nv][n^(dim-1)], then (3-D) 12 edges of nv x n values.
__host__ __device__ constexpr int ipow_c(int b, int e) { return e == 0 ? 1 : b * ipow_c(b, e - 1); }
__host__ __device__ constexpr int trace_face_stride(int dim, int n, int nv) { return 2 * nv * ipow_c(n, dim - 1); }
__host__ __device__ constexpr int trace_edge_off(int dim, int n, int nv) { return 2 * dim * trace_face_stride(dim, n, nv); }
__host__ __device__ constexpr int trace_stride(int dim, int n, int nv) {
  return trace_edge_off(dim, n, nv) + (dim == 3 ? 12 * nv * n : 0);
}

}  // namespace sd
