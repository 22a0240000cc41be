// Reference-element operators of the SD method (section 2.1), FP64 host code.
//
// Solution points: n-point Gauss-Legendre rule; flux points: the two element
// ends plus the (n-1)-point Gauss-Legendre rule.  The rules come from the
// eigen-decomposition of the symmetric Jacobi matrix of the Legendre
// recurrence (Golub-Welsch), solved with cyclic Jacobi rotations; the
// interpolation matrix L (eq. Lmat) and differentiation matrix M (eq. Mmat)
// use the barycentric form of the Lagrange bases (eq. lagr:poly).
#include <cmath>
#include <cstring>

#include "sd_internal.h"

namespace sd {
namespace {

// Gauss-Legendre rule of size m: nodes ascending and weights.
void golub_welsch(int m, double *x, double *w) {
  if (m == 1) { x[0] = 0.0; w[0] = 2.0; return; }
  double A[kMaxN][kMaxN] = {};
  double V[kMaxN][kMaxN] = {};
  for (int i = 0; i < m; ++i) V[i][i] = 1.0;
  for (int k = 1; k < m; ++k) {
    double b = k / std::sqrt(4.0 * k * k - 1.0);
    A[k - 1][k] = A[k][k - 1] = b;
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = i + 1; j < m; ++j) off += A[i][j] * A[i][j];
    if (off < 1e-34) break;
    for (int pi = 0; pi < m; ++pi)
      for (int q = pi + 1; q < m; ++q) {
        if (std::fabs(A[pi][q]) < 1e-300) continue;
        double theta = (A[q][q] - A[pi][pi]) / (2.0 * A[pi][q]);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < m; ++k) {  // A <- A G
          double akp = A[k][pi], akq = A[k][q];
          A[k][pi] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {  // A <- G^T A
          double apk = A[pi][k], aqk = A[q][k];
          A[pi][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          double vkp = V[k][pi], vkq = V[k][q];
          V[k][pi] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  int idx[kMaxN];
  for (int i = 0; i < m; ++i) idx[i] = i;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j)
      if (A[idx[j]][idx[j]] < A[idx[i]][idx[i]]) { int t = idx[i]; idx[i] = idx[j]; idx[j] = t; }
  for (int i = 0; i < m; ++i) {
    int k = idx[i];
    double z = A[k][k];
    // one Newton polish on P_m through the Bonnet recurrence
    double p0 = 1.0, p1 = z;
    for (int r = 2; r <= m; ++r) { double p2 = ((2 * r - 1) * z * p1 - (r - 1) * p0) / r; p0 = p1; p1 = p2; }
    double dp = m * (p0 - z * p1) / (1.0 - z * z);
    z -= p1 / dp;
    x[i] = z;
    w[i] = 2.0 * V[0][k] * V[0][k];
  }
  // symmetric rule: enforce exact antisymmetry of the nodes
  for (int i = 0; i < m / 2; ++i) {
    double a = 0.5 * (x[m - 1 - i] - x[i]);
    x[i] = -a; x[m - 1 - i] = a;
    double ww = 0.5 * (w[i] + w[m - 1 - i]);
    w[i] = w[m - 1 - i] = ww;
  }
  if (m % 2 == 1) x[m / 2] = 0.0;
}

// barycentric weights of the node set
void bary_weights(const double *x, int m, double *bw) {
  for (int j = 0; j < m; ++j) {
    double p = 1.0;
    for (int k = 0; k < m; ++k)
      if (k != j) p *= (x[j] - x[k]);
    bw[j] = 1.0 / p;
  }
}

}  // namespace

int build_host_ops(int p, HostOps *o) {
  const int n = p + 1;
  if (p < 1 || n > kMaxN) return -1;
  std::memset(o, 0, sizeof(*o));
  o->n = n;
  golub_welsch(n, o->xs, o->ws);
  double gx[kMaxN], gw[kMaxN];
  golub_welsch(n - 1, gx, gw);
  o->xf[0] = -1.0;
  for (int i = 0; i < n - 1; ++i) o->xf[i + 1] = gx[i];
  o->xf[n] = 1.0;
  // L: basis of the solution points at the flux points (never coincident)
  double bs[kMaxN];
  bary_weights(o->xs, n, bs);
  for (int i = 0; i <= n; ++i) {
    double den = 0.0;
    for (int j = 0; j < n; ++j) den += bs[j] / (o->xf[i] - o->xs[j]);
    for (int j = 0; j < n; ++j) o->L[i * n + j] = (bs[j] / (o->xf[i] - o->xs[j])) / den;
  }
  // M: derivative of the flux-point basis at the solution points, from the
  // quotient rule on the barycentric form N(x)/D(x)
  double bf[kMaxN + 1];
  bary_weights(o->xf, n + 1, bf);
  for (int i = 0; i < n; ++i) {
    double x = o->xs[i];
    double D = 0.0, Dp = 0.0;
    for (int k = 0; k <= n; ++k) {
      double r = 1.0 / (x - o->xf[k]);
      D += bf[k] * r;
      Dp -= bf[k] * r * r;
    }
    for (int j = 0; j <= n; ++j) {
      double r = 1.0 / (x - o->xf[j]);
      double Nj = bf[j] * r, Njp = -bf[j] * r * r;
      o->M[i * (n + 1) + j] = (Njp * D - Nj * Dp) / (D * D);
    }
  }
  return 0;
}

}  // namespace sd
