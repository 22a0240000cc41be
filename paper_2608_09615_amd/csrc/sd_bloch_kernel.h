// Temporal (Bloch) eigenanalysis of the 1-D SD diffusion operator (section 3)
// and the combined-mode analysis of the appendix, batched over wavenumbers.
//
// For a Bloch wave u_e = z^e u_0, z = exp(i theta), on a uniform periodic
// mesh, the semi-discrete diffusion operator (unit coefficient) acts on the
// n solution values of one element as an n x n complex matrix B(theta).
// Column c of B is the right-hand side of the element for u_0 = e_c, built
// here with the same steps as the solver's 1-D right-hand side (traces,
// common solution, auxiliary gradient, face gradients, common gradient with
// the optional interior penalty, fluxes and divergence), every neighbour
// quantity being z^{+-1} times the element's own.
//
// n >= 5: one block of 64 lanes (one wavefront) handles one theta at a time:
// the matrices live in LDS, lanes run over matrix entries, and every branch
// depends only on LDS values that all lanes read alike, so the block's
// barriers are reached uniformly.  n <= 4: one lane per theta (B and its
// eigenvalues) or per (theta, t) pair (combined mode) with the matrices in
// registers (k_bloch_lane_eig, k_bloch_lane_cm, at the end of this file).
#pragma once

namespace sd {

struct cplx {
  double re, im;
};
__device__ __forceinline__ cplx cx(double r, double i = 0.0) { return cplx{r, i}; }
__device__ __forceinline__ cplx operator+(cplx a, cplx b) { return cplx{a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ cplx operator-(cplx a, cplx b) { return cplx{a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ cplx operator*(cplx a, cplx b) {
  return cplx{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
__device__ __forceinline__ cplx operator*(double s, cplx a) { return cplx{s * a.re, s * a.im}; }
__device__ __forceinline__ cplx conjg(cplx a) { return cplx{a.re, -a.im}; }
// acc + a b as four fused multiply-adds
__device__ __forceinline__ cplx cfma(cplx a, cplx b, cplx acc) {
  return cplx{fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
__device__ __forceinline__ double cabs2(cplx a) { return a.re * a.re + a.im * a.im; }
__device__ __forceinline__ double cabs(cplx a) { return hypot(a.re, a.im); }
__device__ __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm: no overflow for large |b|
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return cplx{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  double r = b.re / b.im, d = b.im + b.re * r;
  return cplx{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}
__device__ __forceinline__ cplx csqrt_(cplx a) {
  // principal square root
  double m = cabs(a);
  if (m == 0.0) return cplx{0.0, 0.0};
  double r = sqrt(0.5 * (m + fabs(a.re)));
  if (a.re >= 0.0) return cplx{r, 0.5 * a.im / r};
  return cplx{0.5 * fabs(a.im) / r, a.im >= 0.0 ? r : -r};
}

// Operators of one degree, passed by value (kernel arguments).
template <int N>
struct BlochOps {
  double Lend[2][N];        // face rows of L
  double Lint[N - 1][N];    // interior rows of L
  double D[N][N];           // M L
  double M[N][N + 1];       // flux-point to solution-point derivative
  double Mc[2][N];          // columns 0 and n of M
  double rrow[2][N];        // face row of L M (L u with the face ends replaced)
  double kap[2], kapx[2];   // (L M)[end_s][end_s], (L M)[end_s][end_other]
  double xs[N];             // solution points on [-1, 1]
  double inv_J;             // 1 / J = 2 / h
  double tau;               // interior penalty eta (p+1)^2 / h, 0 when off
  int br1;                  // 1: standard BR1 gradient, 0: compact
};

template <int N>
struct BlochSmem {
  cplx A[N * N];   // B(theta), row-major
  cplx H[N * N];   // Hessenberg / Schur work
  cplx X[N * N];   // exponential work: scaled B t, Taylor sum, squares
  cplx Y[N * N];
  cplx v[N];       // Householder vector
  cplx u0[N];      // Fourier mode at the solution points
  cplx w[N];
  cplx lam[N];
  cplx rot_s[N];   // Givens rotations of one QR sweep
  double rot_c[N];
  cplx mu;
  double scal;
  int lo, hi, iters, sq;
};

// Column c of B(theta) (lane c < N).
template <int N>
__device__ __forceinline__ void bloch_column(const BlochOps<N> &o, cplx z, int c, cplx *A) {
  const cplx zi = conjg(z);
  const double T0 = o.Lend[0][c], T1 = o.Lend[1][c];
  // common solution at the left face (left neighbour's right trace z^-1 T1)
  // and at the right face (right neighbour's left trace z T0)
  const cplx uh0 = 0.5 * (zi * cx(T1) + cx(T0));
  const cplx uh1 = 0.5 * (cx(T1) + z * cx(T0));
  // standard auxiliary gradient at the solution points
  cplx g[N];
#pragma unroll
  for (int i = 0; i < N; ++i)
    g[i] = o.inv_J * (cx(o.D[i][c]) + o.Mc[0][i] * (uh0 - cx(T0)) + o.Mc[1][i] * (uh1 - cx(T1)));
  // face rows: own normal gradient (L M u^F)[end_s] with u^F's face ends
  // replaced by the common solution (compact: only face s; BR1: both)
  cplx nn0 = cx(o.rrow[0][c]), nn1 = cx(o.rrow[1][c]);
  if (o.br1) {
    nn0 = nn0 + o.kapx[0] * uh1;
    nn1 = nn1 + o.kapx[1] * uh0;
  }
  // common gradient at the faces: average of the two one-sided values
  // (the neighbour's row is z^-+1 times the element's own), plus the penalty
  const cplx vo0 = o.inv_J * (nn0 + o.kap[0] * uh0), vn0 = o.inv_J * (zi * nn1 + o.kap[1] * uh0);
  const cplx vo1 = o.inv_J * (nn1 + o.kap[1] * uh1), vn1 = o.inv_J * (z * nn0 + o.kap[0] * uh1);
  const cplx vh0 = 0.5 * (vn0 + vo0) + o.tau * (cx(T0) - zi * cx(T1));
  const cplx vh1 = 0.5 * (vo1 + vn1) + o.tau * (z * cx(T0) - cx(T1));
  // flux points: common gradient at the faces, interpolated gradient inside;
  // du/dt = (1/J) M v  (the diffusive flux is -v, the divergence -(1/J) M F)
  cplx F[N + 1];
  F[0] = vh0;
  F[N] = vh1;
#pragma unroll
  for (int r = 1; r < N; ++r) {
    cplx acc = cx(0.0);
#pragma unroll
    for (int i = 0; i < N; ++i) acc = acc + o.Lint[r - 1][i] * g[i];
    F[r] = acc;
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cplx acc = cx(0.0);
#pragma unroll
    for (int r = 0; r <= N; ++r) acc = acc + o.M[i][r] * F[r];
    A[i * N + c] = o.inv_J * acc;
  }
}

// Eigenvalues of A (copied to H): Householder reduction to Hessenberg form,
// then single-shift complex QR with Wilkinson shifts and deflation on the
// active window.  Returns with s.lam[0..N) filled (NaN if not converged).
template <int N>
__device__ void bloch_eigs(BlochSmem<N> &s, int lane) {
  cplx *H = s.H;
  for (int e = lane; e < N * N; e += 64) H[e] = s.A[e];
  __syncthreads();
  for (int k = 0; k + 2 < N; ++k) {
    // reflector I - 2 v v^H taking H[k+1.., k] onto a multiple of e_1
    if (lane == 0) {
      double nx = 0.0;
      for (int i = k + 1; i < N; ++i) nx += cabs2(H[i * N + k]);
      nx = sqrt(nx);
      double tail = 0.0;
      for (int i = k + 2; i < N; ++i) tail += cabs2(H[i * N + k]);
      s.scal = 0.0;
      if (tail > 0.0) {
        cplx x0 = H[(k + 1) * N + k];
        double a0 = cabs(x0);
        cplx ph = a0 > 0.0 ? cplx{x0.re / a0, x0.im / a0} : cx(1.0);
        // v = x + e^{i arg x0} |x| e_1, then normalised
        for (int i = 0; i < N; ++i) s.v[i] = cx(0.0);
        s.v[k + 1] = x0 + nx * ph;
        for (int i = k + 2; i < N; ++i) s.v[i] = H[i * N + k];
        double nv = 0.0;
        for (int i = k + 1; i < N; ++i) nv += cabs2(s.v[i]);
        nv = 1.0 / sqrt(nv);
        for (int i = k + 1; i < N; ++i) s.v[i] = nv * s.v[i];
        s.scal = 1.0;
      }
    }
    __syncthreads();
    const bool skip = s.scal == 0.0;
    __syncthreads();   // every lane has read the flag before it is rewritten
    if (skip) continue;
    // left: H <- H - 2 v (v^H H), columns j
    if (lane < N) {
      cplx acc = cx(0.0);
      for (int i = k + 1; i < N; ++i) acc = acc + conjg(s.v[i]) * H[i * N + lane];
      s.w[lane] = acc;
    }
    __syncthreads();
    for (int e = lane; e < N * N; e += 64) {
      int i = e / N, j = e % N;
      if (i > k) H[e] = H[e] - 2.0 * (s.v[i] * s.w[j]);
    }
    __syncthreads();
    // right: H <- H - 2 (H v) v^H, rows i
    if (lane < N) {
      cplx acc = cx(0.0);
      for (int j = k + 1; j < N; ++j) acc = acc + H[lane * N + j] * s.v[j];
      s.w[lane] = acc;
    }
    __syncthreads();
    for (int e = lane; e < N * N; e += 64) {
      int i = e / N, j = e % N;
      if (j > k) H[e] = H[e] - 2.0 * (s.w[i] * conjg(s.v[j]));
    }
    __syncthreads();
  }
  // clear what the reduction leaves below the subdiagonal (rounding only)
  for (int e = lane; e < N * N; e += 64)
    if (e / N > e % N + 1) H[e] = cx(0.0);
  if (lane == 0) {
    s.hi = N - 1;
    s.iters = 0;
  }
  __syncthreads();
  const double eps = 2.220446049250313e-16;
  const int max_iters = 60 * N;
  while (true) {
    if (lane == 0) {
      // deflation: the lowest negligible subdiagonal in the window
      int hi = s.hi, l = hi;
      while (l > 0) {
        double d = cabs(H[(l - 1) * N + l - 1]) + cabs(H[l * N + l]);
        if (cabs(H[l * N + l - 1]) <= eps * d) {
          H[l * N + l - 1] = cx(0.0);
          break;
        }
        --l;
      }
      s.lo = l;
      if (l == hi) {
        s.lam[hi] = H[hi * N + hi];
        s.hi = hi - 1;
        s.iters = 0;
      } else {
        // Wilkinson shift: eigenvalue of the trailing 2 x 2 nearer H[hi][hi]
        // (an exceptional shift every tenth iteration breaks cycles)
        cplx a = H[(hi - 1) * N + hi - 1], b = H[(hi - 1) * N + hi], c = H[hi * N + hi - 1], d = H[hi * N + hi];
        cplx mu;
        if (s.iters % 10 == 9) {
          mu = d + cx(0.75 * cabs(c), 0.0);
        } else {
          cplx tr2 = 0.5 * (a + d);
          cplx disc = csqrt_(0.25 * ((a - d) * (a - d)) + b * c);
          cplx m1 = tr2 + disc, m2 = tr2 - disc;
          mu = cabs2(m1 - d) <= cabs2(m2 - d) ? m1 : m2;
        }
        s.mu = mu;
        ++s.iters;
      }
    }
    __syncthreads();
    const int lo = s.lo, hi = s.hi, iters = s.iters;
    const cplx mu = s.mu;
    __syncthreads();   // every lane has read the window before lane 0 moves it
    if (hi < 0) break;
    if (lo > hi || iters == 0) continue;  // deflated: look again
    if (iters > max_iters) {
      if (lane == 0)
        for (int i = 0; i <= hi; ++i) s.lam[i] = cx(__builtin_nan(""), __builtin_nan(""));
      __syncthreads();
      break;
    }
    for (int e = lane; e <= hi - lo; e += 64) H[(lo + e) * N + lo + e] = H[(lo + e) * N + lo + e] - mu;
    __syncthreads();
    // QR of the shifted window by Givens rotations G_k acting on rows k, k+1
    for (int k = lo; k < hi; ++k) {
      if (lane == 0) {
        cplx x = H[k * N + k], y = H[(k + 1) * N + k];
        double r = sqrt(cabs2(x) + cabs2(y));
        double cc;
        cplx sn;
        if (r == 0.0) {
          cc = 1.0;
          sn = cx(0.0);
        } else {
          // [c s; -conj(s) c] [x; y] = [r'; 0] with c real
          double ax = cabs(x);
          if (ax == 0.0) {
            cc = 0.0;
            sn = cdiv(conjg(y), cx(cabs(y)));
          } else {
            cc = ax / r;
            cplx ph = cplx{x.re / ax, x.im / ax};
            sn = (1.0 / r) * (ph * conjg(y));
          }
        }
        s.rot_c[k] = cc;
        s.rot_s[k] = sn;
      }
      __syncthreads();
      const double cc = s.rot_c[k];
      const cplx sn = s.rot_s[k];
      for (int j = k + lane; j <= hi; j += 64) {
        cplx x = H[k * N + j], y = H[(k + 1) * N + j];
        H[k * N + j] = cc * x + sn * y;
        H[(k + 1) * N + j] = cc * y - conjg(sn) * x;
      }
      __syncthreads();
    }
    // R Q: the same rotations applied to columns k, k+1 from the right
    for (int k = lo; k < hi; ++k) {
      const double cc = s.rot_c[k];
      const cplx sn = s.rot_s[k];
      const int top = k + 2 < hi ? k + 2 : hi;
      for (int i = lo + lane; i <= top; i += 64) {
        cplx x = H[i * N + k], y = H[i * N + k + 1];
        H[i * N + k] = cc * x + conjg(sn) * y;
        H[i * N + k + 1] = cc * y - sn * x;
      }
      __syncthreads();
    }
    for (int e = lane; e <= hi - lo; e += 64) H[(lo + e) * N + lo + e] = H[(lo + e) * N + lo + e] + mu;
    __syncthreads();
  }
  // order: real part descending (least damped first), then imaginary part
  if (lane == 0) {
    for (int i = 1; i < N; ++i) {
      cplx x = s.lam[i];
      int j = i - 1;
      while (j >= 0 && (s.lam[j].re < x.re || (s.lam[j].re == x.re && s.lam[j].im > x.im))) {
        s.lam[j + 1] = s.lam[j];
        --j;
      }
      s.lam[j + 1] = x;
    }
  }
  __syncthreads();
}

// C = P Q on N x N matrices in LDS (lanes over entries).
template <int N>
__device__ __forceinline__ void cmatmul(const cplx *P, const cplx *Q, cplx *C, int lane) {
  cplx out[(N * N + 63) / 64];
#pragma unroll
  for (int r = 0; r < (N * N + 63) / 64; ++r) {
    int e = lane + 64 * r;
    cplx acc = cx(0.0);
    if (e < N * N) {
      int i = e / N, j = e % N;
#pragma unroll
      for (int k = 0; k < N; ++k) acc = cfma(P[i * N + k], Q[k * N + j], acc);
    }
    out[r] = acc;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < (N * N + 63) / 64; ++r) {
    int e = lane + 64 * r;
    if (e < N * N) C[e] = out[r];
  }
  __syncthreads();
}

// Combined mode for one t: u(t) = exp(B t) u0 by scaling and squaring of a
// degree-18 Taylor polynomial (||B t / 2^s||_1 <= 1/2), G = u0^H u(t) /
// u0^H u0, omega = (i / t) log G.  u0 is in s.u0.
template <int N>
__device__ void bloch_combined(BlochSmem<N> &s, double t, int lane, cplx &G, cplx &om) {
  if (lane == 0) {
    double nrm = 0.0;
    for (int j = 0; j < N; ++j) {
      double cs = 0.0;
      for (int i = 0; i < N; ++i) cs += cabs(s.A[i * N + j]);
      nrm = fmax(nrm, cs);
    }
    nrm *= t;
    int sq = 0;
    while (nrm > 0.5 && sq < 1000) {
      nrm *= 0.5;
      ++sq;
    }
    s.sq = sq;
    s.scal = ldexp(t, -sq);
  }
  __syncthreads();
  const double sc = s.scal;
  const int sq = s.sq;
  // X = (B t / 2^s); Horner: Y = I + X/m (I + X/(m-1) (... (I + X/1)))
  constexpr int kDeg = 18;
  for (int e = lane; e < N * N; e += 64) {
    s.X[e] = sc * s.A[e];
    s.Y[e] = cx(e / N == e % N ? 1.0 : 0.0);
  }
  __syncthreads();
  for (int m = kDeg; m >= 1; --m) {
    cmatmul<N>(s.X, s.Y, s.H, lane);   // H = X Y
    for (int e = lane; e < N * N; e += 64) s.Y[e] = (1.0 / m) * s.H[e] + cx(e / N == e % N ? 1.0 : 0.0);
    __syncthreads();
  }
  for (int q = 0; q < sq; ++q) {
    cmatmul<N>(s.Y, s.Y, s.H, lane);
    for (int e = lane; e < N * N; e += 64) s.Y[e] = s.H[e];
    __syncthreads();
  }
  if (lane == 0) {
    cplx num = cx(0.0);
    double den = 0.0;
    for (int i = 0; i < N; ++i) {
      cplx ui = cx(0.0);
      for (int j = 0; j < N; ++j) ui = ui + s.Y[i * N + j] * s.u0[j];
      num = num + conjg(s.u0[i]) * ui;
      den += cabs2(s.u0[i]);
    }
    G = (1.0 / den) * num;
    // (i / t) (log|G| + i arg G)
    om = cplx{-atan2(G.im, G.re) / t, log(cabs(G)) / t};
  }
  __syncthreads();
}

template <int N>
__global__ void __launch_bounds__(64) k_bloch(BlochOps<N> o, const double *__restrict__ theta, long long ntheta,
                                              const double *__restrict__ tv, int nt, double *__restrict__ Bout,
                                              double *__restrict__ lam_out, double *__restrict__ Gout,
                                              double *__restrict__ om_out) {
  __shared__ BlochSmem<N> s;
  const int lane = threadIdx.x;
  for (long long it = blockIdx.x; it < ntheta; it += gridDim.x) {
    const double th = theta[it];
    const cplx z = cplx{cos(th), sin(th)};
    if (lane < N) {
      bloch_column<N>(o, z, lane, s.A);
      // Fourier mode exp(i k x) at the solution points, k (2J) = theta
      const double ph = 0.5 * th * (o.xs[lane] + 1.0);
      s.u0[lane] = cplx{cos(ph), sin(ph)};
    }
    __syncthreads();
    if (Bout)
      for (int e = lane; e < N * N; e += 64) {
        Bout[(it * N * N + e) * 2] = s.A[e].re;
        Bout[(it * N * N + e) * 2 + 1] = s.A[e].im;
      }
    if (lam_out) {
      bloch_eigs<N>(s, lane);
      if (lane < N) {
        lam_out[(it * N + lane) * 2] = s.lam[lane].re;
        lam_out[(it * N + lane) * 2 + 1] = s.lam[lane].im;
      }
    }
    if (Gout || om_out)
      for (int k = 0; k < nt; ++k) {
        const double t = tv[k];
        cplx G = cx(__builtin_nan(""), __builtin_nan("")), om = G;
        if (t > 0.0 && isfinite(t)) bloch_combined<N>(s, t, lane, G, om);
        if (lane == 0) {
          if (Gout) {
            Gout[(it * nt + k) * 2] = G.re;
            Gout[(it * nt + k) * 2 + 1] = G.im;
          }
          if (om_out) {
            om_out[(it * nt + k) * 2] = om.re;
            om_out[(it * nt + k) * 2 + 1] = om.im;
          }
        }
      }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Small degrees (n <= 4): one lane per theta, every matrix in registers and
// every loop over matrix indices unrolled.  Same arithmetic as above; the QR
// iteration runs on the whole matrix instead of the active window: every
// negligible subdiagonal is set to zero, which makes the rotations across it
// identities, so each diagonal block undergoes its own shifted QR step (the
// shift is taken from the trailing undeflated block).
// ---------------------------------------------------------------------------

template <int N>
__device__ __forceinline__ cplx pick(const cplx (&a)[N * N], int i, int j) {
  cplx r = cx(0.0);
#pragma unroll
  for (int e = 0; e < N * N; ++e)
    if (e == i * N + j) r = a[e];
  return r;
}

template <int N>
__device__ void lane_eigs(const cplx (&A)[N * N], cplx (&lam)[N]) {
  cplx H[N * N];
#pragma unroll
  for (int e = 0; e < N * N; ++e) H[e] = A[e];
  // Householder reduction to Hessenberg form
#pragma unroll
  for (int k = 0; k + 2 < N; ++k) {
    double nx = 0.0, tail = 0.0;
#pragma unroll
    for (int i = k + 1; i < N; ++i) nx += cabs2(H[i * N + k]);
#pragma unroll
    for (int i = k + 2; i < N; ++i) tail += cabs2(H[i * N + k]);
    if (tail > 0.0) {
      nx = sqrt(nx);
      cplx v[N];
      const cplx x0 = H[(k + 1) * N + k];
      const double a0 = cabs(x0);
      const cplx ph = a0 > 0.0 ? cplx{x0.re / a0, x0.im / a0} : cx(1.0);
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = cx(0.0);
      v[k + 1] = x0 + nx * ph;
#pragma unroll
      for (int i = k + 2; i < N; ++i) v[i] = H[i * N + k];
      double nv = 0.0;
#pragma unroll
      for (int i = k + 1; i < N; ++i) nv += cabs2(v[i]);
      nv = 1.0 / sqrt(nv);
#pragma unroll
      for (int i = k + 1; i < N; ++i) v[i] = nv * v[i];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        cplx w = cx(0.0);
#pragma unroll
        for (int i = k + 1; i < N; ++i) w = w + conjg(v[i]) * H[i * N + j];
#pragma unroll
        for (int i = k + 1; i < N; ++i) H[i * N + j] = H[i * N + j] - 2.0 * (v[i] * w);
      }
#pragma unroll
      for (int i = 0; i < N; ++i) {
        cplx w = cx(0.0);
#pragma unroll
        for (int j = k + 1; j < N; ++j) w = w + H[i * N + j] * v[j];
#pragma unroll
        for (int j = k + 1; j < N; ++j) H[i * N + j] = H[i * N + j] - 2.0 * (w * conjg(v[j]));
      }
    }
  }
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j + 1 < i; ++j) H[i * N + j] = cx(0.0);
  const double eps = 2.220446049250313e-16;
  int hi = N - 1, iters = 0;
#pragma unroll
  for (int i = 0; i < N; ++i) lam[i] = cx(__builtin_nan(""), __builtin_nan(""));
  for (int guard = 0; guard < N * (60 * N + 1) && hi >= 0; ++guard) {
    // zero every negligible subdiagonal
#pragma unroll
    for (int l = 1; l < N; ++l) {
      const double d = cabs(H[(l - 1) * N + l - 1]) + cabs(H[l * N + l]);
      if (cabs(H[l * N + l - 1]) <= eps * d) H[l * N + l - 1] = cx(0.0);
    }
    const cplx sub = hi > 0 ? pick<N>(H, hi, hi - 1) : cx(0.0);
    if (sub.re == 0.0 && sub.im == 0.0) {
      const cplx ev = pick<N>(H, hi, hi);
#pragma unroll
      for (int i = 0; i < N; ++i)
        if (i == hi) lam[i] = ev;
      --hi;
      iters = 0;
      continue;
    }
    if (iters >= 60 * N) break;
    cplx mu;
    {
      const cplx a = pick<N>(H, hi - 1, hi - 1), b = pick<N>(H, hi - 1, hi), c = sub, d = pick<N>(H, hi, hi);
      if (iters % 10 == 9) {
        mu = d + cx(0.75 * cabs(c), 0.0);
      } else {
        const cplx tr2 = 0.5 * (a + d);
        const cplx disc = csqrt_(0.25 * ((a - d) * (a - d)) + b * c);
        const cplx m1 = tr2 + disc, m2 = tr2 - disc;
        mu = cabs2(m1 - d) <= cabs2(m2 - d) ? m1 : m2;
      }
    }
    ++iters;
#pragma unroll
    for (int i = 0; i < N; ++i) H[i * N + i] = H[i * N + i] - mu;
    double rc[N];
    cplx rs[N];
#pragma unroll
    for (int k = 0; k + 1 < N; ++k) {
      const cplx x = H[k * N + k], y = H[(k + 1) * N + k];
      const double r = sqrt(cabs2(x) + cabs2(y));
      double cc = 1.0;
      cplx sn = cx(0.0);
      if (r != 0.0) {
        const double ax = cabs(x);
        if (ax == 0.0) {
          cc = 0.0;
          sn = cdiv(conjg(y), cx(cabs(y)));
        } else {
          cc = ax / r;
          sn = (1.0 / r) * (cplx{x.re / ax, x.im / ax} * conjg(y));
        }
      }
      rc[k] = cc;
      rs[k] = sn;
#pragma unroll
      for (int j = k; j < N; ++j) {
        const cplx xj = H[k * N + j], yj = H[(k + 1) * N + j];
        H[k * N + j] = cc * xj + sn * yj;
        H[(k + 1) * N + j] = cc * yj - conjg(sn) * xj;
      }
    }
#pragma unroll
    for (int k = 0; k + 1 < N; ++k) {
#pragma unroll
      for (int i = 0; i <= (k + 1 < N - 1 ? k + 1 : N - 1); ++i) {
        const cplx xi = H[i * N + k], yi = H[i * N + k + 1];
        H[i * N + k] = rc[k] * xi + conjg(rs[k]) * yi;
        H[i * N + k + 1] = rc[k] * yi - rs[k] * xi;
      }
    }
#pragma unroll
    for (int i = 0; i < N; ++i) H[i * N + i] = H[i * N + i] + mu;
  }
  // real part descending, then imaginary part (a sorting network)
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int j = 0; j + 1 < N - i; ++j) {
      const cplx a = lam[j], b = lam[j + 1];
      if (a.re < b.re || (a.re == b.re && a.im > b.im)) {
        lam[j] = b;
        lam[j + 1] = a;
      }
    }
}

// B is built here (about 2 n^3 operations), so that only two matrices
// occupy registers.
template <int N>
__device__ void lane_combined(const BlochOps<N> &o, cplx z, const cplx (&u0)[N], double t, cplx &G, cplx &om) {
  cplx X[N * N], Y[N * N];
#pragma unroll
  for (int c = 0; c < N; ++c) bloch_column<N>(o, z, c, X);
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    double cs = 0.0;
#pragma unroll
    for (int i = 0; i < N; ++i) cs += cabs(X[i * N + j]);
    nrm = fmax(nrm, cs);
  }
  nrm *= t;
  int sq = 0;
  while (nrm > 0.5 && sq < 1000) {
    nrm *= 0.5;
    ++sq;
  }
  const double sc = ldexp(t, -sq);
#pragma unroll
  for (int e = 0; e < N * N; ++e) {
    X[e] = sc * X[e];
    Y[e] = cx(e / N == e % N ? 1.0 : 0.0);
  }
  // Horner, one column at a time: column j of X Y needs only column j of Y
  for (int m = 18; m >= 1; --m) {
    const double inv = 1.0 / m;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      cplx col[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
        cplx acc = cx(0.0);
#pragma unroll
        for (int k = 0; k < N; ++k) acc = cfma(X[i * N + k], Y[k * N + j], acc);
        col[i] = acc;
      }
#pragma unroll
      for (int i = 0; i < N; ++i) Y[i * N + j] = cplx{fma(inv, col[i].re, i == j ? 1.0 : 0.0), inv * col[i].im};
    }
  }
  for (int q = 0; q < sq; ++q) {
#pragma unroll
    for (int e = 0; e < N * N; ++e) {
      const int i = e / N, j = e % N;
      cplx acc = cx(0.0);
#pragma unroll
      for (int k = 0; k < N; ++k) acc = cfma(Y[i * N + k], Y[k * N + j], acc);
      X[e] = acc;
    }
#pragma unroll
    for (int e = 0; e < N * N; ++e) Y[e] = X[e];
  }
  cplx num = cx(0.0);
  double den = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cplx ui = cx(0.0);
#pragma unroll
    for (int j = 0; j < N; ++j) ui = ui + Y[i * N + j] * u0[j];
    num = num + conjg(u0[i]) * ui;
    den += cabs2(u0[i]);
  }
  G = (1.0 / den) * num;
  om = cplx{-atan2(G.im, G.re) / t, log(cabs(G)) / t};
}

// B(theta) and its eigenvalues, one lane per theta
template <int N>
__global__ void __launch_bounds__(256) k_bloch_lane_eig(BlochOps<N> o, const double *__restrict__ theta,
                                                        long long ntheta, double *__restrict__ Bout,
                                                        double *__restrict__ lam_out) {
  const long long it = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (it >= ntheta) return;
  const double th = theta[it];
  const cplx z = cplx{cos(th), sin(th)};
  cplx A[N * N];
#pragma unroll
  for (int c = 0; c < N; ++c) bloch_column<N>(o, z, c, A);
  if (Bout)
#pragma unroll
    for (int e = 0; e < N * N; ++e) {
      Bout[(it * N * N + e) * 2] = A[e].re;
      Bout[(it * N * N + e) * 2 + 1] = A[e].im;
    }
  if (lam_out) {
    cplx lam[N];
    lane_eigs<N>(A, lam);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      lam_out[(it * N + i) * 2] = lam[i].re;
      lam_out[(it * N + i) * 2 + 1] = lam[i].im;
    }
  }
}

// combined mode, one lane per (theta, t) pair (t fastest)
template <int N>
__global__ void __launch_bounds__(256) k_bloch_lane_cm(BlochOps<N> o, const double *__restrict__ theta,
                                                       long long ntheta, const double *__restrict__ tv, int nt,
                                                       double *__restrict__ Gout, double *__restrict__ om_out) {
  const long long id = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= ntheta * nt) return;
  const long long it = id / nt;
  const int k = (int)(id % nt);
  const double th = theta[it], t = tv[k];
  cplx G = cx(__builtin_nan(""), __builtin_nan("")), om = G;
  if (t > 0.0 && isfinite(t)) {
    const cplx z = cplx{cos(th), sin(th)};
    cplx u0[N];
#pragma unroll
    for (int c = 0; c < N; ++c) {
      const double ph = 0.5 * th * (o.xs[c] + 1.0);
      u0[c] = cplx{cos(ph), sin(ph)};
    }
    lane_combined<N>(o, z, u0, t, G, om);
  }
  if (Gout) {
    Gout[id * 2] = G.re;
    Gout[id * 2 + 1] = G.im;
  }
  if (om_out) {
    om_out[id * 2] = om.re;
    om_out[id * 2 + 1] = om.im;
  }
}

}  // namespace sd
