// Spline, geometry and assembly kernels of the TT-IGA hot path.
//
//  k_basis_tables   - Gauss nodes/weights per knot span and the p+1 non-zero
//                     B-splines and derivatives there (Cox-de Boor recursion and
//                     derivative formula of Section 2.1); also used for the
//                     geometry's own knot vectors.
//  k_factors        - exact NURBS map in homogeneous form (Section 2.3) at each
//                     sample point, Jacobian, det J and the metric factor
//                     R = det J J^-1 J^-T = adj(J) adj(J)^T / det J (eq. Rxi),
//                     plus f(x) det J (eq. ffinal).
//  k_assemble_band  - TT-matrix core of K_ij in mode d (Section 4.2.1):
//                     M[a][k][t][b] = sum_q w_q G[a][q][b] Row_q[k] Col_q[k+t-p],
//                     Row/Col the value or derivative selected by a_ij^(d).
//  k_assemble_vec   - TT core of F (Section 4.2.2): sum_q w_q G[a][q][b] N_k(q).
//  k_slice_*        - removal of Dirichlet indices (Section 4.3).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "iga.hpp"

namespace ttiga {

constexpr int kMaxDeg = 8;

__device__ inline double safe_div(double a, double b) { return b == 0.0 ? 0.0 : a / b; }

// Gauss-Legendre node t (ascending) and weight of the g-point rule on [-1, 1],
// Newton iteration on the Legendre recurrence.
__device__ void gauss_legendre(int g, int t, double* x, double* w) {
  double z = cos(3.141592653589793 * (t + 0.75) / (g + 0.5));
  double dp = 1.0;
  for (int it = 0; it < 100; ++it) {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= g; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (g == 1) { p1 = z; p0 = 1.0; }
    dp = g * (z * p1 - p0) / (z * z - 1.0);
    const double dz = p1 / dp;
    z -= dz;
    if (fabs(dz) < 1e-16) break;
  }
  {
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= g; ++k) {
      const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (g == 1) { p1 = z; p0 = 1.0; }
    dp = g * (z * p1 - p0) / (z * z - 1.0);
  }
  *x = -z;
  *w = 2.0 / ((1.0 - z * z) * dp * dp);
}

// Non-zero basis N_{s-p..s}^p(xi) and derivatives on span s of `knots`.
__device__ void local_basis(const double* knots, int p, int s, double xi, double* N, double* dN) {
  double cur[kMaxDeg + 1], prev[kMaxDeg + 1];
  cur[0] = 1.0;
  for (int q = 1; q <= p; ++q) {
    for (int j = 0; j < q; ++j) prev[j] = cur[j];
    for (int j = 0; j <= q; ++j) {
      const int i = s - q + j;
      double v = 0.0;
      if (j - 1 >= 0) v += safe_div(xi - knots[i], knots[i + q] - knots[i]) * prev[j - 1];
      if (j <= q - 1) v += safe_div(knots[i + q + 1] - xi, knots[i + q + 1] - knots[i + 1]) * prev[j];
      cur[j] = v;
    }
    if (q == p) {
      for (int j = 0; j <= p; ++j) {
        const int i = s - p + j;
        double d = 0.0;
        if (j - 1 >= 0) d += p * safe_div(1.0, knots[i + p] - knots[i]) * prev[j - 1];
        if (j <= p - 1) d -= p * safe_div(1.0, knots[i + p + 1] - knots[i + 1]) * prev[j];
        dN[j] = d;
      }
    }
  }
  if (p == 0) dN[0] = 0.0;
  for (int j = 0; j <= p; ++j) N[j] = cur[j];
}

// Span s with knots[s] <= xi < knots[s+1], s in [p, nb-1]; xi at the right end maps to
// the last non-empty span.
__device__ int find_span(const double* knots, int p, int nb, double xi) {
  if (xi >= knots[nb]) {
    int s = nb - 1;
    while (s > p && knots[s] == knots[s + 1]) --s;
    return s;
  }
  if (xi <= knots[p]) return p;
  int lo = p, hi = nb;  // knots[lo] <= xi < knots[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (knots[mid] <= xi) lo = mid; else hi = mid;
  }
  return lo;
}

// Solution tables: Gauss points of the E = n - p uniform spans (g per span).
__global__ void k_basis_tables(int n, int p, int g, const double* __restrict__ knots,
                               double* __restrict__ xi_out, double* __restrict__ w_out,
                               double* __restrict__ B, double* __restrict__ D) {
  const int E = n - p;
  const int Q = E * g;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= Q) return;
  const int e = q / g, t = q % g;
  double x, w;
  gauss_legendre(g, t, &x, &w);
  const double a = knots[p + e], b = knots[p + e + 1];
  const double xi = 0.5 * (a + b) + 0.5 * (b - a) * x;
  xi_out[q] = xi;
  w_out[q] = 0.5 * (b - a) * w;
  double N[kMaxDeg + 1], dN[kMaxDeg + 1];
  local_basis(knots, p, p + e, xi, N, dN);
  for (int j = 0; j <= p; ++j) {
    B[(long)q * (p + 1) + j] = N[j];
    D[(long)q * (p + 1) + j] = dN[j];
  }
}

// Geometry tables at arbitrary parametric points (span + non-zero basis + derivative).
__global__ void k_geo_tables(int count, const double* __restrict__ xi, int stride, int nb, int pg,
                             const double* __restrict__ knots, int* __restrict__ span,
                             double* __restrict__ B, double* __restrict__ D) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  const double x = xi[(long)q * stride];
  const int s = find_span(knots, pg, nb, x);
  span[q] = s;
  double N[kMaxDeg + 1], dN[kMaxDeg + 1];
  local_basis(knots, pg, s, x, N, dN);
  for (int j = 0; j <= pg; ++j) {
    B[(long)q * (pg + 1) + j] = N[j];
    D[(long)q * (pg + 1) + j] = dN[j];
  }
}

__device__ double source_value(const SourceDev& src, double x, double y, double z) {
  if (src.kind == TTIGA_SOURCE_MANUFACTURED_ANNULUS) {
    const double r = sqrt(x * x + y * y);
    const double th = atan2(y, x);
    const double pi = 3.141592653589793;
    const double radial = (2.0 * pi * pi + 4.0 / (r * r)) * sin(pi * r) - (pi / r) * cos(pi * r);
    return radial * sin(2.0 * th) * sin(pi * z);
  }
  if (src.kind == TTIGA_SOURCE_FOURIER) {
    const double xs = (x - src.origin[0]) / src.scale, ys = (y - src.origin[1]) / src.scale,
                 zs = (z - src.origin[2]) / src.scale;
    double f = 0.0;
    for (int m = 0; m < src.n_modes; ++m) {
      const double* k = src.k + 3 * m;
      f += src.a[m] * sin(3.141592653589793 * (k[0] * xs + k[1] * ys + k[2] * zs) + src.phi[m]);
    }
    return f;
  }
  return 0.0;
}

// Fourier source with integral wave vectors: with u_d = e^{i pi (x_d - o_d) / scale},
// e^{i (pi k.x_hat + phi)} = e^{i phi} prod_d u_d^{k_d}, so three sincos and a few complex
// products replace one sine per mode; the powers come from repeated multiplication (a
// few ulps for |k_d| <= 8).
__device__ double fourier_int(const SourceDev& src, double x, double y, double z, const double* cph,
                              const double* sph) {
  const double is = 1.0 / src.scale;
  const double xs[3] = {(x - src.origin[0]) * is, (y - src.origin[1]) * is, (z - src.origin[2]) * is};
  double ur[3], ui[3];
  for (int d = 0; d < 3; ++d) sincospi(xs[d], &ui[d], &ur[d]);
  double f = 0.0;
  for (int m = 0; m < src.n_modes; ++m) {
    double re = 1.0, im = 0.0;
    for (int d = 0; d < 3; ++d) {
      const int k = (int)src.k[3 * m + d];
      const double si = k < 0 ? -ui[d] : ui[d];
      for (int j = 0; j < (k < 0 ? -k : k); ++j) {
        const double t = re * ur[d] - im * si;
        im = re * si + im * ur[d];
        re = t;
      }
    }
    // sin(theta + phi) = Im(e^{i theta} e^{i phi})
    f += src.a[m] * (im * cph[m] + re * sph[m]);
  }
  return f;
}

__device__ void factors_from_sums(const double H[4], const double dH[3][4], const SourceDev& src,
                                  const double* cph, const double* sph, double* out7, double* det_out);

// det J alone from the homogeneous sums (the quotient rule for J, then the 3 x 3 determinant).
__device__ double jacobian_det(const double H[4], const double dH[3][4]) {
  const double iW = 1.0 / H[3];
  double J[3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) J[k][i] = (dH[i][k] - H[k] * iW * dH[i][3]) * iW;
  return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
         J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

// Homogeneous sums H = (x w, y w, z w, w) of the NURBS map at one sample point and their
// derivatives dH[i] along xi_i.  ia/ib/ic index the per-direction geometry tables.
__device__ void homogeneous_sums(const GeoDev& geo, int ia, int ib, int ic, double H[4], double dH[3][4]) {
  const int p0 = geo.pg[0], p1 = geo.pg[1], p2 = geo.pg[2];
  const int s0 = geo.span[0][ia], s1 = geo.span[1][ib], s2 = geo.span[2][ic];
  const double* B0 = geo.B[0] + (long)ia * (p0 + 1);
  const double* B1 = geo.B[1] + (long)ib * (p1 + 1);
  const double* B2 = geo.B[2] + (long)ic * (p2 + 1);
  const double* D0 = geo.D[0] + (long)ia * (p0 + 1);
  const double* D1 = geo.D[1] + (long)ib * (p1 + 1);
  const double* D2 = geo.D[2] + (long)ic * (p2 + 1);
  for (int s = 0; s < 4; ++s) {
    H[s] = 0.0;
    dH[0][s] = dH[1][s] = dH[2][s] = 0.0;
  }
  for (int a = 0; a <= p0; ++a) {
    for (int b = 0; b <= p1; ++b) {
      // partial sums over c first (sum factorisation of the inner direction)
      double h[4] = {0, 0, 0, 0}, h2[4] = {0, 0, 0, 0};
      const long base = ((long)(s0 - p0 + a) * geo.m[1] + (s1 - p1 + b)) * geo.m[2] + (s2 - p2);
      for (int c = 0; c <= p2; ++c) {
        const double* P = geo.Pw + (base + c) * 4;
        for (int s = 0; s < 4; ++s) {
          h[s] += B2[c] * P[s];
          h2[s] += D2[c] * P[s];
        }
      }
      const double bb = B0[a] * B1[b], db0 = D0[a] * B1[b], db1 = B0[a] * D1[b];
      for (int s = 0; s < 4; ++s) {
        H[s] += bb * h[s];
        dH[0][s] += db0 * h[s];
        dH[1][s] += db1 * h[s];
        dH[2][s] += bb * h2[s];
      }
    }
  }
}

// One sample point: 7 factors and det J.
__device__ void point_factors(const GeoDev& geo, const SourceDev& src, int ia, int ib, int ic,
                              double* out7, double* det_out) {
  double H[4], dH[3][4];
  homogeneous_sums(geo, ia, ib, ic, H, dH);
  factors_from_sums(H, dH, src, nullptr, nullptr, out7, det_out);
}

// Exact solutions against which a computed solution's L2 error is measured (Section 5):
// the manufactured field of the quarter-annulus workload, the radial Laplace solution
// between two coaxial cylinders (the ring experiment of Section 5.2) and the L-shape
// solution of Section 5.1.
__device__ double exact_value(const ExactDev& ex, double x, double y, double z) {
  const double pi = 3.141592653589793;
  const double r = sqrt(x * x + y * y);
  if (ex.kind == TTIGA_EXACT_MANUFACTURED_ANNULUS)
    return sin(pi * r) * sin(2.0 * atan2(y, x)) * sin(pi * z);
  if (ex.kind == TTIGA_EXACT_RADIAL_LOG)
    return (ex.prm[2] * log(ex.prm[1] / r) + ex.prm[3] * log(r / ex.prm[0])) / log(ex.prm[1] / ex.prm[0]);
  if (ex.kind == TTIGA_EXACT_SINE_XY) return sin(pi * x) * sin(pi * y) / (2.0 * pi * pi);
  return 0.0;
}

// Error-grid sampling of the slabs b0 .. b0+c1-1 of the second direction: per point the
// exact solution u(x(xi)) and the physical quadrature weight w0 w1 w2 det J; output
// F[2][Q0][c1][Q2], per-block sums of squares of both (slots 0, 1) and min det J (slot 7)
// to part[block][8].
__global__ __launch_bounds__(256) void k_exact_grid(GeoDev geo, ExactDev ex, const double* __restrict__ w0,
                                                    const double* __restrict__ w1, const double* __restrict__ w2,
                                                    int Q0, int b0, int c1, int Q2, double* __restrict__ F,
                                                    double* __restrict__ part) {
  __shared__ double sh[3][256];
  const long total = (long)Q0 * c1 * Q2;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double acc[3] = {0.0, 0.0, 1e300};
  if (e < total) {
    const int i2 = (int)(e % Q2);
    const int i1 = b0 + (int)((e / Q2) % c1);
    const int i0 = (int)(e / ((long)c1 * Q2));
    double H[4], dH[3][4];
    homogeneous_sums(geo, i0, i1, i2, H, dH);
    const double iW = 1.0 / H[3];
    const double u = exact_value(ex, H[0] * iW, H[1] * iW, H[2] * iW);
    const double det = jacobian_det(H, dH);
    const double wt = w0[i0] * w1[i1] * w2[i2] * det;
    F[e] = u;
    F[total + e] = wt;
    acc[0] = u * u;
    acc[1] = wt * wt;
    acc[2] = det;
  }
  for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
      sh[2][threadIdx.x] = fmin(sh[2][threadIdx.x], sh[2][threadIdx.x + o]);
    }
    __syncthreads();
  }
  // the layout of the factor statistics: sums of squares in slots 0 and 1, min det J in slot 7
  if (threadIdx.x < 8)
    part[(long)blockIdx.x * 8 + threadIdx.x] = threadIdx.x < 2 ? sh[threadIdx.x][0] : (threadIdx.x == 7 ? sh[2][0] : 0.0);
}

// Surface element of a face xi_d = const (geometry tables of direction d hold that one
// point): |dx/dxi_i x dx/dxi_j| at the tangential Gauss points (qi, qj), i < j the other two
// directions; out[qi * Qj + qj].
__global__ void k_surface_jac(GeoDev geo, int d, int Qi, int Qj, double* __restrict__ out) {
  const long total = (long)Qi * Qj;
  const int i = d == 0 ? 1 : 0, j = d == 2 ? 1 : 2;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int qi = (int)(e / Qj), qj = (int)(e % Qj);
    int idx[3];
    idx[d] = 0;
    idx[i] = qi;
    idx[j] = qj;
    double H[4], dH[3][4];
    homogeneous_sums(geo, idx[0], idx[1], idx[2], H, dH);
    const double iW = 1.0 / H[3];
    double ti[3], tj[3];
    for (int k = 0; k < 3; ++k) {
      const double xk = H[k] * iW;
      ti[k] = (dH[i][k] - xk * dH[i][3]) * iW;
      tj[k] = (dH[j][k] - xk * dH[j][3]) * iW;
    }
    const double c0 = ti[1] * tj[2] - ti[2] * tj[1], c1 = ti[2] * tj[0] - ti[0] * tj[2],
                 c2 = ti[0] * tj[1] - ti[1] * tj[0];
    out[e] = sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  }
}

// Grid values of a solution TT: out[a][q][b] = sum_j B[q][j] u[a][(e_q + j) - lo][b] over the
// p+1 B-splines non-zero at error-grid point q (span e_q = q / g), interior indices only.
__global__ void k_eval_core(int ra, int rb, int Q, int g, int p, int lo, int ni, const double* __restrict__ B,
                            const double* __restrict__ U, double* __restrict__ out) {
  const long total = (long)ra * Q * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int b = (int)(e % rb);
    const int q = (int)((e / rb) % Q);
    const int a = (int)(e / ((long)rb * Q));
    const int el = q / g;
    double s = 0.0;
    for (int j = 0; j <= p; ++j) {
      const int k = el + j - lo;
      if (k >= 0 && k < ni) s += B[(long)q * (p + 1) + j] * U[((long)a * ni + k) * rb + b];
    }
    out[e] = s;
  }
}

// The 7 factors and det J at one point from the homogeneous sums H (x w, y w, z w, w)
// and their derivatives dH[i] along xi_i: the quotient rule gives the Jacobian, the
// adjugate gives J^-1 det J, and R = adj adj^T / det J.  cph/sph, when given, hold
// cos and sin of the Fourier phase shifts (integral wave vectors only).
__device__ void factors_from_sums(const double H[4], const double dH[3][4], const SourceDev& src,
                                  const double* cph, const double* sph, double* out7, double* det_out) {
  const double iW = 1.0 / H[3];
  const double x[3] = {H[0] * iW, H[1] * iW, H[2] * iW};
  double J[3][3];
  for (int k = 0; k < 3; ++k)
    for (int i = 0; i < 3; ++i) J[k][i] = (dH[i][k] - x[k] * dH[i][3]) * iW;
  // adjugate (transpose of the cofactor matrix): J^-1 = adj / det
  double A[3][3];
  A[0][0] = J[1][1] * J[2][2] - J[1][2] * J[2][1];
  A[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
  A[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
  A[1][0] = J[1][2] * J[2][0] - J[1][0] * J[2][2];
  A[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
  A[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
  A[2][0] = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  A[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
  A[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
  const double det = J[0][0] * A[0][0] + J[0][1] * A[1][0] + J[0][2] * A[2][0];
  // R = det J^-1 J^-T = adj adj^T / det
  const int pi_[6] = {0, 1, 2, 0, 0, 1}, pj_[6] = {0, 1, 2, 1, 2, 2};
  const double idet = 1.0 / det;
  for (int f = 0; f < 6; ++f) {
    const int i = pi_[f], j = pj_[f];
    out7[f] = (A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2]) * idet;
  }
  const double f = cph ? fourier_int(src, x[0], x[1], x[2], cph, sph) : source_value(src, x[0], x[1], x[2]);
  out7[6] = f * det;
  *det_out = det;
}

// Gauss-grid sampling of the slabs b0 .. b0+c1-1 of the second direction (all of the
// first and third): thread per point (i0, i1, i2), i2 fastest; factor-major output
// F[f][(i0 c1 + i1 - b0) Q2 + i2].  Per-block partial sums of squares of the 7 factors
// and the minimum det J go to part[block][8].
__global__ __launch_bounds__(256) void k_factors_grid(GeoDev geo, SourceDev src, int Q0, int b0,
                                                      int c1, int Q2, double* __restrict__ F,
                                                      double* __restrict__ part) {
  __shared__ double sh[8][256];
  const long total = (long)Q0 * c1 * Q2;
  const long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 1e300};
  if (e < total) {
    const int i2 = e % Q2;
    const int i1 = b0 + (int)((e / Q2) % c1);
    const int i0 = (int)(e / ((long)c1 * Q2));
    double v[7], det;
    point_factors(geo, src, i0, i1, i2, v, &det);
    for (int f = 0; f < 7; ++f) {
      F[(long)f * total + e] = v[f];
      acc[f] = v[f] * v[f];
    }
    acc[7] = det;
  }
  for (int f = 0; f < 8; ++f) sh[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int f = 0; f < 7; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + o];
      sh[7][threadIdx.x] = fmin(sh[7][threadIdx.x], sh[7][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) part[(long)blockIdx.x * 8 + threadIdx.x] = sh[threadIdx.x][0];
}

// Gauss-grid sampling by rows: one block per row (i0, i1) of the slabs b0 .. b0+c1-1 of the
// second direction, threads over i2.  Sum factorisation: the homogeneous net summed over
// the first two directions with B0 B1, D0 B1 and B0 D1 (value and the two in-plane
// derivatives) is formed once per row for every net index of the third direction, so a
// point only needs p_g2+1 terms per sum.  Output and partial statistics as k_factors_grid.
//
// rows0 (optional) lists the first-direction indices to sample (block row r samples
// i0 = rows0[r / c1]).
__global__ __launch_bounds__(256) void k_factors_rows(GeoDev geo, SourceDev src, int b0, int c1, int Q2,
                                                      const int* __restrict__ rows0,
                                                      double* __restrict__ F, double* __restrict__ part) {
  extern __shared__ double T[];  // [3][m2][4]
  __shared__ double cph[kMaxRowModes], sph[kMaxRowModes];
  __shared__ double red[8][4];
  const int row = blockIdx.x;
  const int i0 = rows0 ? rows0[row / c1] : row / c1, i1 = b0 + row % c1;
  const int p0 = geo.pg[0], p1 = geo.pg[1], p2 = geo.pg[2];
  const int m1 = geo.m[1], m2 = geo.m[2];
  const int s0 = geo.span[0][i0], s1 = geo.span[1][i1];
  const double* B0 = geo.B[0] + (long)i0 * (p0 + 1);
  const double* D0 = geo.D[0] + (long)i0 * (p0 + 1);
  const double* B1 = geo.B[1] + (long)i1 * (p1 + 1);
  const double* D1 = geo.D[1] + (long)i1 * (p1 + 1);
  for (int e = threadIdx.x; e < 3 * m2 * 4; e += blockDim.x) {
    const int v = e / (m2 * 4), c = (e / 4) % m2, sc = e % 4;
    double acc = 0.0;
    for (int a = 0; a <= p0; ++a) {
      const double wa = (v == 1) ? D0[a] : B0[a];
      for (int b = 0; b <= p1; ++b) {
        const double wb = (v == 2) ? D1[b] : B1[b];
        acc += wa * wb * geo.Pw[(((long)(s0 - p0 + a) * m1 + (s1 - p1 + b)) * m2 + c) * 4 + sc];
      }
    }
    T[e] = acc;
  }
  const bool fast_src = src.kind == TTIGA_SOURCE_FOURIER && src.int_kmax >= 0 && src.n_modes <= kMaxRowModes;
  if (fast_src)
    for (int m = threadIdx.x; m < src.n_modes; m += blockDim.x) sincos(src.phi[m], &sph[m], &cph[m]);
  __syncthreads();
  const long total = (long)gridDim.x * Q2;
  const long base = (long)row * Q2;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 1e300};
  for (int i2 = threadIdx.x; i2 < Q2; i2 += blockDim.x) {
    const int s2 = geo.span[2][i2];
    const double* B2 = geo.B[2] + (long)i2 * (p2 + 1);
    const double* D2 = geo.D[2] + (long)i2 * (p2 + 1);
    double H[4] = {0, 0, 0, 0}, dH[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
    for (int c = 0; c <= p2; ++c) {
      const int cc = s2 - p2 + c;
      const double* t0 = T + (0 * m2 + cc) * 4;
      const double* t1 = T + (1 * m2 + cc) * 4;
      const double* t2 = T + (2 * m2 + cc) * 4;
      for (int sc = 0; sc < 4; ++sc) {
        H[sc] += B2[c] * t0[sc];
        dH[0][sc] += B2[c] * t1[sc];
        dH[1][sc] += B2[c] * t2[sc];
        dH[2][sc] += D2[c] * t0[sc];
      }
    }
    double v[7], det;
    factors_from_sums(H, dH, src, fast_src ? cph : nullptr, fast_src ? sph : nullptr, v, &det);
    for (int f = 0; f < 7; ++f) {
      F[(long)f * total + base + i2] = v[f];
      acc[f] += v[f] * v[f];
    }
    acc[7] = fmin(acc[7], det);
  }
  // block reduction: within each 64-lane wave by shuffles, then across the waves
  for (int f = 0; f < 8; ++f) {
    double x = acc[f];
    for (int o = 32; o > 0; o >>= 1) {
      const double y = __shfl_xor(x, o, 64);
      x = (f < 7) ? x + y : fmin(x, y);
    }
    acc[f] = x;
  }
  const int wave = threadIdx.x / 64, nw = (blockDim.x + 63) / 64;
  if ((threadIdx.x & 63) == 0)
    for (int f = 0; f < 8; ++f) red[f][wave] = acc[f];
  __syncthreads();
  if (threadIdx.x < 8) {
    double x = red[threadIdx.x][0];
    for (int w = 1; w < nw; ++w) x = (threadIdx.x < 7) ? x + red[threadIdx.x][w] : fmin(x, red[threadIdx.x][w]);
    part[(long)blockIdx.x * 8 + threadIdx.x] = x;
  }
}

// Reduces the per-block partials; with accumulate the result is merged into out
// (sums added, minimum kept), so slabs sampled one chunk after another give one total.
__global__ void k_factors_reduce(const double* __restrict__ part, long blocks, int accumulate,
                                 double* __restrict__ out) {
  __shared__ double sh[8][256];
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 1e300};
  for (long b = threadIdx.x; b < blocks; b += blockDim.x) {
    for (int f = 0; f < 7; ++f) acc[f] += part[b * 8 + f];
    acc[7] = fmin(acc[7], part[b * 8 + 7]);
  }
  for (int f = 0; f < 8; ++f) sh[f][threadIdx.x] = acc[f];
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      for (int f = 0; f < 7; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + o];
      sh[7][threadIdx.x] = fmin(sh[7][threadIdx.x], sh[7][threadIdx.x + o]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 8) {
    const double v = sh[threadIdx.x][0];
    if (!accumulate) out[threadIdx.x] = v;
    else if (threadIdx.x < 7) out[threadIdx.x] += v;
    else out[7] = fmin(out[7], v);
  }
}

// Minimum of det J over the slabs b0 .. b0+c1-1 of the second direction of the Gauss grid
// (the positivity check of the map; nothing else is computed or stored).  Each wave takes
// one grid row (i0, i1) at a time, four rows per block and iteration, with the row's sums
// over the first two directions staged in LDS as in k_factors_rows; blocks stride over the
// rows with the same trip count, so every wave reaches every barrier.  part[block] receives
// the block's minimum.
__global__ __launch_bounds__(256) void k_detj_rows(GeoDev geo, int b0, int c1, int Q2, long rows, int iters,
                                                   double* __restrict__ part) {
  extern __shared__ double T[];  // [4 waves][3][m2][4]
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p0 = geo.pg[0], p1 = geo.pg[1], p2 = geo.pg[2];
  const int m1 = geo.m[1], m2 = geo.m[2];
  const int tsz = 12 * m2;
  double* Tw = T + w * tsz;
  double mn = 1e300;
  for (int it = 0; it < iters; ++it) {
    const long row = ((long)it * gridDim.x + blockIdx.x) * 4 + w;
    const bool live = row < rows;
    if (live) {
      const int i0 = (int)(row / c1), i1 = b0 + (int)(row % c1);
      const int s0 = geo.span[0][i0], s1 = geo.span[1][i1];
      const double* B0 = geo.B[0] + (long)i0 * (p0 + 1);
      const double* D0 = geo.D[0] + (long)i0 * (p0 + 1);
      const double* B1 = geo.B[1] + (long)i1 * (p1 + 1);
      const double* D1 = geo.D[1] + (long)i1 * (p1 + 1);
      for (int e = lane; e < tsz; e += 64) {
        const int v = e / (m2 * 4), c = (e / 4) % m2, sc = e % 4;
        double acc = 0.0;
        for (int a = 0; a <= p0; ++a) {
          const double wa = (v == 1) ? D0[a] : B0[a];
          for (int b = 0; b <= p1; ++b) {
            const double wb = (v == 2) ? D1[b] : B1[b];
            acc += wa * wb * geo.Pw[(((long)(s0 - p0 + a) * m1 + (s1 - p1 + b)) * m2 + c) * 4 + sc];
          }
        }
        Tw[e] = acc;
      }
    }
    __syncthreads();
    if (live)
      for (int i2 = lane; i2 < Q2; i2 += 64) {
        const int s2 = geo.span[2][i2];
        const double* B2 = geo.B[2] + (long)i2 * (p2 + 1);
        const double* D2 = geo.D[2] + (long)i2 * (p2 + 1);
        double H[4] = {0, 0, 0, 0}, dH[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
        for (int c = 0; c <= p2; ++c) {
          const int cc = s2 - p2 + c;
          const double* t0 = Tw + (0 * m2 + cc) * 4;
          const double* t1 = Tw + (1 * m2 + cc) * 4;
          const double* t2 = Tw + (2 * m2 + cc) * 4;
          const double b2 = B2[c], d2 = D2[c];
          for (int sc = 0; sc < 4; ++sc) {
            H[sc] += b2 * t0[sc];
            dH[0][sc] += b2 * t1[sc];
            dH[1][sc] += b2 * t2[sc];
            dH[2][sc] += d2 * t0[sc];
          }
        }
        mn = fmin(mn, jacobian_det(H, dH));
      }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if (lane == 0) red[w] = mn;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// The same minimum for geometry degree P2 in the third direction: each lane takes a contiguous
// run of points along the row, so neighbouring points share their knot span, and keeps the
// staged sums of that span in registers, reloading them from LDS only when the span changes
// (the generic kernel reads 12 (p_g2 + 1) LDS values per point).  The arithmetic, and so the
// minimum, is the generic kernel's.
template <int P2>
__global__ __launch_bounds__(256) void k_detj_rows_reg(GeoDev geo, int b0, int c1, int Q2, long rows, int iters,
                                                       double* __restrict__ part) {
  extern __shared__ double T[];  // [4 waves][3][m2][4]
  __shared__ double red[4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p0 = geo.pg[0], p1 = geo.pg[1];
  const int m1 = geo.m[1], m2 = geo.m[2];
  const int tsz = 12 * m2;
  double* Tw = T + w * tsz;
  const int run = (Q2 + 63) / 64;
  const int i2a = lane * run, i2b = min(Q2, i2a + run);
  double mn = 1e300;
  for (int it = 0; it < iters; ++it) {
    const long row = ((long)it * gridDim.x + blockIdx.x) * 4 + w;
    const bool live = row < rows;
    if (live) {
      const int i0 = (int)(row / c1), i1 = b0 + (int)(row % c1);
      const int s0 = geo.span[0][i0], s1 = geo.span[1][i1];
      const double* B0 = geo.B[0] + (long)i0 * (p0 + 1);
      const double* D0 = geo.D[0] + (long)i0 * (p0 + 1);
      const double* B1 = geo.B[1] + (long)i1 * (p1 + 1);
      const double* D1 = geo.D[1] + (long)i1 * (p1 + 1);
      for (int e = lane; e < tsz; e += 64) {
        const int v = e / (m2 * 4), c = (e / 4) % m2, sc = e % 4;
        double acc = 0.0;
        for (int a = 0; a <= p0; ++a) {
          const double wa = (v == 1) ? D0[a] : B0[a];
          for (int b = 0; b <= p1; ++b) {
            const double wb = (v == 2) ? D1[b] : B1[b];
            acc += wa * wb * geo.Pw[(((long)(s0 - p0 + a) * m1 + (s1 - p1 + b)) * m2 + c) * 4 + sc];
          }
        }
        Tw[e] = acc;
      }
    }
    __syncthreads();
    if (live && i2a < i2b) {
      double t0[P2 + 1][4], t1[P2 + 1][4], t2[P2 + 1][4];
      int cur = -1;
      // the next point's span and basis values are loaded one point ahead, so that their
      // latency overlaps the current point's arithmetic (two waves per SIMD hide little)
      int s2n = geo.span[2][i2a];
      double bn[P2 + 1], dn[P2 + 1];
#pragma unroll
      for (int c = 0; c <= P2; ++c) {
        bn[c] = geo.B[2][(long)i2a * (P2 + 1) + c];
        dn[c] = geo.D[2][(long)i2a * (P2 + 1) + c];
      }
      for (int i2 = i2a; i2 < i2b; ++i2) {
        const int s2 = s2n;
        double b2v[P2 + 1], d2v[P2 + 1];
#pragma unroll
        for (int c = 0; c <= P2; ++c) {
          b2v[c] = bn[c];
          d2v[c] = dn[c];
        }
        if (i2 + 1 < i2b) {
          s2n = geo.span[2][i2 + 1];
#pragma unroll
          for (int c = 0; c <= P2; ++c) {
            bn[c] = geo.B[2][(long)(i2 + 1) * (P2 + 1) + c];
            dn[c] = geo.D[2][(long)(i2 + 1) * (P2 + 1) + c];
          }
        }
        if (s2 != cur) {
          cur = s2;
#pragma unroll
          for (int c = 0; c <= P2; ++c) {
            const int cc = s2 - P2 + c;
#pragma unroll
            for (int sc = 0; sc < 4; ++sc) {
              t0[c][sc] = Tw[(0 * m2 + cc) * 4 + sc];
              t1[c][sc] = Tw[(1 * m2 + cc) * 4 + sc];
              t2[c][sc] = Tw[(2 * m2 + cc) * 4 + sc];
            }
          }
        }
        double H[4] = {0, 0, 0, 0}, dH[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
        for (int c = 0; c <= P2; ++c) {
          const double b2 = b2v[c], d2 = d2v[c];
#pragma unroll
          for (int sc = 0; sc < 4; ++sc) {
            H[sc] += b2 * t0[c][sc];
            dH[0][sc] += b2 * t1[c][sc];
            dH[1][sc] += b2 * t2[c][sc];
            dH[2][sc] += d2 * t0[c][sc];
          }
        }
        mn = fmin(mn, jacobian_det(H, dH));
      }
    }
    __syncthreads();
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if (lane == 0) red[w] = mn;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// The same minimum for geometries of degree 1 in the third direction, one grid row per lane.
// On a knot span [k_s, k_s+1] of that direction every homogeneous sum is linear in the local
// coordinate t = N_s(xi2) (the second basis value of the span): H(t) = A + B t, the in-plane
// derivatives C + D t and E + F t, and the derivative along xi2 a constant G.  The quotient
// rule gives J = M / w^2 with M_ki = w dH_i,k - H_k dH_i,w (quadratic in t for i = 0, 1, linear
// for i = 2), so det J = det M(t) / w(t)^6 with det M a polynomial of degree 5.  Each lane
// builds the six coefficients of its row's span once (the staged sums of the span's two
// control planes, as in the row kernels) and then evaluates each point by Horner's rule and
// one division (none when the weight is constant along the span, as in extrusions): about 8
// to 20 instructions a point instead of the 100 of the direct formula, four points at a time.
// All lanes of a wave walk the same points of their rows in step, so the span and table loads
// are uniform (scalar).  Agreement with the direct formula: a few units of roundoff relative to the product
// of the Jacobian's column norms.
__device__ inline void poly_mul(const double* a, int na, const double* b, int nb, double* out) {
  for (int i = 0; i < na + nb - 1; ++i) out[i] = 0.0;
  for (int i = 0; i < na; ++i)
    for (int j = 0; j < nb; ++j) out[i + j] += a[i] * b[j];
}

__global__ __launch_bounds__(256) void k_detj_lin(GeoDev geo, int Q1, int Q2, long rows, double* __restrict__ part) {
  __shared__ double red[4];
  const int p0 = geo.pg[0], p1 = geo.pg[1];
  const int m1 = geo.m[1], m2 = geo.m[2];
  double mn = 1e300;
  for (long row = blockIdx.x * 256L + threadIdx.x; row < rows; row += (long)gridDim.x * 256L) {
    const int i0 = (int)(row / Q1), i1 = (int)(row % Q1);
    const int s0 = geo.span[0][i0], s1 = geo.span[1][i1];
    const double* B0 = geo.B[0] + (long)i0 * (p0 + 1);
    const double* D0 = geo.D[0] + (long)i0 * (p0 + 1);
    const double* B1 = geo.B[1] + (long)i1 * (p1 + 1);
    const double* D1 = geo.D[1] + (long)i1 * (p1 + 1);
    int cur = -1;
    double cf[6] = {0, 0, 0, 0, 0, 0}, a3 = 1.0, b3 = 0.0, inv6 = 1.0;
    for (int i2 = 0; i2 < Q2;) {
      const int s2 = geo.span[2][i2];
      if (s2 != cur) {
        cur = s2;
        // T[e][v][sc]: control plane s2 - 1 + e summed over the first two directions (v = 0
        // value, 1 and 2 the derivatives along xi0 and xi1)
        double T[2][3][4];
        for (int e = 0; e < 2; ++e)
          for (int v = 0; v < 3; ++v)
            for (int sc = 0; sc < 4; ++sc) T[e][v][sc] = 0.0;
        for (int a = 0; a <= p0; ++a)
          for (int b = 0; b <= p1; ++b) {
            const double wv = B0[a] * B1[b], w0 = D0[a] * B1[b], w1 = B0[a] * D1[b];
            for (int e = 0; e < 2; ++e) {
              const double* P = geo.Pw + (((long)(s0 - p0 + a) * m1 + (s1 - p1 + b)) * m2 + (s2 - 1 + e)) * 4;
              for (int sc = 0; sc < 4; ++sc) {
                T[e][0][sc] += wv * P[sc];
                T[e][1][sc] += w0 * P[sc];
                T[e][2][sc] += w1 * P[sc];
              }
            }
          }
        const double d20 = geo.D[2][(long)i2 * 2], d21 = geo.D[2][(long)i2 * 2 + 1];
        double A[4], Bc[4], C[4], D[4], E[4], F[4], G[4];
        for (int sc = 0; sc < 4; ++sc) {
          A[sc] = T[0][0][sc];
          Bc[sc] = T[1][0][sc] - T[0][0][sc];
          C[sc] = T[0][1][sc];
          D[sc] = T[1][1][sc] - T[0][1][sc];
          E[sc] = T[0][2][sc];
          F[sc] = T[1][2][sc] - T[0][2][sc];
          G[sc] = d20 * T[0][0][sc] + d21 * T[1][0][sc];
        }
        // M[k][i] coefficients in t (quadratic for i = 0, 1; linear for i = 2)
        double M[3][3][3];
        for (int k = 0; k < 3; ++k) {
          M[k][0][0] = A[3] * C[k] - A[k] * C[3];
          M[k][0][1] = (A[3] * D[k] + Bc[3] * C[k]) - (A[k] * D[3] + Bc[k] * C[3]);
          M[k][0][2] = Bc[3] * D[k] - Bc[k] * D[3];
          M[k][1][0] = A[3] * E[k] - A[k] * E[3];
          M[k][1][1] = (A[3] * F[k] + Bc[3] * E[k]) - (A[k] * F[3] + Bc[k] * E[3]);
          M[k][1][2] = Bc[3] * F[k] - Bc[k] * F[3];
          M[k][2][0] = A[3] * G[k] - A[k] * G[3];
          M[k][2][1] = Bc[3] * G[k] - Bc[k] * G[3];
          M[k][2][2] = 0.0;
        }
        // cofactor expansion along the first row, as polynomials in t: minors of degree 3, 3
        // and 4, the determinant of degree 5
        double x[5], y[5], mn0[4], mn1[4], mn2[5];
        poly_mul(M[1][1], 3, M[2][2], 2, x);
        poly_mul(M[1][2], 2, M[2][1], 3, y);
        for (int i = 0; i < 4; ++i) mn0[i] = x[i] - y[i];
        poly_mul(M[1][0], 3, M[2][2], 2, x);
        poly_mul(M[1][2], 2, M[2][0], 3, y);
        for (int i = 0; i < 4; ++i) mn1[i] = x[i] - y[i];
        poly_mul(M[1][0], 3, M[2][1], 3, x);
        poly_mul(M[1][1], 3, M[2][0], 3, y);
        for (int i = 0; i < 5; ++i) mn2[i] = x[i] - y[i];
        double u0[6], u1[6], u2[6];
        poly_mul(M[0][0], 3, mn0, 4, u0);
        poly_mul(M[0][1], 3, mn1, 4, u1);
        poly_mul(M[0][2], 2, mn2, 5, u2);
        for (int i = 0; i < 6; ++i) cf[i] = u0[i] - u1[i] + u2[i];
        a3 = A[3];
        b3 = Bc[3];
        // a weight constant along the span (extrusions): one division per span
        const double a2 = a3 * a3;
        inv6 = 1.0 / (a2 * a2 * a2);
      }
      auto value = [&](double t) {
        double sdet = cf[5];
#pragma unroll
        for (int i = 4; i >= 0; --i) sdet = sdet * t + cf[i];
        if (b3 == 0.0) return sdet * inv6;
        const double w = a3 + b3 * t;
        const double w2 = w * w;
        return sdet / (w2 * w2 * w2);
      };
      // four points at a time while they stay on this span (the spans do not decrease)
      if (i2 + 3 < Q2 && geo.span[2][i2 + 3] == s2) {
        const double* tb = geo.B[2] + (long)i2 * 2 + 1;
        const double v0 = value(tb[0]), v1 = value(tb[2]), v2 = value(tb[4]), v3 = value(tb[6]);
        mn = fmin(mn, fmin(fmin(v0, v1), fmin(v2, v3)));
        i2 += 4;
      } else {
        mn = fmin(mn, value(geo.B[2][(long)i2 * 2 + 1]));
        i2 += 1;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

// The same minimum for geometry degree P2 = 2 or 3 in the third direction, one grid row per
// lane, by the rational form of k_detj_lin generalised: on a knot span of xi2 every homogeneous
// sum is a polynomial of degree P2 in the local coordinate t = (xi2 - k_s) / h, with the span's
// basis polynomials from P2 + 1 equispaced values (Cox-de Boor) and the inverse Vandermonde
// matrix of those nodes; then M = w dH - H dw has degree 2 P2, det M degree 6 P2 and
// det J = det M(t) / w(t)^6.  Per point: Horner's rule of degree 6 P2, w(t), one division.
// Against the direct formula (CPU check on the bumpy cube and the twisted box, degree 3):
// within 1e-14 of the product of J's column norms.
template <int P2>
__global__ __launch_bounds__(256) void k_detj_poly(GeoDev geo, int Q1, int Q2, long rows, double* __restrict__ part) {
  constexpr int NQ = P2 + 1, NM = 2 * P2 + 1, NMIN = 4 * P2 + 1, NDET = 6 * P2 + 1;
  __shared__ double red[4];
  const int p0 = geo.pg[0], p1 = geo.pg[1];
  const int m1 = geo.m[1], m2 = geo.m[2];
  double mn = 1e300;
  for (long row = blockIdx.x * 256L + threadIdx.x; row < rows; row += (long)gridDim.x * 256L) {
    const int i0 = (int)(row / Q1), i1 = (int)(row % Q1);
    const int s0 = geo.span[0][i0], s1 = geo.span[1][i1];
    const double* B0 = geo.B[0] + (long)i0 * (p0 + 1);
    const double* D0 = geo.D[0] + (long)i0 * (p0 + 1);
    const double* B1 = geo.B[1] + (long)i1 * (p1 + 1);
    const double* D1 = geo.D[1] + (long)i1 * (p1 + 1);
    int cur = -1;
    double cf[NDET], wc[NQ], ka = 0.0, hinv = 1.0;
    for (int i = 0; i < NDET; ++i) cf[i] = 0.0;
    for (int i = 0; i < NQ; ++i) wc[i] = 0.0;
    for (int i2 = 0; i2 < Q2;) {
      const int s2 = geo.span[2][i2];
      if (s2 != cur) {
        cur = s2;
        ka = geo.knots2[s2];
        const double h = geo.knots2[s2 + 1] - ka;
        hinv = 1.0 / h;
        // basis polynomials of the span: A[j][c] = coefficient of t^j in N_{s2-P2+c}
        double A[NQ][NQ];
        {
          double vals[NQ][NQ], dummy[NQ];
          for (int j = 0; j < NQ; ++j) local_basis(geo.knots2, P2, s2, ka + h * ((double)j / P2), vals[j], dummy);
          // inverse Vandermonde of the nodes j / P2 (rows: powers of t, columns: nodes)
          const double vi2[3][3] = {{1.0, 0.0, 0.0}, {-3.0, 4.0, -1.0}, {2.0, -4.0, 2.0}};
          const double vi3[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                    {-5.5, 9.0, -4.5, 1.0},
                                    {9.0, -22.5, 18.0, -4.5},
                                    {-4.5, 13.5, -13.5, 4.5}};
          for (int j = 0; j < NQ; ++j)
            for (int c = 0; c < NQ; ++c) {
              double acc = 0.0;
              for (int q = 0; q < NQ; ++q) acc += (P2 == 2 ? vi2[j][q] : vi3[j][q]) * vals[q][c];
              A[j][c] = acc;
            }
        }
        // staged sums of the span's control planes, as polynomials: q[v][sc][j]
        double q[3][4][NQ];
        for (int v = 0; v < 3; ++v)
          for (int sc = 0; sc < 4; ++sc)
            for (int j = 0; j < NQ; ++j) q[v][sc][j] = 0.0;
        for (int c = 0; c < NQ; ++c) {
          double T[3][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}, {0, 0, 0, 0}};
          for (int a = 0; a <= p0; ++a)
            for (int b = 0; b <= p1; ++b) {
              const double wv = B0[a] * B1[b], w0 = D0[a] * B1[b], w1 = B0[a] * D1[b];
              const double* Pc = geo.Pw + (((long)(s0 - p0 + a) * m1 + (s1 - p1 + b)) * m2 + (s2 - P2 + c)) * 4;
              for (int sc = 0; sc < 4; ++sc) {
                T[0][sc] += wv * Pc[sc];
                T[1][sc] += w0 * Pc[sc];
                T[2][sc] += w1 * Pc[sc];
              }
            }
          for (int v = 0; v < 3; ++v)
            for (int sc = 0; sc < 4; ++sc)
              for (int j = 0; j < NQ; ++j) q[v][sc][j] += A[j][c] * T[v][sc];
        }
        // the derivative along xi2 of the value polynomials (degree P2 - 1, top coefficient 0)
        double g[4][NQ];
        for (int sc = 0; sc < 4; ++sc) {
          for (int j = 0; j + 1 < NQ; ++j) g[sc][j] = (j + 1) * q[0][sc][j + 1] * hinv;
          g[sc][NQ - 1] = 0.0;
        }
        // M[k][i] = w D_i,k - H_k D_i,w (degree 2 P2)
        double M[3][3][NM];
        for (int k = 0; k < 3; ++k)
          for (int i = 0; i < 3; ++i) {
            const double* Dk = i == 0 ? q[1][k] : (i == 1 ? q[2][k] : g[k]);
            const double* Dw = i == 0 ? q[1][3] : (i == 1 ? q[2][3] : g[3]);
            double x[NM], y[NM];
            poly_mul(q[0][3], NQ, Dk, NQ, x);
            poly_mul(q[0][k], NQ, Dw, NQ, y);
            for (int e = 0; e < NM; ++e) M[k][i][e] = x[e] - y[e];
          }
        double x[NMIN], y[NMIN], mn0[NMIN], mn1[NMIN], mn2[NMIN];
        poly_mul(M[1][1], NM, M[2][2], NM, x);
        poly_mul(M[1][2], NM, M[2][1], NM, y);
        for (int e = 0; e < NMIN; ++e) mn0[e] = x[e] - y[e];
        poly_mul(M[1][0], NM, M[2][2], NM, x);
        poly_mul(M[1][2], NM, M[2][0], NM, y);
        for (int e = 0; e < NMIN; ++e) mn1[e] = x[e] - y[e];
        poly_mul(M[1][0], NM, M[2][1], NM, x);
        poly_mul(M[1][1], NM, M[2][0], NM, y);
        for (int e = 0; e < NMIN; ++e) mn2[e] = x[e] - y[e];
        double u[NDET];
        poly_mul(M[0][0], NM, mn0, NMIN, cf);
        poly_mul(M[0][1], NM, mn1, NMIN, u);
        for (int e = 0; e < NDET; ++e) cf[e] -= u[e];
        poly_mul(M[0][2], NM, mn2, NMIN, u);
        for (int e = 0; e < NDET; ++e) cf[e] += u[e];
        for (int j = 0; j < NQ; ++j) wc[j] = q[0][3][j];
      }
      auto value = [&](double xi) {
        const double t = (xi - ka) * hinv;
        double sdet = cf[NDET - 1];
#pragma unroll
        for (int e = NDET - 2; e >= 0; --e) sdet = sdet * t + cf[e];
        double w = wc[NQ - 1];
#pragma unroll
        for (int j = NQ - 2; j >= 0; --j) w = w * t + wc[j];
        const double w2 = w * w;
        return sdet / (w2 * w2 * w2);
      };
      if (i2 + 3 < Q2 && geo.span[2][i2 + 3] == s2) {
        const double* xv = geo.xi2 + i2;
        const double v0 = value(xv[0]), v1 = value(xv[1]), v2 = value(xv[2]), v3 = value(xv[3]);
        mn = fmin(mn, fmin(fmin(v0, v1), fmin(v2, v3)));
        i2 += 4;
      } else {
        mn = fmin(mn, value(geo.xi2[i2]));
        i2 += 1;
      }
    }
  }
  for (int o = 32; o > 0; o >>= 1) mn = fmin(mn, __shfl_xor(mn, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mn;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

__global__ void k_min_reduce(const double* __restrict__ part, long count, double* __restrict__ out) {
  __shared__ double sh[256];
  double v = 1e300;
  for (long b = threadIdx.x; b < count; b += blockDim.x) v = fmin(v, part[b]);
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + o]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// Scattered points: the geometry tables are indexed by the point itself in all directions.
// Grid points given by their three indices: out[f][q] and det_out[q] (optional).
__global__ void k_factors_at(GeoDev geo, SourceDev src, long count, const int* __restrict__ i0,
                             const int* __restrict__ i1, const int* __restrict__ i2, double* __restrict__ out,
                             double* __restrict__ det_out) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= count) return;
  double v[7], det;
  point_factors(geo, src, i0[q], i1[q], i2[q], v, &det);
  for (int f = 0; f < 7; ++f) out[(long)f * count + q] = v[f];
  if (det_out) det_out[q] = det;
}

__global__ void k_factors_points(GeoDev geo, SourceDev src, long count, double* __restrict__ out,
                                 double* __restrict__ det_out) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= count) return;
  double v[7], det;
  point_factors(geo, src, (int)q, (int)q, (int)q, v, &det);
  for (int f = 0; f < 7; ++f) out[(long)f * count + q] = v[f];
  det_out[q] = det;
}

__global__ void k_assemble_band(int n, int p, int g, int ra, int rb, const double* __restrict__ G,
                                const double* __restrict__ w, const double* __restrict__ Brow,
                                const double* __restrict__ Bcol, double* __restrict__ M) {
  const int band = 2 * p + 1;
  const int E = n - p, Q = E * g;
  const long total = (long)ra * n * band * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % rb;
    const int t = (e / rb) % band;
    const int k = (e / ((long)rb * band)) % n;
    const int a = e / ((long)rb * band * n);
    const int l = k + t - p;
    double acc = 0.0;
    if (l >= 0 && l < n) {
      const int elo = max(max(k, l) - p, 0), ehi = min(min(k, l), E - 1);
      for (int el = elo; el <= ehi; ++el) {
        for (int gq = 0; gq < g; ++gq) {
          const int q = el * g + gq;
          acc += w[q] * G[((long)a * Q + q) * rb + b] * Brow[(long)q * (p + 1) + (k - el)] *
                 Bcol[(long)q * (p + 1) + (l - el)];
        }
      }
    }
    M[e] = acc;
  }
}

__global__ void k_assemble_vec(int n, int p, int g, int ra, int rb, const double* __restrict__ G,
                               const double* __restrict__ w, const double* __restrict__ B,
                               double* __restrict__ V) {
  const int E = n - p, Q = E * g;
  const long total = (long)ra * n * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % rb;
    const int k = (e / rb) % n;
    const int a = e / ((long)rb * n);
    double acc = 0.0;
    const int elo = max(k - p, 0), ehi = min(k, E - 1);
    for (int el = elo; el <= ehi; ++el)
      for (int gq = 0; gq < g; ++gq) {
        const int q = el * g + gq;
        acc += w[q] * G[((long)a * Q + q) * rb + b] * B[(long)q * (p + 1) + (k - el)];
      }
    V[e] = acc;
  }
}

// Banded core restricted to rows/columns [lo, lo + n2): band entries pointing outside vanish.
__global__ void k_slice_band(int n, int p, int lo, int n2, int ra, int rb, const double* __restrict__ M,
                             double* __restrict__ O) {
  const int band = 2 * p + 1;
  const long total = (long)ra * n2 * band * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % rb;
    const int t = (e / rb) % band;
    const int i2 = (e / ((long)rb * band)) % n2;
    const int a = e / ((long)rb * band * n2);
    const int j2 = i2 + t - p;
    double v = 0.0;
    if (j2 >= 0 && j2 < n2) v = M[(((long)a * n + (i2 + lo)) * band + t) * rb + b];
    O[e] = v;
  }
}

__global__ void k_slice_vec(int n, int lo, int n2, int ra, int rb, const double* __restrict__ V,
                            double* __restrict__ O) {
  const long total = (long)ra * n2 * rb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % rb;
    const int i2 = (e / rb) % n2;
    const int a = e / ((long)rb * n2);
    O[e] = V[((long)a * n + (i2 + lo)) * rb + b];
  }
}

// Homogeneous control net (w x, w y, w z, w).
__global__ void k_homogeneous(long count, const double* __restrict__ xyz, const double* __restrict__ wts,
                              double* __restrict__ Pw) {
  const long q = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (q >= count) return;
  const double w = wts ? wts[q] : 1.0;
  Pw[q * 4 + 0] = w * xyz[q * 3 + 0];
  Pw[q * 4 + 1] = w * xyz[q * 3 + 1];
  Pw[q * 4 + 2] = w * xyz[q * 3 + 2];
  Pw[q * 4 + 3] = w;
}

// ------------------------------------------------------------------ launchers
static int blocks_for(long total, int per = 256) { return (int)((total + per - 1) / per); }
void launch_basis_tables(Context& ctx, int n, int p, int g, const double* knots, double* xi,
                         double* w, double* B, double* D) {
  const int Q = (n - p) * g;
  hipLaunchKernelGGL(k_basis_tables, dim3(blocks_for(Q)), dim3(256), 0, ctx.stream, n, p, g, knots,
                     xi, w, B, D);
  TTIGA_HIP(hipGetLastError());
}

void launch_geo_tables(Context& ctx, int count, const double* xi, int stride, int nb, int pg,
                       const double* knots, int* span, double* B, double* D) {
  hipLaunchKernelGGL(k_geo_tables, dim3(blocks_for(count)), dim3(256), 0, ctx.stream, count, xi,
                     stride, nb, pg, knots, span, B, D);
  TTIGA_HIP(hipGetLastError());
}

bool detj_rows_fit(const GeoDev& geo) { return 4 * 12 * (size_t)geo.m[2] * sizeof(double) <= 65536; }

void launch_detj_min(Context& ctx, const GeoDev& geo, const int* Q, double* min_out) {
  TTIGA_CHECK(detj_rows_fit(geo), TTIGA_E_ARG, "geometry net too large for the det J rows kernel");
  const long rows = (long)Q[0] * Q[1];
  const long total = rows * Q[2];
  // degree 1 along xi2: a rational function per row and span, about 20 flop a point (the
  // direct formula: 32 (p_g2 + 1) + 40)
  const bool lin = geo.pg[2] == 1;
  // degrees 2 and 3: the polynomial form, given the sample coordinates and knots along xi2
  const bool poly = (geo.pg[2] == 2 || geo.pg[2] == 3) && geo.xi2 && geo.knots2;
  ProfScope prof(ctx, "geometry_detj",
                 (lin ? 20.0 : (poly ? 14.0 * geo.pg[2] + 20.0 : 32.0 * (geo.pg[2] + 1) + 40.0)) * total, 0.0);
  // two blocks per compute unit: the kernel loops over rows for its whole duration, so a
  // larger grid would hold every wave slot while the kernels of other streams wait (the
  // degree-1 kernel: one row per lane, 256 rows per block and pass)
  const int blocks = (int)std::min<long>(lin || poly ? (rows + 255) / 256 : (rows + 3) / 4, 512);
  const int iters = (int)((rows + 4L * blocks - 1) / (4L * blocks));
  DBuf part(ctx.alloc, sizeof(double) * blocks);
  const size_t lds = sizeof(double) * 4 * 12 * geo.m[2];
  if (lin)
    hipLaunchKernelGGL(k_detj_lin, dim3(blocks), dim3(256), 0, ctx.stream, geo, Q[1], Q[2], rows, part.d());
  else if (poly && geo.pg[2] == 2)
    hipLaunchKernelGGL(k_detj_poly<2>, dim3(blocks), dim3(256), 0, ctx.stream, geo, Q[1], Q[2], rows, part.d());
  else if (poly)
    hipLaunchKernelGGL(k_detj_poly<3>, dim3(blocks), dim3(256), 0, ctx.stream, geo, Q[1], Q[2], rows, part.d());
  else if (geo.pg[2] == 2)
    hipLaunchKernelGGL(k_detj_rows_reg<2>, dim3(blocks), dim3(256), lds, ctx.stream, geo, 0, Q[1], Q[2], rows, iters,
                       part.d());
  else if (geo.pg[2] == 3)
    hipLaunchKernelGGL(k_detj_rows_reg<3>, dim3(blocks), dim3(256), lds, ctx.stream, geo, 0, Q[1], Q[2], rows, iters,
                       part.d());
  else
    hipLaunchKernelGGL(k_detj_rows, dim3(blocks), dim3(256), lds, ctx.stream, geo, 0, Q[1], Q[2], rows, iters,
                       part.d());
  hipLaunchKernelGGL(k_min_reduce, dim3(1), dim3(256), 0, ctx.stream, part.d(), (long)blocks, min_out);
  TTIGA_HIP(hipGetLastError());
}

void launch_factors_grid(Context& ctx, const GeoDev& geo, const SourceDev& src, const int* Q,
                         int b0, int c1, double* F, double* stats8, bool accumulate, const int* rows0,
                         int nrows0) {
  TTIGA_CHECK(b0 >= 0 && c1 > 0 && b0 + c1 <= Q[1], TTIGA_E_ARG, "factor slab range out of the grid");
  const long n0 = rows0 ? nrows0 : Q[0];
  const long total = n0 * c1 * Q[2];
  // per point: the p_g2+1-term sums of the value and three derivatives of the homogeneous
  // map, the quotient rule, adjugate, det J, R and f det J (per row the sums over the
  // first two directions are shared); bytes: the seven factor values written
  const double pg2 = geo.pg[2] + 1;
  const double src_flops = src.kind == TTIGA_SOURCE_FOURIER ? 20.0 * src.n_modes + 60.0 : 40.0;
  const double per_pt = 32.0 * pg2 + 150.0 + src_flops;
  ProfScope prof(ctx, "geometry_factors", per_pt * total, 56.0 * total);
  const size_t tbytes = sizeof(double) * 3 * geo.m[2] * 4;
  if (tbytes <= 32768) {
    const long rows = n0 * c1;
    const int threads = Q[2] >= 192 ? 256 : (Q[2] >= 128 ? 192 : (Q[2] >= 64 ? 128 : 64));
    DBuf part(ctx.alloc, sizeof(double) * 8 * rows);
    hipLaunchKernelGGL(k_factors_rows, dim3((unsigned)rows), dim3(threads), tbytes, ctx.stream, geo, src, b0,
                       c1, Q[2], rows0, F, part.d());
    hipLaunchKernelGGL(k_factors_reduce, dim3(1), dim3(256), 0, ctx.stream, part.d(), rows,
                       accumulate ? 1 : 0, stats8);
  } else {
    TTIGA_CHECK(!rows0, TTIGA_E_ARG, "geometry net too large for row sampling");
    const long blocks = (total + 255) / 256;
    DBuf part(ctx.alloc, sizeof(double) * 8 * blocks);
    hipLaunchKernelGGL(k_factors_grid, dim3((unsigned)blocks), dim3(256), 0, ctx.stream, geo, src, Q[0],
                       b0, c1, Q[2], F, part.d());
    hipLaunchKernelGGL(k_factors_reduce, dim3(1), dim3(256), 0, ctx.stream, part.d(), blocks,
                       accumulate ? 1 : 0, stats8);
  }
  TTIGA_HIP(hipGetLastError());
}

void launch_exact_grid(Context& ctx, const GeoDev& geo, const ExactDev& ex, const double* const* w, const int* Q,
                       int b0, int c1, double* F, double* stats8) {
  TTIGA_CHECK(b0 >= 0 && c1 > 0 && b0 + c1 <= Q[1], TTIGA_E_ARG, "error-grid slab range out of the grid");
  const long total = (long)Q[0] * c1 * Q[2];
  const long blocks = (total + 255) / 256;
  DBuf part(ctx.alloc, sizeof(double) * 8 * blocks);
  hipLaunchKernelGGL(k_exact_grid, dim3((unsigned)blocks), dim3(256), 0, ctx.stream, geo, ex, w[0], w[1], w[2],
                     Q[0], b0, c1, Q[2], F, part.d());
  hipLaunchKernelGGL(k_factors_reduce, dim3(1), dim3(256), 0, ctx.stream, part.d(), blocks, 0, stats8);
  TTIGA_HIP(hipGetLastError());
}

void launch_surface_jac(Context& ctx, const GeoDev& geo, int d, int Qi, int Qj, double* out) {
  hipLaunchKernelGGL(k_surface_jac, dim3(grid_for((long)Qi * Qj)), dim3(256), 0, ctx.stream, geo, d, Qi, Qj, out);
  TTIGA_HIP(hipGetLastError());
}

void launch_eval_core(Context& ctx, int ra, int rb, int Q, int g, int p, int lo, int ni, const double* B,
                      const double* U, double* out) {
  const long total = (long)ra * Q * rb;
  hipLaunchKernelGGL(k_eval_core, dim3(grid_for(total)), dim3(256), 0, ctx.stream, ra, rb, Q, g, p, lo, ni, B, U,
                     out);
  TTIGA_HIP(hipGetLastError());
}

void launch_factors_at(Context& ctx, const GeoDev& geo, const SourceDev& src, long count, const int* i0,
                       const int* i1, const int* i2, double* out, double* det) {
  if (count <= 0) return;
  hipLaunchKernelGGL(k_factors_at, dim3(blocks_for(count)), dim3(256), 0, ctx.stream, geo, src, count, i0, i1,
                     i2, out, det);
  TTIGA_HIP(hipGetLastError());
}

void launch_factors_points(Context& ctx, const GeoDev& geo, const SourceDev& src, long count,
                           double* out, double* det) {
  hipLaunchKernelGGL(k_factors_points, dim3(blocks_for(count)), dim3(256), 0, ctx.stream, geo, src,
                     count, out, det);
  TTIGA_HIP(hipGetLastError());
}

void launch_assemble_band(Context& ctx, int n, int p, int g, int ra, int rb, const double* G,
                          const double* w, const double* Brow, const double* Bcol, double* M) {
  const long total = (long)ra * n * (2 * p + 1) * rb;
  ProfScope prof(ctx, "assemble_cores", 4.0 * total * (p + 1) * g, 8.0 * (total + (double)ra * rb * (n - p) * g));
  hipLaunchKernelGGL(k_assemble_band, dim3(grid_for(total)), dim3(256), 0, ctx.stream, n, p, g, ra,
                     rb, G, w, Brow, Bcol, M);
  TTIGA_HIP(hipGetLastError());
}

void launch_assemble_vec(Context& ctx, int n, int p, int g, int ra, int rb, const double* G,
                         const double* w, const double* B, double* V) {
  const long total = (long)ra * n * rb;
  hipLaunchKernelGGL(k_assemble_vec, dim3(grid_for(total)), dim3(256), 0, ctx.stream, n, p, g, ra, rb,
                     G, w, B, V);
  TTIGA_HIP(hipGetLastError());
}

void launch_slice_band(Context& ctx, int n, int p, int lo, int n2, int ra, int rb, const double* M,
                       double* O) {
  const long total = (long)ra * n2 * (2 * p + 1) * rb;
  hipLaunchKernelGGL(k_slice_band, dim3(grid_for(total)), dim3(256), 0, ctx.stream, n, p, lo, n2, ra,
                     rb, M, O);
  TTIGA_HIP(hipGetLastError());
}

void launch_slice_vec(Context& ctx, int n, int lo, int n2, int ra, int rb, const double* V, double* O) {
  const long total = (long)ra * n2 * rb;
  hipLaunchKernelGGL(k_slice_vec, dim3(grid_for(total)), dim3(256), 0, ctx.stream, n, lo, n2, ra, rb,
                     V, O);
  TTIGA_HIP(hipGetLastError());
}

void launch_homogeneous(Context& ctx, long count, const double* xyz, const double* wts, double* Pw) {
  hipLaunchKernelGGL(k_homogeneous, dim3(blocks_for(count)), dim3(256), 0, ctx.stream, count, xyz, wts,
                     Pw);
  TTIGA_HIP(hipGetLastError());
}

}  // namespace ttiga
