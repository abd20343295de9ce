// Randomised rounding of y = alpha K x + beta z without forming the product cores.
//
// K x has the cores y_k[(a b)][i][(a' b')] = sum_t K_k[a][i][t][a'] x_k[b][i+t-p][b'] (banded
// TT-matrix times TT), of ranks rK rx: at the complex-geometry configuration (K ranks about 84,
// n = 512) they would take tens of GB.  The randomised rounding of a TT (Gaussian TT sketch,
// then QR of the sketched unfoldings from left to right, then a deterministic rounding of the
// small result) only needs y through products with the sketch cores and with the left
// factors it builds, and each of those products can be taken through K and x one core at a
// time: the middle core couples row i and column j = i + t - p, so a contraction over the
// K rank becomes one batched GEMM per band offset t over the rows i whose column is in range.
// The sketch matrices are drawn exactly as the rounding of an explicit train draws them, so
// both give the same result up to the order of the floating-point sums.
#include <algorithm>
#include <cstdio>
#include <cstdlib>

#include "runtime.hpp"

namespace ttiga {

namespace {

// out[a][j][l] = sum_t K[a][i][t] O[l][i], i = j + p - t: the last core of a banded TT-matrix
// (trailing rank 1) times the sketch rows O (l x n) over its row index.
__global__ void k_band_last_sketch(int n, int p, int ra, int l, const double* __restrict__ K,
                                   const double* __restrict__ O, double* __restrict__ out) {
  const int band = 2 * p + 1;
  const long total = (long)ra * n * l;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int ll = e % l;
    const int j = (e / l) % n;
    const long a = e / ((long)l * n);
    double s = 0.0;
    for (int t = 0; t < band; ++t) {
      const int i = j + p - t;
      if (i < 0 || i >= n) continue;
      s += K[(a * n + i) * band + t] * O[(long)ll * n + i];
    }
    out[e] = s;
  }
}

// Y[i][l] = alpha sum_t sum_a K0[i][t][a] V[i+t-p][a][l]: the first core of a banded TT-matrix
// (leading rank 1) applied along its row index to V (n x ra x l).
__global__ void k_band_first_apply(int n, int p, int ra, int l, double alpha, const double* __restrict__ K0,
                                   const double* __restrict__ V, double* __restrict__ Y) {
  const int band = 2 * p + 1;
  const long total = (long)n * l;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int ll = e % l;
    const int i = (int)(e / l);
    double s = 0.0;
    for (int t = 0; t < band; ++t) {
      const int j = i + t - p;
      if (j < 0 || j >= n) continue;
      const double* k = K0 + ((long)i * band + t) * ra;
      const double* v = V + (long)j * ra * l + ll;
      for (int a = 0; a < ra; ++a) s += k[a] * v[(long)a * l];
    }
    Y[e] = alpha * s;
  }
}

// S[l][a][j] = sum_t Q[i][l] K0[i][t][a], i = j + p - t: the rows Q (n x lq) contracted with
// the first core of a banded TT-matrix over its row index.
__global__ void k_band_first_adjoint(int n, int p, int ra, int lq, const double* __restrict__ Q,
                                     const double* __restrict__ K0, double* __restrict__ S) {
  const int band = 2 * p + 1;
  const long total = (long)lq * ra * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int j = e % n;
    const int a = (e / n) % ra;
    const int ll = (int)(e / ((long)n * ra));
    double s = 0.0;
    for (int t = 0; t < band; ++t) {
      const int i = j + p - t;
      if (i < 0 || i >= n) continue;
      s += Q[(long)i * lq + ll] * K0[((long)i * band + t) * ra + a];
    }
    S[e] = s;
  }
}

// C[l][i] = sum_t sum_a K2[a][i][t] F[l][a][i+t-p]: the last core of a banded TT-matrix
// (trailing rank 1) applied along its row index.
__global__ void k_band_last_apply(int n, int p, int ra, int l, const double* __restrict__ K2,
                                  const double* __restrict__ F, double* __restrict__ C) {
  const int band = 2 * p + 1;
  const long total = (long)l * n;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = e % n;
    const int ll = (int)(e / n);
    double s = 0.0;
    for (int t = 0; t < band; ++t) {
      const int j = i + t - p;
      if (j < 0 || j >= n) continue;
      for (int a = 0; a < ra; ++a)
        s += K2[((long)a * n + i) * band + t] * F[((long)ll * ra + a) * n + j];
    }
    C[e] = s;
  }
}

// out = in with its four axes permuted: out axis k is in axis perm[k] (dims of in).
__global__ void k_permute4(long d0, long d1, long d2, long d3, int p0, int p1, int p2, int p3,
                           const double* __restrict__ in, double* __restrict__ out) {
  const long d[4] = {d0, d1, d2, d3};
  const int pm[4] = {p0, p1, p2, p3};
  const long od[4] = {d[pm[0]], d[pm[1]], d[pm[2]], d[pm[3]]};
  const long total = d0 * d1 * d2 * d3;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    long rem = e, o[4];
    for (int k = 3; k >= 0; --k) {
      o[k] = rem % od[k];
      rem /= od[k];
    }
    long idx[4];
    for (int k = 0; k < 4; ++k) idx[pm[k]] = o[k];
    out[e] = in[((idx[0] * d1 + idx[1]) * d2 + idx[2]) * d3 + idx[3]];
  }
}

void permute4(Context& ctx, const double* in, long d0, long d1, long d2, long d3, int p0, int p1, int p2,
              int p3, double* out) {
  const long total = d0 * d1 * d2 * d3;
  if (total <= 0) return;
  hipLaunchKernelGGL(k_permute4, dim3(grid_for(total)), dim3(256), 0, ctx.stream, d0, d1, d2, d3, p0, p1, p2,
                     p3, in, out);
  TTIGA_HIP(hipGetLastError());
}

// Rows of the middle mode contracted together: the band products run over blocks of i so
// that their intermediates (bytes_per_row each row) stay within a fixed budget, 4 GiB unless
// TTIGA_MATVEC_BLOCK_BYTES sets another, however large the ranks are.
int middle_block(size_t bytes_per_row, int n1, int p) {
  size_t budget = size_t(4) << 30;
  if (const char* e = std::getenv("TTIGA_MATVEC_BLOCK_BYTES")) budget = std::max<size_t>(1, std::strtoull(e, nullptr, 10));
  const long rows = (long)(budget / std::max<size_t>(bytes_per_row, 1)) - 2 * p;
  return (int)std::max<long>(1, std::min<long>(n1, rows));
}

// The sketched train (Q1, Q2, C3) of y = alpha K x + beta z for sketch widths (l1, l2).
void sketch_project_matvec(Context& ctx, const TT& K, int p, const TT& x, double alpha, const TT* z, double beta,
                           int l1, int l2, TT& y) {
  const int band = 2 * p + 1;
  const int n0 = x.n[0], n1 = x.n[1], n2 = x.n[2];
  const int rK1 = K.r[1], rK2 = K.r[2], rx1 = x.r[1], rx2 = x.r[2];
  const bool hz = z && !z->zero() && beta != 0.0;
  const int rz1 = hz ? z->r[1] : 0, rz2 = hz ? z->r[2] : 0;
  const double *K0 = K.c[0].d(), *K1 = K.c[1].d(), *K2 = K.c[2].d();
  const double *x0 = x.c[0].d(), *x1 = x.c[1].d(), *x2 = x.c[2].d();
  // the sketch, drawn as the rounding of an explicit train draws it
  DBuf O2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * l2), O3(ctx.alloc, sizeof(double) * (size_t)l2 * n2);
  gaussian_fill(ctx, O2.d(), (long)l1 * n1 * l2);
  gaussian_fill(ctx, O3.d(), (long)l2 * n2);
  ProfScope prof(ctx, "matvec_sketch",
                 2.0 * band * ((double)rK1 * rK2 * rx1 * l2 * n1 + (double)rK1 * rK2 * rx2 * l1 * n1), 0.0);
  // right sketches: W3 = y_2 O3^T ([a'][b'][l2]), W2 = y_1 (W3 (x) O2) ([a][b][l1])
  DBuf P(ctx.alloc, sizeof(double) * (size_t)rK2 * n2 * l2), W3(ctx.alloc, sizeof(double) * (size_t)rK2 * rx2 * l2);
  hipLaunchKernelGGL(k_band_last_sketch, dim3(grid_for((long)rK2 * n2 * l2)), dim3(256), 0, ctx.stream, n2, p, rK2,
                     l2, K2, O3.d(), P.d());
  TTIGA_HIP(hipGetLastError());
  gemm_c(ctx, false, false, false, rx2, l2, n2, 1.0, x2, n2, 0, P.d(), l2, (long)n2 * l2, 0.0, W3.d(), l2,
       (long)rx2 * l2, rK2);
  DBuf W2(ctx.alloc, sizeof(double) * (size_t)rK1 * rx1 * l1);
  {
    DBuf W3p(ctx.alloc, sizeof(double) * (size_t)rK2 * rx2 * l2);
    permute4(ctx, W3.d(), 1, rK2, rx2, l2, 0, 2, 1, 3, W3p.d());  // [b'][a'][l2]
    // over blocks [i0, i1) of the middle mode, which read rows j in [i0 - p, i1 + p) of x_1
    const int ib = middle_block(sizeof(double) * 2 * ((size_t)rx1 * rK2 * l2 + (size_t)rK1 * rx1 * l2), n1, p);
    const size_t usz = (size_t)rx1 * std::min(n1, ib + 2 * p) * rK2 * l2, tsz = (size_t)ib * rK1 * rx1 * l2;
    DBuf U(ctx.alloc, sizeof(double) * usz), Up(ctx.alloc, sizeof(double) * usz);
    DBuf Tt(ctx.alloc, sizeof(double) * tsz), T(ctx.alloc, sizeof(double) * tsz);
    for (int i0 = 0; i0 < n1; i0 += ib) {
      const int i1 = std::min(n1, i0 + ib), ic = i1 - i0;
      const int j0 = std::max(0, i0 - p), jc = std::min(n1, i1 + p) - j0;
      if (jc == n1)
        gemm_c(ctx, false, false, false, rx1 * n1, rK2 * l2, rx2, 1.0, x1, rx2, 0, W3p.d(), (long)rK2 * l2, 0, 0.0, U.d(),
             (long)rK2 * l2, 0);
      else  // one product per row b of x_1, over its rows j0..j0+jc
        gemm_c(ctx, false, false, false, jc, rK2 * l2, rx2, 1.0, x1 + (long)j0 * rx2, rx2, (long)n1 * rx2, W3p.d(),
             (long)rK2 * l2, 0, 0.0, U.d(), (long)rK2 * l2, (long)jc * rK2 * l2, rx1);
      permute4(ctx, U.d(), rx1, jc, rK2, l2, 1, 2, 0, 3, Up.d());  // [j][a'][b][l2]
      fill(ctx, Tt.d(), (size_t)ic * rK1 * rx1 * l2, 0.0);
      for (int t = 0; t < band; ++t) {
        const int ilo = std::max(i0, p - t), ihi = std::min(i1, n1 + p - t);
        if (ihi <= ilo) continue;
        gemm_c(ctx, true, false, false, rK1, rx1 * l2, rK2, 1.0, K1 + ((long)ilo * band + t) * rK2, (long)n1 * band * rK2,
             (long)band * rK2, Up.d() + (long)(ilo + t - p - j0) * rK2 * rx1 * l2, (long)rx1 * l2,
             (long)rK2 * rx1 * l2, 1.0, Tt.d() + (long)(ilo - i0) * rK1 * rx1 * l2, (long)rx1 * l2,
             (long)rK1 * rx1 * l2, ihi - ilo);
      }
      permute4(ctx, Tt.d(), ic, rK1, rx1, l2, 1, 2, 0, 3, T.d());  // [a][b][i][l2]
      gemm_c(ctx, false, false, true, rK1 * rx1, l1, ic * l2, 1.0, T.d(), (long)ic * l2, 0, O2.d() + (long)i0 * l2,
           (long)n1 * l2, 0, i0 == 0 ? 0.0 : 1.0, W2.d(), l1, 0);
    }
  }
  DBuf W3z, W2z;
  if (hz) {
    W3z = DBuf(ctx.alloc, sizeof(double) * (size_t)rz2 * l2);
    gemm_c(ctx, false, false, true, rz2, l2, n2, 1.0, z->c[2].d(), n2, 0, O3.d(), n2, 0, 0.0, W3z.d(), l2, 0);
    DBuf Tz(ctx.alloc, sizeof(double) * (size_t)rz1 * n1 * l2);
    gemm_c(ctx, false, false, false, rz1 * n1, l2, rz2, 1.0, z->c[1].d(), rz2, 0, W3z.d(), l2, 0, 0.0, Tz.d(), l2, 0);
    W2z = DBuf(ctx.alloc, sizeof(double) * (size_t)rz1 * l1);
    gemm_c(ctx, false, false, true, rz1, l1, n1 * l2, 1.0, Tz.d(), (long)n1 * l2, 0, O2.d(), (long)n1 * l2, 0, 0.0,
         W2z.d(), l1, 0);
  }
  // first core: Y1 = y_0 W2 (n0 x l1), Q1 its orthonormal basis, M1 = Q1^T y_0
  DBuf Q1(ctx.alloc, sizeof(double) * (size_t)n0 * l1);
  DBuf M1(ctx.alloc, sizeof(double) * (size_t)l1 * rK1 * rx1), M1z;
  {
    DBuf W2p(ctx.alloc, sizeof(double) * (size_t)rK1 * rx1 * l1), V(ctx.alloc, sizeof(double) * (size_t)n0 * rK1 * l1);
    permute4(ctx, W2.d(), 1, rK1, rx1, l1, 0, 2, 1, 3, W2p.d());  // [b][a][l1]
    gemm_c(ctx, false, false, false, n0, rK1 * l1, rx1, 1.0, x0, rx1, 0, W2p.d(), (long)rK1 * l1, 0, 0.0, V.d(),
         (long)rK1 * l1, 0);
    DBuf Y1(ctx.alloc, sizeof(double) * (size_t)n0 * l1), Rq(ctx.alloc, sizeof(double) * (size_t)l1 * l1);
    hipLaunchKernelGGL(k_band_first_apply, dim3(grid_for((long)n0 * l1)), dim3(256), 0, ctx.stream, n0, p, rK1, l1,
                       alpha, K0, V.d(), Y1.d());
    TTIGA_HIP(hipGetLastError());
    if (hz)
      gemm_c(ctx, false, false, false, n0, l1, rz1, beta, z->c[0].d(), rz1, 0, W2z.d(), l1, 0, 1.0, Y1.d(), l1, 0);
    qr_tall(ctx, Y1.d(), false, n0, l1, l1, Q1.d(), Rq.d());
    DBuf S(ctx.alloc, sizeof(double) * (size_t)l1 * rK1 * n0);
    hipLaunchKernelGGL(k_band_first_adjoint, dim3(grid_for((long)l1 * rK1 * n0)), dim3(256), 0, ctx.stream, n0, p,
                       rK1, l1, Q1.d(), K0, S.d());
    TTIGA_HIP(hipGetLastError());
    gemm_c(ctx, false, false, false, l1 * rK1, rx1, n0, alpha, S.d(), n0, 0, x0, rx1, 0, 0.0, M1.d(), rx1, 0);
    if (hz) {
      M1z = DBuf(ctx.alloc, sizeof(double) * (size_t)l1 * rz1);
      gemm_c(ctx, false, true, false, l1, rz1, n0, beta, Q1.d(), l1, 0, z->c[0].d(), rz1, 0, 0.0, M1z.d(), rz1, 0);
    }
  }
  // middle core: Z2 = M1 y_1 (rows (i, l1), columns (a', b')), Y2 = Z2 W3, Q2 its basis,
  // M2 = Q2^T Z2.  Z2 is formed over blocks of i; when it takes more than one block it is
  // formed twice (once for Y2, once for M2) instead of being stored whole.
  const int zb = middle_block(sizeof(double) * 2 * ((size_t)l1 * rK1 * rx2 + (size_t)l1 * rK2 * rx2), n1, p);
  const size_t esz = (size_t)l1 * rK1 * std::min(n1, zb + 2 * p) * rx2, zsz = (size_t)zb * l1 * rK2 * rx2;
  DBuf E(ctx.alloc, sizeof(double) * esz), Ep(ctx.alloc, sizeof(double) * esz);
  DBuf Zt(ctx.alloc, sizeof(double) * zsz), Zc(ctx.alloc, sizeof(double) * zsz);
  auto z2_block = [&](int i0, int i1) {  // Zc = rows i0..i1 of Z2, [i][l1][a'][b']
    const int ic = i1 - i0, j0 = std::max(0, i0 - p), jc = std::min(n1, i1 + p) - j0;
    gemm_c(ctx, false, false, false, l1 * rK1, jc * rx2, rx1, 1.0, M1.d(), rx1, 0, x1 + (long)j0 * rx2, (long)n1 * rx2, 0,
         0.0, E.d(), (long)jc * rx2, 0);
    permute4(ctx, E.d(), l1, rK1, jc, rx2, 2, 1, 0, 3, Ep.d());  // [j][a][l1][b']
    fill(ctx, Zt.d(), (size_t)ic * rK2 * l1 * rx2, 0.0);
    for (int t = 0; t < band; ++t) {
      const int ilo = std::max(i0, p - t), ihi = std::min(i1, n1 + p - t);
      if (ihi <= ilo) continue;
      gemm_c(ctx, true, true, false, rK2, l1 * rx2, rK1, 1.0, K1 + ((long)ilo * band + t) * rK2, (long)n1 * band * rK2,
           (long)band * rK2, Ep.d() + (long)(ilo + t - p - j0) * rK1 * l1 * rx2, (long)l1 * rx2,
           (long)rK1 * l1 * rx2, 1.0, Zt.d() + (long)(ilo - i0) * rK2 * l1 * rx2, (long)l1 * rx2,
           (long)rK2 * l1 * rx2, ihi - ilo);
    }
    permute4(ctx, Zt.d(), ic, rK2, l1, rx2, 0, 2, 1, 3, Zc.d());  // [i][l1][a'][b']
  };
  DBuf Z2z;
  if (hz) {  // [i][l1][c'] = M1z z_1
    Z2z = DBuf(ctx.alloc, sizeof(double) * (size_t)n1 * l1 * rz2);
    gemm_c(ctx, false, false, false, l1, rz2, rz1, 1.0, M1z.d(), rz1, 0, z->c[1].d(), (long)n1 * rz2, rz2, 0.0, Z2z.d(),
         rz2, (long)l1 * rz2, n1);
  }
  DBuf Q2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * l2);
  DBuf M2(ctx.alloc, sizeof(double) * (size_t)l2 * rK2 * rx2), M2z;
  {
    DBuf Y2(ctx.alloc, sizeof(double) * (size_t)n1 * l1 * l2), Rq(ctx.alloc, sizeof(double) * (size_t)l2 * l2);
    for (int i0 = 0; i0 < n1; i0 += zb) {
      const int i1 = std::min(n1, i0 + zb);
      z2_block(i0, i1);
      gemm_c(ctx, false, false, false, (i1 - i0) * l1, l2, rK2 * rx2, 1.0, Zc.d(), (long)rK2 * rx2, 0, W3.d(), l2, 0, 0.0,
           Y2.d() + (long)i0 * l1 * l2, l2, 0);
    }
    if (hz)
      gemm_c(ctx, false, false, false, n1 * l1, l2, rz2, 1.0, Z2z.d(), rz2, 0, W3z.d(), l2, 0, 1.0, Y2.d(), l2, 0);
    DBuf Qi(ctx.alloc, sizeof(double) * (size_t)n1 * l1 * l2);
    qr_tall(ctx, Y2.d(), false, n1 * l1, l2, l2, Qi.d(), Rq.d());
    for (int i0 = 0; i0 < n1; i0 += zb) {
      const int i1 = std::min(n1, i0 + zb);
      if (zb < n1) z2_block(i0, i1);
      gemm_c(ctx, false, true, false, l2, rK2 * rx2, (i1 - i0) * l1, 1.0, Qi.d() + (long)i0 * l1 * l2, l2, 0, Zc.d(),
           (long)rK2 * rx2, 0, i0 == 0 ? 0.0 : 1.0, M2.d(), (long)rK2 * rx2, 0);
    }
    if (hz) {
      M2z = DBuf(ctx.alloc, sizeof(double) * (size_t)l2 * rz2);
      gemm_c(ctx, false, true, false, l2, rz2, n1 * l1, 1.0, Qi.d(), l2, 0, Z2z.d(), rz2, 0, 0.0, M2z.d(), rz2, 0);
    }
    permute4(ctx, Qi.d(), 1, n1, l1, l2, 0, 2, 1, 3, Q2.d());  // [l1][i][l2]
  }
  E = DBuf();
  Ep = DBuf();
  Zt = DBuf();
  Zc = DBuf();
  // last core: C3 = M2 y_2 (l2 x n2)
  DBuf C3(ctx.alloc, sizeof(double) * (size_t)l2 * n2);
  {
    DBuf F(ctx.alloc, sizeof(double) * (size_t)l2 * rK2 * n2);
    gemm_c(ctx, false, false, false, l2 * rK2, n2, rx2, 1.0, M2.d(), rx2, 0, x2, n2, 0, 0.0, F.d(), n2, 0);
    hipLaunchKernelGGL(k_band_last_apply, dim3(grid_for((long)l2 * n2)), dim3(256), 0, ctx.stream, n2, p, rK2, l2,
                       K2, F.d(), C3.d());
    TTIGA_HIP(hipGetLastError());
    if (hz) gemm_c(ctx, false, false, false, l2, n2, rz2, 1.0, M2z.d(), rz2, 0, z->c[2].d(), n2, 0, 1.0, C3.d(), n2, 0);
  }
  y.n[0] = n0;
  y.n[1] = n1;
  y.n[2] = n2;
  y.r[0] = 1;
  y.r[1] = l1;
  y.r[2] = l2;
  y.r[3] = 1;
  y.c[0] = std::move(Q1);
  y.c[1] = std::move(Q2);
  y.c[2] = std::move(C3);
}

}  // namespace

void tt_matvec_round(Context& ctx, const TT& K, int p, const TT& x, double alpha, const TT* z, double beta,
                     double eps_rel, int max_rank, int& hint, TT& out) {
  int n[3];
  for (int k = 0; k < 3; ++k) n[k] = x.n[k];
  const bool hz = z && !z->zero() && beta != 0.0;
  if (K.zero() || x.zero() || alpha == 0.0) {
    if (!hz) {
      out.set_zero(n);
      return;
    }
    tt_axpby(ctx, beta, *z, 0.0, *z, out);
    tt_round_auto(ctx, out, eps_rel, max_rank, hint);
    return;
  }
  for (int k = 0; k < 3; ++k)
    TTIGA_CHECK(K.n[k] == x.n[k] * (2 * p + 1), TTIGA_E_ARG, "matvec: mode sizes differ");
  const int R1 = K.r[1] * x.r[1] + (hz ? z->r[1] : 0), R2 = K.r[2] * x.r[2] + (hz ? z->r[2] : 0);
  int l = std::max(hint, 1) + 10;
  while (true) {
    const int l1 = std::min(l, std::min(R1, n[0]));
    int l2 = std::min(l, std::min(R2, n[2]));
    l2 = std::min(l2, l1 * n[1]);
    TT y;
    sketch_project_matvec(ctx, K, p, x, alpha, z, beta, l1, l2, y);
    tt_round(ctx, y, eps_rel, -1.0, max_rank, nullptr, true);
    if (y.zero()) {
      out.set_zero(n);
      return;
    }
    const bool sat1 = y.r[1] > l1 - 4 && l1 < std::min(R1, n[0]);
    const bool sat2 = y.r[2] > l2 - 4 && l2 < std::min(R2, n[2]);
    if (sat1 || sat2) {  // the sketch may have cut real directions: widen it
      l += 12;
      continue;
    }
    if (const char* e = std::getenv("TTIGA_TRACE_ROUND"); e && e[0] == '1')
      std::fprintf(stderr, "[matvec_round] K (%d,%d) x (%d,%d) l (%d,%d) eps %.1e -> (%d,%d)\n", K.r[1], K.r[2],
                   x.r[1], x.r[2], l1, l2, eps_rel, y.r[1], y.r[2]);
    hint = std::max(y.r[1], y.r[2]);
    out = std::move(y);
    return;
  }
}

size_t matvec_product_bytes(const TT& K, const TT& x) {
  size_t s = 0;
  for (int k = 0; k < 3; ++k) s += (size_t)K.r[k] * x.r[k] * x.n[k] * K.r[k + 1] * x.r[k + 1];
  return s * sizeof(double);
}

}  // namespace ttiga
