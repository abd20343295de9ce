// TT algebra on the device (Section 4.1.1 format; rounding and TT-SVD of
// Oseledets 2011, which the paper cites for its TT format and for the
// rounding after each summation in Section 4.2.1).
//
// Cores live in paper order [r_k][n_k][r_{k+1}], row-major, so the unfolding
// (r_k n_k) x r_{k+1} is a plain row-major matrix and r_k x (n_k r_{k+1}) is its
// transpose view: every contraction below is one strided GEMM.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "runtime.hpp"

namespace ttiga {

void TT::alloc(Context& ctx, const int* nn, const int* rr) {
  for (int k = 0; k < 3; ++k) n[k] = nn[k];
  for (int k = 0; k < 4; ++k) r[k] = rr[k];
  for (int k = 0; k < 3; ++k) c[k] = DBuf(ctx.alloc, sizeof(double) * core_elems(k));
}

// --------------------------------------------------------------- kernels
// Low-precision operands.  BF16 is kept as its 16 raw bits: FP32 rounded to nearest
// even on the upper half (so FP64 -> BF16 rounds through FP32), NaN kept quiet.
__device__ inline uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float lp_to_f32(float v) { return v; }
__device__ inline float lp_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ inline double lp_to_f32(double v) { return v; }
__device__ inline void lp_store(float* p, double v) { *p = (float)v; }
__device__ inline void lp_store(uint16_t* p, double v) { *p = f32_to_bf16((float)v); }

template <class T>
__global__ void k_to_lowp(const double* __restrict__ src, long n, T* __restrict__ dst) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x)
    lp_store(dst + e, src[e]);
}

// One core of the banded TT-matrix x TT-vector product (Section 4.1.1: the cores of K x are
// the mode-wise products of the matrix and vector cores, ranks multiplying):
//   y[(b a)][i][(b' a')] = sum_t M[b][i][t][b'] x[a][i+t-p][a'],   j = i + t - p in range.
// A workgroup takes one (b, a) pair (blockIdx.y) and a tile of TI rows i (blockIdx.x): the
// band entries M[b][i0..i0+TI)[.][.] and the rows x[a][i0-p .. i0+TI+p)[.] (zero outside
// 0..n-1, which drops the out-of-range band entries) are copied to LDS with coalesced loads,
// then each thread owns pairs (i, a'), keeps the 2p+1 values x[a][i+t-p][a'] in registers and
// sweeps b', so the output slab y[(b a)][i0..i0+TI)[.][.] (contiguous) is written once, in
// order, with non-temporal stores (the product is read back only by the next kernel, long
// after it has left the caches; keeping it out of them measured 1.3-2x faster).  The work is bound by writing y (rK rx times the size of x), so the band entries and
// x are read from HBM about once per (b, a).  TK / TX / TS: operator, vector and arithmetic
// types (FP64 throughout, or FP32/BF16 operator with FP32 vector and FP32 arithmetic);
// y is FP64.
template <int P, class TK, class TX, class TS>
__global__ __launch_bounds__(256) void k_band_matvec(int n, int p_rt, int ti, int rK0, int rK1, int rx0, int rx1,
                                                     const TK* __restrict__ M, const TX* __restrict__ X,
                                                     double* __restrict__ Y) {
  extern __shared__ unsigned char lds_raw[];
  // P > 0: the half-width is a compile-time constant and the 2P+1 values of x sit in
  // registers; P = 0: any half-width, x read from LDS in the inner loop
  const int p = P > 0 ? P : p_rt;
  const int band = 2 * p + 1;
  const int ba = blockIdx.y, b = ba / rx0, a = ba - b * rx0;
  const int i0 = blockIdx.x * ti;
  const int rows = min(ti, n - i0);
  // LDS: band entries Ms[il][t][b'] (rows * band * rK1), then x rows Xs[jl][a'] for
  // j = i0 - p + jl, jl < rows + 2p
  TS* Ms = reinterpret_cast<TS*>(lds_raw);
  TS* Xs = Ms + (size_t)ti * band * rK1;
  const int nm = rows * band * rK1;
  const TK* Mg = M + ((size_t)b * n + i0) * band * rK1;
  for (int e = threadIdx.x; e < nm; e += blockDim.x) Ms[e] = (TS)lp_to_f32(Mg[e]);
  const int nxr = rows + 2 * p;
  const TX* Xg = X + (size_t)a * n * rx1;
  for (int e = threadIdx.x; e < nxr * rx1; e += blockDim.x) {
    const int jl = e / rx1;
    const int j = i0 - p + jl;
    Xs[e] = (j >= 0 && j < n) ? (TS)Xg[(size_t)j * rx1 + (e - jl * rx1)] : (TS)0;
  }
  __syncthreads();
  const size_t R1 = (size_t)rK1 * rx1;
  double* Yg = Y + ((size_t)ba * n + i0) * R1;
  const int pairs = rows * rx1;
  for (int q = threadIdx.x; q < pairs; q += blockDim.x) {
    const int il = q / rx1, a2 = q - il * rx1;
    const TS* Mrow = Ms + (size_t)il * band * rK1;
    double* yrow = Yg + (size_t)il * R1 + a2;
    if constexpr (P > 0) {
      TS xv[2 * P + 1];
#pragma unroll
      for (int t = 0; t < 2 * P + 1; ++t) xv[t] = Xs[(il + t) * rx1 + a2];
      for (int b2 = 0; b2 < rK1; ++b2) {
        TS s = (TS)0;
#pragma unroll
        for (int t = 0; t < 2 * P + 1; ++t) s += Mrow[t * rK1 + b2] * xv[t];
        __builtin_nontemporal_store((double)s, yrow + (size_t)b2 * rx1);
      }
    } else {
      const TS* xcol = Xs + (size_t)il * rx1 + a2;
      for (int b2 = 0; b2 < rK1; ++b2) {
        TS s = (TS)0;
        for (int t = 0; t < band; ++t) s += Mrow[t * rK1 + b2] * xcol[(size_t)t * rx1];
        __builtin_nontemporal_store((double)s, yrow + (size_t)b2 * rx1);
      }
    }
  }
}

// Rows per workgroup: as many as fit in 24 KiB of LDS (band entries of the rows plus their
// x halo), at most 256, at least 1: small tiles keep several workgroups per compute unit in
// flight, which hides the load phase of one behind the stores of the others.
static int band_rows(int n, int p, int rK1, int rx1, size_t elem) {
  const size_t budget = (size_t(24) << 10) / elem;
  const size_t per_row = (size_t)(2 * p + 1) * rK1 + rx1;
  const size_t fixed = (size_t)2 * p * rx1;
  long ti = budget > fixed ? (long)((budget - fixed) / per_row) : 1;
  ti = std::max<long>(1, std::min<long>(ti, 256));
  return (int)std::min<long>(ti, n);
}

template <class TK, class TX, class TS>
static void launch_band_matvec(Context& ctx, int n, int p, int rK0, int rK1, int rx0, int rx1, const TK* M,
                               const TX* X, double* Y) {
  const int ti = band_rows(n, p, rK1, rx1, sizeof(TS));
  TTIGA_CHECK((long)rK0 * rx0 <= 65535, TTIGA_E_ARG, "matvec: rK * rx above 65535 on a core's left rank");
  const size_t lds = sizeof(TS) * ((size_t)ti * (2 * p + 1) * rK1 + (size_t)(ti + 2 * p) * rx1);
  TTIGA_CHECK(lds <= (size_t(64) << 10), TTIGA_E_ARG, "matvec: ranks too large for one LDS row tile");
  dim3 grid((n + ti - 1) / ti, rK0 * rx0);
#define TTIGA_BAND_LAUNCH(PP)                                                                       \
  hipLaunchKernelGGL((k_band_matvec<PP, TK, TX, TS>), grid, dim3(256), lds, ctx.stream, n, p, ti, rK0, rK1, \
                     rx0, rx1, M, X, Y)
  switch (p) {
    case 1: TTIGA_BAND_LAUNCH(1); break;
    case 2: TTIGA_BAND_LAUNCH(2); break;
    case 3: TTIGA_BAND_LAUNCH(3); break;
    case 4: TTIGA_BAND_LAUNCH(4); break;
    case 5: TTIGA_BAND_LAUNCH(5); break;
    default: TTIGA_BAND_LAUNCH(0); break;
  }
#undef TTIGA_BAND_LAUNCH
  TTIGA_HIP(hipGetLastError());
}

// out core k of alpha x + beta y (block structure of the TT sum).
__global__ void k_axpby_core(int k, int d, int n, int rx0, int rx1, int ry0, int ry1,
                             const double* __restrict__ X, const double* __restrict__ Yc,
                             const double* alpha_p, double alpha, const double* beta_p,
                             double beta, double* __restrict__ O) {
  const double al = alpha_p ? *alpha_p : alpha;
  const double be = beta_p ? *beta_p : beta;
  const int o0 = (k == 0) ? 1 : rx0 + ry0;
  const int o1 = (k == d - 1) ? 1 : rx1 + ry1;
  const long total = (long)o0 * n * o1;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % o1;
    const int i = (e / o1) % n;
    const int a = e / ((long)o1 * n);
    double v = 0.0;
    if (k == 0) {
      if (b < rx1) v = al * X[(long)i * rx1 + b];
      else v = be * Yc[(long)i * ry1 + (b - rx1)];
    } else if (k == d - 1) {
      if (a < rx0) v = X[(long)a * n + i];
      else v = Yc[(long)(a - rx0) * n + i];
    } else {
      if (a < rx0 && b < rx1) v = X[((long)a * n + i) * rx1 + b];
      else if (a >= rx0 && b >= rx1) v = Yc[((long)(a - rx0) * n + i) * ry1 + (b - rx1)];
    }
    O[e] = v;
  }
}

__global__ void k_scale_copy(const double* __restrict__ X, long n, const double* alpha_p,
                             double alpha, double* __restrict__ O) {
  const double al = alpha_p ? *alpha_p : alpha;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x)
    O[e] = al * X[e];
}

// US[i][j] = U[i][j] * s[j] for j < s_cols (U is m x ldu).
__global__ void k_scale_cols(const double* __restrict__ U, int m, int ldu, const double* __restrict__ s,
                             int cols, double* __restrict__ O) {
  const long total = (long)m * cols;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e / cols, j = e % cols;
    O[e] = U[(long)i * ldu + j] * s[j];
  }
}

// Identity core [m][m] (m x m row-major).
__global__ void k_eye(int m, double* __restrict__ O) {
  const long total = (long)m * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x)
    O[e] = ((e / m) == (e % m)) ? 1.0 : 0.0;
}


// O (rows x s) = first s columns of U (rows x ld)
__global__ void k_copy_cols(const double* __restrict__ U, int rows, int ld, int s,
                            double* __restrict__ O) {
  const long total = (long)rows * s;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x)
    O[e] = U[(e / s) * ld + (e % s)];
}

// O (s x rows) = transpose of the first s columns of V (rows x ld)
__global__ void k_transpose_cols(const double* __restrict__ V, int rows, int ld, int s,
                                 double* __restrict__ O) {
  const long total = (long)rows * s;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int j = e / rows, i = e % rows;
    O[e] = V[(long)i * ld + j];
  }
}

// O[i][:] = s[i] * V[i][:] for a row-major (rows x M) matrix
// Reciprocals of the leading singular values.
__global__ void k_reciprocal(const double* __restrict__ S, int s, double* __restrict__ R) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < s) R[i] = 1.0 / S[i];
}

__global__ void k_scale_rows(const double* __restrict__ V, int rows, long M, const double* __restrict__ s,
                             double* __restrict__ O) {
  const long total = (long)rows * M;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x)
    O[e] = s[e / M] * V[e];
}

// O = diag(1 / s) V: the reciprocal of each row's s, then the product (as k_reciprocal followed
// by k_scale_rows, in one launch)
__global__ void k_scale_rows_inv(const double* __restrict__ V, int rows, long M, const double* __restrict__ s,
                                 double* __restrict__ O) {
  const long total = (long)rows * M;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const double r = 1.0 / s[e / M];
    O[e] = r * V[e];
  }
}

// Standard normal numbers from a counter-based hash (SplitMix64 finaliser + Box-Muller).
__device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

__global__ void k_gaussian(double* __restrict__ O, long n, uint64_t seed);

void gaussian_fill(Context& ctx, double* out, long n) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gaussian, dim3(grid_for(n)), dim3(256), 0, ctx.stream, out, n, ++ctx.rng_counter);
  TTIGA_HIP(hipGetLastError());
}

__global__ void k_gaussian(double* __restrict__ O, long n, uint64_t seed) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n;
       e += (long)gridDim.x * blockDim.x) {
    const uint64_t h1 = mix64(seed * 0x9e3779b97f4a7c15ULL + 2 * (uint64_t)e + 1);
    const uint64_t h2 = mix64(h1 ^ 0xda942042e4dd58b5ULL);
    const double u1 = ((h1 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = ((h2 >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    O[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  }
}

// --------------------------------------------------------------- host ops
void tt_copy(Context& ctx, const TT& src, TT& dst) {
  if (src.zero()) { dst.set_zero(src.n); return; }
  dst.alloc(ctx, src.n, src.r);
  for (int k = 0; k < 3; ++k) copy(ctx, dst.c[k].d(), src.c[k].d(), src.core_elems(k));
}

void tt_from_view(Context& ctx, const ttiga_tt_view& v, TT& out) {
  int n[3], r[4];
  for (int k = 0; k < 3; ++k) n[k] = v.n[k];
  for (int k = 0; k < 4; ++k) r[k] = v.r[k];
  TTIGA_CHECK(r[0] == 1 && r[3] == 1, TTIGA_E_ARG, "TT view needs r0 = r3 = 1");
  for (int k = 0; k < 3; ++k) TTIGA_CHECK(n[k] > 0 && r[k + 1] > 0 && v.core[k], TTIGA_E_ARG, "bad TT view");
  out.alloc(ctx, n, r);
  for (int k = 0; k < 3; ++k) copy(ctx, out.c[k].d(), v.core[k], out.core_elems(k));
}

void tt_matvec_banded(Context& ctx, const TT& K, int p, const TT& x, TT& y) {
  // K is stored as a TT with mode sizes n_k (2p+1).
  int n[3], r[4];
  for (int k = 0; k < 3; ++k) n[k] = x.n[k];
  if (K.zero() || x.zero()) { y.set_zero(n); return; }
  for (int k = 0; k < 3; ++k)
    TTIGA_CHECK(K.n[k] == x.n[k] * (2 * p + 1), TTIGA_E_ARG, "matvec: mode sizes differ");
  for (int k = 0; k < 4; ++k) r[k] = K.r[k] * x.r[k];
  y.alloc(ctx, n, r);
  for (int k = 0; k < 3; ++k) {
    const long total = (long)y.core_elems(k);
    // algorithmic work: the in-range band entries only; bytes: K core, x core, y core
    const double band_nnz = (double)n[k] * (2 * p + 1) - (double)p * (p + 1);
    ProfScope prof(ctx, "tt_matvec_banded",
                   2.0 * band_nnz * K.r[k] * K.r[k + 1] * x.r[k] * x.r[k + 1],
                   8.0 * ((double)K.core_elems(k) + (double)x.core_elems(k) + (double)total));
    launch_band_matvec<double, double, double>(ctx, n[k], p, K.r[k], K.r[k + 1], x.r[k], x.r[k + 1], K.c[k].d(),
                                               x.c[k].d(), y.c[k].d());
  }
}

static size_t lowp_bytes(int dtype) { return dtype == TTIGA_BF16 ? 2 : 4; }

void tt_to_lowp(Context& ctx, const TT& src, int dtype, LowpTT& dst) {
  TTIGA_CHECK(dtype == TTIGA_FP32 || dtype == TTIGA_BF16, TTIGA_E_ARG, "low precision is FP32 or BF16");
  dst.dtype = dtype;
  for (int k = 0; k < 3; ++k) dst.n[k] = src.n[k];
  for (int k = 0; k < 4; ++k) dst.r[k] = src.r[k];
  for (int k = 0; k < 3; ++k) {
    const long ne = (long)src.core_elems(k);
    dst.c[k] = DBuf(ctx.alloc, lowp_bytes(dtype) * std::max<long>(ne, 1));
    if (!ne) continue;
    if (dtype == TTIGA_FP32)
      hipLaunchKernelGGL(k_to_lowp<float>, dim3(grid_for(ne)), dim3(256), 0, ctx.stream, src.c[k].d(), ne,
                         dst.c[k].as<float>());
    else
      hipLaunchKernelGGL(k_to_lowp<uint16_t>, dim3(grid_for(ne)), dim3(256), 0, ctx.stream, src.c[k].d(),
                         ne, dst.c[k].as<uint16_t>());
  }
  TTIGA_HIP(hipGetLastError());
}

void tt_matvec_banded_lp(Context& ctx, const LowpTT& K, int p, const TT& x, TT& y) {
  const int band = 2 * p + 1;
  if (x.zero() || K.r[1] == 0) { y.set_zero(x.n); return; }
  int n[3], r[4];
  for (int k = 0; k < 3; ++k) {
    n[k] = x.n[k];
    TTIGA_CHECK(K.n[k] == n[k] * band, TTIGA_E_ARG, "matvec: operator and vector sizes differ");
  }
  for (int k = 0; k < 4; ++k) r[k] = K.r[k] * x.r[k];
  y.alloc(ctx, n, r);
  const size_t kb = lowp_bytes(K.dtype);
  for (int k = 0; k < 3; ++k) {
    const long total = (long)y.core_elems(k);
    const long nx = (long)x.core_elems(k);
    const double band_nnz = (double)n[k] * band - (double)p * (p + 1);
    ProfScope prof(ctx, K.dtype == TTIGA_BF16 ? "tt_matvec_bf16" : "tt_matvec_fp32",
                   2.0 * band_nnz * K.r[k] * K.r[k + 1] * x.r[k] * x.r[k + 1],
                   (double)kb * K.r[k] * K.r[k + 1] * n[k] * band + 12.0 * nx + 8.0 * (double)total);
    DBuf x32(ctx.alloc, sizeof(float) * nx);
    hipLaunchKernelGGL(k_to_lowp<float>, dim3(grid_for(nx)), dim3(256), 0, ctx.stream, x.c[k].d(), nx,
                       x32.as<float>());
    if (K.dtype == TTIGA_FP32)
      launch_band_matvec<float, float, float>(ctx, n[k], p, K.r[k], K.r[k + 1], x.r[k], x.r[k + 1],
                                              K.c[k].as<float>(), x32.as<float>(), y.c[k].d());
    else
      launch_band_matvec<uint16_t, float, float>(ctx, n[k], p, K.r[k], K.r[k + 1], x.r[k], x.r[k + 1],
                                                 K.c[k].as<uint16_t>(), x32.as<float>(), y.c[k].d());
  }
}

static void axpby_impl(Context& ctx, const double* ap, double a, const TT& x, const double* bp,
                       double b, const TT& y, TT& out) {
  if (x.zero() && y.zero()) { out.set_zero(x.n); return; }
  if (x.zero() || y.zero()) {
    const TT& s = x.zero() ? y : x;
    const double* sp = x.zero() ? bp : ap;
    const double sv = x.zero() ? b : a;
    out.alloc(ctx, s.n, s.r);
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(s.core_elems(0))), dim3(256), 0, ctx.stream,
                       s.c[0].d(), (long)s.core_elems(0), sp, sv, out.c[0].d());
    for (int k = 1; k < 3; ++k) copy(ctx, out.c[k].d(), s.c[k].d(), s.core_elems(k));
    TTIGA_HIP(hipGetLastError());
    return;
  }
  for (int k = 0; k < 3; ++k) TTIGA_CHECK(x.n[k] == y.n[k], TTIGA_E_ARG, "axpby: mode sizes differ");
  int r[4] = {1, x.r[1] + y.r[1], x.r[2] + y.r[2], 1};
  out.alloc(ctx, x.n, r);
  for (int k = 0; k < 3; ++k) {
    const long total = (long)out.core_elems(k);
    ProfScope prof(ctx, "tt_axpby", 0.0, 8.0 * (total + (double)x.core_elems(k) + (double)y.core_elems(k)));
    hipLaunchKernelGGL(k_axpby_core, dim3(grid_for(total)), dim3(256), 0, ctx.stream, k, 3, x.n[k],
                       x.r[k], x.r[k + 1], y.r[k], y.r[k + 1], x.c[k].d(), y.c[k].d(), ap, a, bp, b,
                       out.c[k].d());
  }
  TTIGA_HIP(hipGetLastError());
}

void tt_axpby(Context& ctx, double alpha, const TT& x, double beta, const TT& y, TT& out) {
  axpby_impl(ctx, nullptr, alpha, x, nullptr, beta, y, out);
}

void tt_axpby_dev(Context& ctx, const double* alpha, const TT& x, const double* beta, const TT& y,
                  TT& out) {
  axpby_impl(ctx, alpha, 0.0, x, beta, 0.0, y, out);
}

// The inner product <x, y> as a chain of GEMMs over the cores: L_1 = x_0^T y_0, then per core
// T[b][i][a'] = sum_a L[a][b] x_k[a][i][a'] and L'[a'][b'] = sum_{b,i} T[(b i)][a'] y_k[(b i)][b'];
// the last (1 x 1) product is written to out_dev.  Every temporary lives in one scratch block
// (two L buffers, one T buffer, one area for the partial tiles of split GEMMs), laid out by
// DotScratch, so the same chain runs on arena memory or on a fixed buffer.
namespace {
struct DotScratch {
  size_t l = 0, t = 0, part = 0;
  DotScratch(const int* n, const int* rx, const int* ry) {
    auto part_of = [&](int M, int N, int K) { return gemm_part_doubles(gemm_plan(true, false, M, N, K, 1), M, N, 1); };
    l = std::max((size_t)rx[1] * ry[1], (size_t)rx[2] * ry[2]);
    t = std::max((size_t)ry[1] * n[1] * rx[2], (size_t)ry[2] * n[2] * rx[3]);
    part = std::max({part_of(rx[1], ry[1], n[0]), part_of(ry[1], n[1] * rx[2], rx[1]),
                     part_of(rx[2], ry[2], ry[1] * n[1]), part_of(ry[2], n[2] * rx[3], rx[2]),
                     part_of(rx[3], ry[3], ry[2] * n[2])});
  }
  size_t total() const { return 2 * l + t + part; }
};
}  // namespace

size_t tt_dot_scratch_doubles(const int* n, const int* rx, const int* ry) { return DotScratch(n, rx, ry).total(); }

void tt_dot_cores(Context& ctx, const int* n, const int* rx, const double* const* xc, const int* ry,
                  const double* const* yc, double* out_dev, double* scratch) {
  const DotScratch sz(n, rx, ry);
  double* Lb[2] = {scratch, scratch + sz.l};
  double* T = scratch + 2 * sz.l;
  double* part = T + sz.t;
  auto mm = [&](bool ta, int M, int N, int K, const double* A, long lda, const double* B, long ldb, double* C,
                long ldc) {
    gemm_planned(ctx, gemm_plan(ta, false, M, N, K, 1), ta, false, M, N, K, 1.0, A, lda, 0, B, ldb, 0, 0.0, C, ldc, 0, 1,
                 part);
  };
  mm(true, rx[1], ry[1], n[0], xc[0], rx[1], yc[0], ry[1], Lb[0], ry[1]);
  int cur = 0;
  for (int k = 1; k < 3; ++k) {
    const int rx0 = rx[k], rx1 = rx[k + 1], ry0 = ry[k], ry1 = ry[k + 1], nk = n[k];
    // T (ry0 x nk rx1) = L^T (ry0 x rx0) * x_k (rx0 x nk rx1)
    mm(true, ry0, nk * rx1, rx0, Lb[cur], ry0, xc[k], (long)nk * rx1, T, (long)nk * rx1);
    // L' (rx1 x ry1) = T^T viewed as (ry0 nk) x rx1, times y_k ((ry0 nk) x ry1)
    double* dst = (k < 2) ? Lb[1 - cur] : out_dev;
    mm(true, rx1, ry1, ry0 * nk, T, rx1, yc[k], ry1, dst, ry1);
    cur = 1 - cur;
  }
}

void tt_dot_dev(Context& ctx, const TT& x, const TT& y, double* out_dev) {
  if (x.zero() || y.zero()) { fill(ctx, out_dev, 1, 0.0); return; }
  DBuf scratch(ctx.alloc, sizeof(double) * tt_dot_scratch_doubles(x.n, x.r, y.r));
  const double* xc[3] = {x.c[0].d(), x.c[1].d(), x.c[2].d()};
  const double* yc[3] = {y.c[0].d(), y.c[1].d(), y.c[2].d()};
  tt_dot_cores(ctx, x.n, x.r, xc, y.r, yc, out_dev, scratch.d());
}

// The products land in device memory and one fenced kernel hands them to the host-mapped
// array (a product kernel's plain stores into host memory need not be visible when the host
// sees the stream drain).
double tt_dot_sync(Context& ctx, const TT& x, const TT& y) {
  const TT* xp = &x;
  const TT* yp = &y;
  double out = 0.0;
  tt_dots_sync(ctx, &xp, &yp, 1, &out);
  return out;
}

void tt_dots_sync(Context& ctx, const TT* const* x, const TT* const* y, int count, double* out) {
  TTIGA_CHECK(count > 0 && count <= 8, TTIGA_E_ARG, "tt_dots_sync: 1..8 pairs");
  DBuf dev(ctx.alloc, sizeof(double) * count);
  for (int i = 0; i < count; ++i) tt_dot_dev(ctx, *x[i], *y[i], dev.d() + i);
  double* hd = ctx.host_device(count);
  publish_to_host(ctx, dev.d(), hd, count);
  ctx.sync();
  for (int i = 0; i < count; ++i) out[i] = ctx.host_scratch[i];
}

// Truncated SVD of B (r x M, row-major): B ~= U_s diag(S_s) Vt_s with orthonormal U_s
// (r x s) and orthonormal rows Vt_s (s x M).  The rank is chosen by trunc_rank_sync:
// delta >= 0 is an absolute threshold, delta < 0 means relative eps = -delta.
struct TruncSVD {
  int s = 0;
  DBuf U, S, Vt;
  double norm = 0.0, delta = 0.0;
};

// Truncated SVD of a wide r x M matrix through its Gram matrix: G = B B^T by one MFMA
// GEMM, then the eigendecomposition of G: a pivoted Cholesky factor G = L L^T (r x k,
// stopped at pivots below u max G_ii) and a one-sided Jacobi SVD of L = E S W^T, so
// G = E S^2 E^T: E are the eigenvectors of G, S = sqrt(lam) the singular values of B
// (Jacobi on L converges in the sweeps of Jacobi on a triangular factor, about a third of
// those of Jacobi on G itself).  U_s the leading eigenvectors and V_s^T = S_s^-1 U_s^T B.
// Squaring resolves singular values down to about sqrt(u) ||B|| and the rows of V_s^T are
// orthonormal to about u (sigma_1 / sigma_s)^2, so this route is taken only for relative
// thresholds of 1e-6 and above; the Schur complement left out of L has trace at most
// r u max G_ii, far below their square.
static TruncSVD truncated_svd_gram(Context& ctx, const double* B, int r, long M, double delta) {
  TruncSVD o;
  DBuf G(ctx.alloc, sizeof(double) * r * r);
  gemm(ctx, false, true, r, r, (int)M, 1.0, B, M, 0, B, M, 0, 0.0, G.d(), r, 0);
  DBuf L(ctx.alloc, sizeof(double) * r * r);
  const int k = pivoted_cholesky(ctx, G.d(), r, L.d(), 2.220446049250313e-16);
  o.S = DBuf(ctx.alloc, sizeof(double) * r);
  fill(ctx, o.S.d(), r, 0.0);
  DBuf V;  // r x k eigenvectors, row-major
  if (k > 0) {
    V = DBuf(ctx.alloc, sizeof(double) * r * k);
    svd_small(ctx, L.d(), false, r, k, r, V.d(), o.S.d(), nullptr, "jacobi_eig");
  }
  double nd[2];
  o.s = trunc_rank_sync(ctx, o.S.d(), r, delta, nd);
  o.norm = nd[0];
  o.delta = nd[1];
  if (o.s == 0) return o;
  o.U = DBuf(ctx.alloc, sizeof(double) * r * o.s);
  hipLaunchKernelGGL(k_copy_cols, dim3(grid_for((long)r * o.s)), dim3(256), 0, ctx.stream, V.d(), r, k, o.s,
                     o.U.d());
  DBuf W(ctx.alloc, sizeof(double) * o.s * M);
  gemm(ctx, true, false, o.s, (int)M, r, 1.0, V.d(), k, 0, B, M, 0, 0.0, W.d(), M, 0);
  o.Vt = DBuf(ctx.alloc, sizeof(double) * o.s * M);
  hipLaunchKernelGGL(k_scale_rows_inv, dim3(grid_for((long)o.s * M)), dim3(256), 0, ctx.stream, W.d(), o.s, M,
                     o.S.d(), o.Vt.d());
  TTIGA_HIP(hipGetLastError());
  return o;
}

// relative rounding thresholds at or above which the right-to-left sweep uses the Gram route
static constexpr double kGramEps = 1e-6;

static TruncSVD truncated_svd(Context& ctx, const double* B, int r, long M, double delta,
                              bool gram = false) {
  if (gram && M >= r) return truncated_svd_gram(ctx, B, r, M, delta);
  TruncSVD o;
  if (M >= r) {
    // B^T = Q T (M x r), B = T^T Q^T, svd(T^T) = Ut S W^T, so B = Ut S (Q W)^T
    DBuf Q(ctx.alloc, sizeof(double) * M * r), T(ctx.alloc, sizeof(double) * r * r);
    qr_tall(ctx, B, true, (int)M, r, M, Q.d(), T.d());
    DBuf Ut(ctx.alloc, sizeof(double) * r * r), W(ctx.alloc, sizeof(double) * r * r);
    o.S = DBuf(ctx.alloc, sizeof(double) * r);
    svd_small(ctx, T.d(), true, r, r, r, Ut.d(), o.S.d(), W.d());
    double nd[2];
    o.s = trunc_rank_sync(ctx, o.S.d(), r, delta, nd);
    o.norm = nd[0];
    o.delta = nd[1];
    if (o.s == 0) return o;
    o.Vt = DBuf(ctx.alloc, sizeof(double) * o.s * M);
    gemm(ctx, true, true, o.s, (int)M, r, 1.0, W.d(), r, 0, Q.d(), r, 0, 0.0, o.Vt.d(), M, 0);
    o.U = DBuf(ctx.alloc, sizeof(double) * r * o.s);
    hipLaunchKernelGGL(k_copy_cols, dim3(grid_for((long)r * o.s)), dim3(256), 0, ctx.stream, Ut.d(),
                       r, r, o.s, o.U.d());
  } else {
    // tall: B = Q T (r x M); Jacobi on the rows of T (converges in about half the
    // sweeps of its columns): T^T = V S Ut^T, so B = (Q Ut) S V^T
    const int c = (int)M;
    DBuf Q(ctx.alloc, sizeof(double) * (size_t)r * c), T(ctx.alloc, sizeof(double) * c * c);
    qr_tall(ctx, B, false, r, c, c, Q.d(), T.d());
    DBuf Ut(ctx.alloc, sizeof(double) * c * c), V(ctx.alloc, sizeof(double) * c * c);
    o.S = DBuf(ctx.alloc, sizeof(double) * c);
    svd_small(ctx, T.d(), true, c, c, c, V.d(), o.S.d(), Ut.d());
    double nd[2];
    o.s = trunc_rank_sync(ctx, o.S.d(), c, delta, nd);
    o.norm = nd[0];
    o.delta = nd[1];
    if (o.s == 0) return o;
    o.U = DBuf(ctx.alloc, sizeof(double) * (size_t)r * o.s);
    gemm(ctx, false, false, r, o.s, c, 1.0, Q.d(), c, 0, Ut.d(), c, 0, 0.0, o.U.d(), o.s, 0);
    o.Vt = DBuf(ctx.alloc, sizeof(double) * o.s * M);
    hipLaunchKernelGGL(k_transpose_cols, dim3(grid_for((long)c * o.s)), dim3(256), 0, ctx.stream,
                       V.d(), c, c, o.s, o.Vt.d());
  }
  TTIGA_HIP(hipGetLastError());
  return o;
}

void tt_round(Context& ctx, TT& x, double eps_rel, double delta_abs, int max_rank,
              double* norm_out, bool left_orthogonal) {
  if (x.zero()) {
    if (norm_out) norm_out[0] = 0.0;
    return;
  }
  // Phase 1: left-orthogonalise cores 0 and 1 (QR of the (r_k n_k) x r_{k+1} unfoldings).
  for (int k = 0; k < (left_orthogonal ? 0 : 2); ++k) {
    const int m = x.r[k] * x.n[k], c = x.r[k + 1];
    const int nn = x.n[k + 1], r2 = x.r[k + 2];
    if (m >= c) {
      DBuf Q(ctx.alloc, sizeof(double) * (size_t)m * c), R(ctx.alloc, sizeof(double) * c * c);
      qr_tall(ctx, x.c[k].d(), false, m, c, c, Q.d(), R.d());
      DBuf nxt(ctx.alloc, sizeof(double) * (size_t)c * nn * r2);
      gemm(ctx, false, false, c, nn * r2, c, 1.0, R.d(), c, 0, x.c[k + 1].d(), (long)nn * r2, 0, 0.0,
           nxt.d(), (long)nn * r2, 0);
      x.c[k] = std::move(Q);
      x.c[k + 1] = std::move(nxt);
    } else {
      // wide unfolding: Q = I_m, R = the unfolding itself; the rank drops to m
      DBuf nxt(ctx.alloc, sizeof(double) * (size_t)m * nn * r2);
      gemm(ctx, false, false, m, nn * r2, c, 1.0, x.c[k].d(), c, 0, x.c[k + 1].d(), (long)nn * r2, 0,
           0.0, nxt.d(), (long)nn * r2, 0);
      DBuf I(ctx.alloc, sizeof(double) * (size_t)m * m);
      hipLaunchKernelGGL(k_eye, dim3(grid_for((long)m * m)), dim3(256), 0, ctx.stream, m, I.d());
      TTIGA_HIP(hipGetLastError());
      x.c[k] = std::move(I);
      x.c[k + 1] = std::move(nxt);
      x.r[k + 1] = m;
    }
  }
  // Phase 2: right-to-left truncated SVDs of the r_k x (n_k r_{k+1}) unfoldings; the
  // whole norm sits in the last core, so the first SVD fixes the threshold.
  double delta = delta_abs >= 0.0 ? delta_abs : -eps_rel;
  const bool gram = delta_abs < 0.0 && eps_rel >= kGramEps;
  for (int k = 2; k >= 1; --k) {
    const int r = x.r[k];
    const long M = (long)x.n[k] * x.r[k + 1];
    TruncSVD t = truncated_svd(ctx, x.c[k].d(), r, M, delta, gram);
    if (k == 2) {
      if (norm_out) norm_out[0] = t.norm;
      delta = t.delta;
    }
    if (t.s == 0) {
      x.set_zero(x.n);
      return;
    }
    if (max_rank > 0 && t.s > max_rank)
      throw Error(TTIGA_E_RANKCAP, "TT rank " + std::to_string(t.s) + " exceeds max_rank");
    // core_{k-1} <- core_{k-1} * U_s S_s   ((r_{k-1} n_{k-1}) x r) * (r x s)
    DBuf US(ctx.alloc, sizeof(double) * r * t.s);
    hipLaunchKernelGGL(k_scale_cols, dim3(grid_for((long)r * t.s)), dim3(256), 0, ctx.stream, t.U.d(),
                       r, t.s, t.S.d(), t.s, US.d());
    TTIGA_HIP(hipGetLastError());
    const int mprev = x.r[k - 1] * x.n[k - 1];
    DBuf prev(ctx.alloc, sizeof(double) * (size_t)mprev * t.s);
    gemm(ctx, false, false, mprev, t.s, r, 1.0, x.c[k - 1].d(), r, 0, US.d(), t.s, 0, 0.0, prev.d(),
         t.s, 0);
    x.c[k] = std::move(t.Vt);
    x.c[k - 1] = std::move(prev);
    x.r[k] = t.s;
  }
}

// Left factor of an (m x M) row-major matrix A to the absolute threshold delta:
// A ~= U (m x s, orthonormal columns) * C (s x M).  Exact SVD when min(m, M) <= kExact,
// otherwise a randomised range finder: Y = A * Omega with Gaussian Omega (M x l),
// U_y = orth(Y), B = U_y^T A, truncated SVD of B; the sketch width l starts at 48
// and doubles while the truncated rank leaves fewer than 12 spare columns.
static constexpr int kExact = kExactSvdSize;

static int left_factor(Context& ctx, const double* A, int m, long M, double delta, DBuf& U,
                       DBuf& C) {
  if (m <= kExact || M <= kExact) {
    TruncSVD t = truncated_svd(ctx, A, m, M, delta);
    if (t.s == 0) return 0;
    U = std::move(t.U);
    C = DBuf(ctx.alloc, sizeof(double) * t.s * M);
    hipLaunchKernelGGL(k_scale_rows, dim3(grid_for((long)t.s * M)), dim3(256), 0, ctx.stream,
                       t.Vt.d(), t.s, M, t.S.d(), C.d());
    TTIGA_HIP(hipGetLastError());
    return t.s;
  }
  int l = std::min(m, 48);
  while (true) {
    DBuf Om(ctx.alloc, sizeof(double) * M * l), Y(ctx.alloc, sizeof(double) * (size_t)m * l);
    const uint64_t seed = ++ctx.rng_counter;
    hipLaunchKernelGGL(k_gaussian, dim3(grid_for(M * l)), dim3(256), 0, ctx.stream, Om.d(), M * l,
                       seed);
    TTIGA_HIP(hipGetLastError());
    gemm(ctx, false, false, m, l, (int)M, 1.0, A, M, 0, Om.d(), l, 0, 0.0, Y.d(), l, 0);
    DBuf Qy(ctx.alloc, sizeof(double) * (size_t)m * l), Ry(ctx.alloc, sizeof(double) * l * l);
    qr_tall(ctx, Y.d(), false, m, l, l, Qy.d(), Ry.d());
    DBuf B(ctx.alloc, sizeof(double) * l * M);
    gemm(ctx, true, false, l, (int)M, m, 1.0, Qy.d(), l, 0, A, M, 0, 0.0, B.d(), M, 0);
    TruncSVD t = truncated_svd(ctx, B.d(), l, M, delta);
    if (t.s == 0) return 0;
    if (t.s > l - 12 && l < m) {
      l = std::min(m, 2 * l);
      continue;
    }
    U = DBuf(ctx.alloc, sizeof(double) * (size_t)m * t.s);
    gemm(ctx, false, false, m, t.s, l, 1.0, Qy.d(), l, 0, t.U.d(), t.s, 0, 0.0, U.d(), t.s, 0);
    C = DBuf(ctx.alloc, sizeof(double) * t.s * M);
    hipLaunchKernelGGL(k_scale_rows, dim3(grid_for((long)t.s * M)), dim3(256), 0, ctx.stream,
                       t.Vt.d(), t.s, M, t.S.d(), C.d());
    TTIGA_HIP(hipGetLastError());
    return t.s;
  }
}

// TT-SVD (Oseledets 2011, Alg. 1) of a dense device tensor A[n0][n1][n2] with an
// absolute per-unfolding threshold delta: A_(0) = U0 C0, then C0 reshaped
// (s0 n1) x n2 = U1 C1; cores U0, U1 (left-orthonormal) and C1.
void tt_compress_dense(Context& ctx, const double* A, const int* n, double delta, TT& out,
                       int max_rank) {
  DBuf U0, C0;
  const long M0 = (long)n[1] * n[2];
  const int s0 = left_factor(ctx, A, n[0], M0, delta, U0, C0);
  if (s0 == 0) { out.set_zero(n); return; }
  DBuf U1, C1;
  const int s1 = left_factor(ctx, C0.d(), s0 * n[1], n[2], delta, U1, C1);
  if (s1 == 0) { out.set_zero(n); return; }
  if (max_rank > 0 && (s0 > max_rank || s1 > max_rank))
    throw Error(TTIGA_E_RANKCAP, "compressed factor rank exceeds max_rank");
  for (int k = 0; k < 3; ++k) out.n[k] = n[k];
  out.r[0] = 1; out.r[1] = s0; out.r[2] = s1; out.r[3] = 1;
  out.c[0] = std::move(U0);
  out.c[1] = std::move(U1);
  out.c[2] = std::move(C1);
}

// Slab-streamed TT-SVD of nt tensors A_t[n0][n1][n2] that exist only one chunk of
// second-direction slabs (all i0, a range of i1, all i2) at a time.  The first
// unfolding A_t (n0 x n1 n2) goes through the randomised range finder in two passes over
// the chunks: Y_t = A_t Omega (n0 x l, one Gaussian Omega shared by all tensors) summed
// over the column blocks, Q_t = orth(Y_t), then B_t = Q_t^T A_t (l x n1 n2), one column
// block per chunk; the truncated SVD of B_t gives the first core Q_t U_s and
// C_t = S_s V_s^T, which is factored like a dense tensor.  The thresholds are set after
// the first pass (they depend on norms gathered while producing); a negative threshold
// marks a tensor as exactly zero.  A tensor whose truncated rank leaves fewer than 12
// spare sketch columns is redone with twice the width.
void tt_compress_streamed(Context& ctx, int nt, const int* n, int chunk, const ChunkFn& produce,
                          const ThresholdFn& thresholds, TT* out, int max_rank) {
  const int n0 = n[0], n1 = n[1], n2 = n[2];
  const long M = (long)n1 * n2;
  TTIGA_CHECK(nt > 0 && chunk > 0 && n0 > kExact && M > kExact && M <= INT32_MAX, TTIGA_E_ARG,
              "streamed compression needs more than 64 rows and columns");
  chunk = std::min(chunk, n1);
  DBuf buf(ctx.alloc, sizeof(double) * (size_t)nt * n0 * chunk * n2);
  std::vector<double> delta(nt, 0.0);
  std::vector<char> todo(nt, 1);
  bool have_delta = false;
  int L = std::min(n0, 48);
  while (true) {
    bool any = false;
    for (int t = 0; t < nt; ++t) any = any || todo[t];
    if (!any) break;
    // pass 1: range sketches, summed over the column blocks
    std::vector<DBuf> Y(nt);
    {
      DBuf Om(ctx.alloc, sizeof(double) * (size_t)M * L);
      hipLaunchKernelGGL(k_gaussian, dim3(grid_for(M * L)), dim3(256), 0, ctx.stream, Om.d(), M * L,
                         ++ctx.rng_counter);
      TTIGA_HIP(hipGetLastError());
      for (int t = 0; t < nt; ++t)
        if (todo[t]) Y[t] = DBuf(ctx.alloc, sizeof(double) * (size_t)n0 * L);
      for (int b = 0; b < n1; b += chunk) {
        const int c = std::min(chunk, n1 - b);
        const long w = (long)c * n2;
        produce(b, c, buf.d());
        for (int t = 0; t < nt; ++t)
          if (todo[t])
            gemm(ctx, false, false, n0, L, (int)w, 1.0, buf.d() + (size_t)t * n0 * w, w, 0,
                 Om.d() + (size_t)b * n2 * L, L, 0, b == 0 ? 0.0 : 1.0, Y[t].d(), L, 0);
      }
    }
    if (!have_delta) {
      thresholds(delta);
      have_delta = true;
      for (int t = 0; t < nt; ++t)
        if (delta[t] < 0.0) {
          todo[t] = 0;
          out[t].set_zero(n);
          Y[t].reset();
        }
    }
    // orthonormal bases of the sketches
    std::vector<DBuf> Qy(nt), B(nt);
    for (int t = 0; t < nt; ++t) {
      if (!todo[t]) continue;
      Qy[t] = DBuf(ctx.alloc, sizeof(double) * (size_t)n0 * L);
      DBuf Ry(ctx.alloc, sizeof(double) * L * L);
      qr_tall(ctx, Y[t].d(), false, n0, L, L, Qy[t].d(), Ry.d());
      Y[t].reset();
      B[t] = DBuf(ctx.alloc, sizeof(double) * (size_t)L * M);
    }
    // pass 2: projections B_t = Q_t^T A_t, one column block per chunk
    for (int b = 0; b < n1; b += chunk) {
      const int c = std::min(chunk, n1 - b);
      const long w = (long)c * n2;
      produce(b, c, buf.d());
      for (int t = 0; t < nt; ++t)
        if (todo[t])
          gemm(ctx, true, false, L, (int)w, n0, 1.0, Qy[t].d(), L, 0, buf.d() + (size_t)t * n0 * w, w,
               0, 0.0, B[t].d() + (size_t)b * n2, M, 0);
    }
    bool widen = false;
    for (int t = 0; t < nt; ++t) {
      if (!todo[t]) continue;
      const bool fits = tt_from_first_unfolding(ctx, Qy[t].d(), L, B[t].d(), n, delta[t], L < n0 ? 12 : 0,
                                                out[t], max_rank);
      B[t].reset();
      if (!fits) {
        widen = true;
        continue;
      }
      todo[t] = 0;
    }
    if (widen) L = std::min(n0, 2 * L);
  }
}

bool tt_from_first_unfolding(Context& ctx, const double* Qb, int L, const double* B, const int* n, double delta,
                             int spare, TT& out, int max_rank) {
  const int n0 = n[0], n1 = n[1], n2 = n[2];
  const long M = (long)n1 * n2;
  TruncSVD sv = truncated_svd(ctx, B, L, M, delta);
  if (sv.s == 0) {
    out.set_zero(n);
    return true;
  }
  if (spare > 0 && sv.s > L - spare) return false;
  const int s0 = sv.s;
  DBuf U0(ctx.alloc, sizeof(double) * (size_t)n0 * s0);
  gemm(ctx, false, false, n0, s0, L, 1.0, Qb, L, 0, sv.U.d(), s0, 0, 0.0, U0.d(), s0, 0);
  DBuf C0(ctx.alloc, sizeof(double) * (size_t)s0 * M);
  hipLaunchKernelGGL(k_scale_rows, dim3(grid_for((long)s0 * M)), dim3(256), 0, ctx.stream, sv.Vt.d(), s0, M,
                     sv.S.d(), C0.d());
  TTIGA_HIP(hipGetLastError());
  DBuf U1, C1;
  const int s1 = left_factor(ctx, C0.d(), s0 * n1, n2, delta, U1, C1);
  if (s1 == 0) {
    out.set_zero(n);
    return true;
  }
  if (max_rank > 0 && (s0 > max_rank || s1 > max_rank))
    throw Error(TTIGA_E_RANKCAP, "compressed factor rank exceeds max_rank");
  for (int k = 0; k < 3; ++k) out.n[k] = n[k];
  out.r[0] = 1; out.r[1] = s0; out.r[2] = s1; out.r[3] = 1;
  out.c[0] = std::move(U0);
  out.c[1] = std::move(U1);
  out.c[2] = std::move(C1);
  return true;
}

int column_basis(Context& ctx, const double* C, int m, int L, double delta, DBuf& U) {
  TTIGA_CHECK(m >= L && L > 0, TTIGA_E_ARG, "column_basis needs m >= L > 0");
  TruncSVD t = truncated_svd(ctx, C, m, L, delta);
  if (t.s == 0) return 0;
  U = std::move(t.U);
  return t.s;
}

void column_basis_batched(Context& ctx, int count, const double* C, long stride, int m, int L, const double* delta,
                          int* k, DBuf* U) {
  TTIGA_CHECK(m > L && L > 0 && count >= 1, TTIGA_E_ARG, "column_basis_batched needs m > L > 0");
  // the tall route of truncated_svd for every matrix at once: C_t = Q_t T_t (one TSQR launch per
  // tree level), Jacobi on the rows of T_t (one launch), the ranks (one host round trip), then
  // U_t = Q_t Ut_t; each problem runs the same kernels as alone, so the bases are the same bits
  const size_t cnt = count;
  DBuf Q(ctx.alloc, sizeof(double) * cnt * m * L), T(ctx.alloc, sizeof(double) * cnt * L * L);
  qr_tall_batched(ctx, count, C, stride, false, m, L, L, Q.d(), (long)m * L, T.d(), (long)L * L);
  DBuf Ut(ctx.alloc, sizeof(double) * cnt * L * L), V(ctx.alloc, sizeof(double) * cnt * L * L),
      S(ctx.alloc, sizeof(double) * cnt * L);
  svd_small_batched(ctx, count, T.d(), (long)L * L, true, L, L, L, V.d(), (long)L * L, S.d(), L, Ut.d(),
                    (long)L * L);
  trunc_ranks_sync(ctx, count, S.d(), L, L, delta, k, nullptr);
  for (int t = 0; t < count; ++t) {
    if (k[t] == 0) continue;
    U[t] = DBuf(ctx.alloc, sizeof(double) * (size_t)m * k[t]);
    gemm(ctx, false, false, m, k[t], L, 1.0, Q.d() + (size_t)t * m * L, L, 0, Ut.d() + (size_t)t * L * L, L, 0, 0.0,
         U[t].d(), k[t], 0);
  }
}

__global__ void k_gather_rows(const double* __restrict__ A, int k, const int* __restrict__ rows, int nr,
                              double* __restrict__ out) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)nr * k; e += (long)gridDim.x * blockDim.x)
    out[e] = A[(long)rows[e / k] * k + e % k];
}

void scale_cols_inv(Context& ctx, const double* A, int m, int cols, const double* S, double* out) {
  DBuf inv(ctx.alloc, sizeof(double) * cols);
  hipLaunchKernelGGL(k_reciprocal, dim3((cols + 255) / 256), dim3(256), 0, ctx.stream, S, cols, inv.d());
  hipLaunchKernelGGL(k_scale_cols, dim3(grid_for((long)m * cols)), dim3(256), 0, ctx.stream, A, m, cols, inv.d(),
                     cols, out);
  TTIGA_HIP(hipGetLastError());
}

void gather_rows(Context& ctx, const double* A, int k, const int* rows, int nr, double* out) {
  if ((long)nr * k <= 0) return;
  hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((long)nr * k)), dim3(256), 0, ctx.stream, A, k, rows, nr, out);
  TTIGA_HIP(hipGetLastError());
}

// Values of a TT at grid points (i0[q], i1[q], i2[q]): one thread per point contracts
// G0[i0, :] G1[:, i1, :] G2[:, i2].
__global__ void k_tt_eval(int r1, int r2, int n1, int n2, const double* __restrict__ G0,
                          const double* __restrict__ G1, const double* __restrict__ G2, long count,
                          const int* __restrict__ i0, const int* __restrict__ i1, const int* __restrict__ i2,
                          double* __restrict__ out) {
  for (long q = blockIdx.x * (long)blockDim.x + threadIdx.x; q < count; q += (long)gridDim.x * blockDim.x) {
    const double* g0 = G0 + (long)i0[q] * r1;
    double v = 0.0;
    for (int b = 0; b < r2; ++b) {
      double t = 0.0;
      for (int a = 0; a < r1; ++a) t += g0[a] * G1[((long)a * n1 + i1[q]) * r2 + b];
      v += t * G2[(long)b * n2 + i2[q]];
    }
    out[q] = v;
  }
}

void tt_eval_points(Context& ctx, const TT& x, long count, const int* i0, const int* i1, const int* i2,
                    double* out) {
  if (count <= 0) return;
  if (x.zero()) {
    fill(ctx, out, count, 0.0);
    return;
  }
  hipLaunchKernelGGL(k_tt_eval, dim3(grid_for(count)), dim3(256), 0, ctx.stream, x.r[1], x.r[2], x.n[1], x.n[2],
                     x.c[0].d(), x.c[1].d(), x.c[2].d(), count, i0, i1, i2, out);
  TTIGA_HIP(hipGetLastError());
}

// Randomised projection of x onto ranks (l1, l2): Gaussian TT Omega with cores
// O2 (l1 x n2 x l2), O3 (l2 x n3); right interfaces W3 = X3 O3^T, W2 = (X2 x3 W3) O2^T;
// then left to right Q1 = orth(X1 W2), Z2 = (Q1^T X1) X2, Q2 = orth(Z2 W3), last core
// (Q2^T Z2) X3.  The result is left-orthogonal with ranks (l1, l2).
static void tt_sketch_project(Context& ctx, const TT& x, int l1, int l2, TT& y) {
  const int n0 = x.n[0], n1 = x.n[1], n2 = x.n[2], R1 = x.r[1], R2 = x.r[2];
  DBuf O2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * l2), O3(ctx.alloc, sizeof(double) * (size_t)l2 * n2);
  gaussian_fill(ctx, O2.d(), (long)l1 * n1 * l2);
  gaussian_fill(ctx, O3.d(), (long)l2 * n2);
  DBuf W3(ctx.alloc, sizeof(double) * (size_t)R2 * l2);
  gemm(ctx, false, true, R2, l2, n2, 1.0, x.c[2].d(), n2, 0, O3.d(), n2, 0, 0.0, W3.d(), l2, 0);
  DBuf T(ctx.alloc, sizeof(double) * (size_t)R1 * n1 * l2);
  gemm(ctx, false, false, R1 * n1, l2, R2, 1.0, x.c[1].d(), R2, 0, W3.d(), l2, 0, 0.0, T.d(), l2, 0);
  DBuf W2(ctx.alloc, sizeof(double) * (size_t)R1 * l1);
  gemm(ctx, false, true, R1, l1, n1 * l2, 1.0, T.d(), (long)n1 * l2, 0, O2.d(), (long)n1 * l2, 0, 0.0,
       W2.d(), l1, 0);
  DBuf Y1(ctx.alloc, sizeof(double) * (size_t)n0 * l1);
  gemm(ctx, false, false, n0, l1, R1, 1.0, x.c[0].d(), R1, 0, W2.d(), l1, 0, 0.0, Y1.d(), l1, 0);
  DBuf Q1(ctx.alloc, sizeof(double) * (size_t)n0 * l1), Rq(ctx.alloc, sizeof(double) * (size_t)l1 * l1);
  qr_tall(ctx, Y1.d(), false, n0, l1, l1, Q1.d(), Rq.d());
  DBuf M1(ctx.alloc, sizeof(double) * (size_t)l1 * R1);
  gemm(ctx, true, false, l1, R1, n0, 1.0, Q1.d(), l1, 0, x.c[0].d(), R1, 0, 0.0, M1.d(), R1, 0);
  DBuf Z2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * R2);
  gemm(ctx, false, false, l1, n1 * R2, R1, 1.0, M1.d(), R1, 0, x.c[1].d(), (long)n1 * R2, 0, 0.0, Z2.d(),
       (long)n1 * R2, 0);
  DBuf Y2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * l2);
  gemm(ctx, false, false, l1 * n1, l2, R2, 1.0, Z2.d(), R2, 0, W3.d(), l2, 0, 0.0, Y2.d(), l2, 0);
  DBuf Q2(ctx.alloc, sizeof(double) * (size_t)l1 * n1 * l2), Rq2(ctx.alloc, sizeof(double) * (size_t)l2 * l2);
  qr_tall(ctx, Y2.d(), false, l1 * n1, l2, l2, Q2.d(), Rq2.d());
  DBuf M2(ctx.alloc, sizeof(double) * (size_t)l2 * R2);
  gemm(ctx, true, false, l2, R2, l1 * n1, 1.0, Q2.d(), l2, 0, Z2.d(), R2, 0, 0.0, M2.d(), R2, 0);
  DBuf C3(ctx.alloc, sizeof(double) * (size_t)l2 * n2);
  gemm(ctx, false, false, l2, n2, R2, 1.0, M2.d(), R2, 0, x.c[2].d(), n2, 0, 0.0, C3.d(), n2, 0);
  y.n[0] = n0; y.n[1] = n1; y.n[2] = n2;
  y.r[0] = 1; y.r[1] = l1; y.r[2] = l2; y.r[3] = 1;
  y.c[0] = std::move(Q1);
  y.c[1] = std::move(Q2);
  y.c[2] = std::move(C3);
}

static bool trace_rounding() {
  static const bool v = [] {
    const char* e = std::getenv("TTIGA_TRACE_ROUND");
    return e && e[0] == '1';
  }();
  return v;
}

void tt_round_auto(Context& ctx, TT& x, double eps_rel, int max_rank, int& hint) {
  if (x.zero()) return;
  int l = std::max(hint, 1) + 10;
  const int in1 = x.r[1], in2 = x.r[2];
  while (true) {
    const int l1 = std::min(l, std::min(x.r[1], x.n[0]));
    const int l2 = std::min(l, std::min(x.r[2], x.n[2]));
    // trains already near the sketch width, or sketches that would not shrink them:
    // deterministic rounding
    if ((x.r[1] <= l1 + 6 && x.r[2] <= l2 + 6) || l1 * x.n[1] < l2) {
      tt_round(ctx, x, eps_rel, -1.0, max_rank);
      hint = x.zero() ? 1 : std::max(x.r[1], x.r[2]);
      if (trace_rounding())
        std::fprintf(stderr, "[round] det in (%d,%d) l %d eps %.1e -> (%d,%d)\n", in1, in2, l, eps_rel, x.r[1], x.r[2]);
      return;
    }
    TT y;
    tt_sketch_project(ctx, x, l1, l2, y);
    tt_round(ctx, y, eps_rel, -1.0, max_rank, nullptr, true);
    if (y.zero()) {
      x.set_zero(x.n);
      return;
    }
    const bool sat1 = y.r[1] > l1 - 4 && l1 < std::min(x.r[1], x.n[0]);
    const bool sat2 = y.r[2] > l2 - 4 && l2 < std::min(x.r[2], x.n[2]);
    if (sat1 || sat2) {  // the sketch may have cut real directions: widen it
      l += 12;
      continue;
    }
    hint = std::max(y.r[1], y.r[2]);
    if (trace_rounding())
      std::fprintf(stderr, "[round] rnd in (%d,%d) l (%d,%d) eps %.1e -> (%d,%d)\n", in1, in2, l1, l2, eps_rel, y.r[1], y.r[2]);
    x = std::move(y);
    return;
  }
}

void tt_mode_product(Context& ctx, TT& x, int d, const double* Mat, bool trans) {
  if (x.zero()) return;
  const int ra = x.r[d], n = x.n[d], rb = x.r[d + 1];
  DBuf out(ctx.alloc, sizeof(double) * x.core_elems(d));
  // out[a] (n x rb) = op(Mat) (n x n) * X[a] (n x rb), batched over a
  gemm_c(ctx, false, trans, false, n, rb, n, 1.0, Mat, n, 0, x.c[d].d(), rb, (long)n * rb, 0.0, out.d(), rb,
       (long)n * rb, ra);
  x.c[d] = std::move(out);
}

}  // namespace ttiga
