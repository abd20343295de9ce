// Dense FP64 linear algebra for TT contractions and TT-rounding on gfx950.
//
//  * qr_tall: Householder QR as a tree over row blocks (TSQR), each block
//    factored in LDS by one workgroup; exact orthogonality also for the
//    rank-deficient unfoldings that TT sums produce.
//  * svd_small: one-sided (Hestenes) Jacobi in a single workgroup, round-robin
//    pair ordering so every wave rotates a disjoint column pair each round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "runtime.hpp"

namespace ttiga {

// ------------------------------------------------------- Householder TSQR
// Householder QR of a tall m x c matrix as a tree (TSQR): the rows are split into
// nb blocks of at least 2c rows; each workgroup factors its block in LDS
// (reflectors H_j = I - tau_j v_j v_j^T, v_j[j] = 1), the c x c R factors are
// stacked and factored again until one block is left.  The thin Q is then built
// top-down: each block applies its reflectors to [Q_parent slice; 0].
// Work arrays are column-major W[j * ldw + i] so a column update is contiguous.

// Lane moves within rows of 16 lanes by DPP (a VALU operand modifier, a few cycles) instead
// of LDS permutes; a double moves as its two 32-bit halves.  Controls (gfx9 encoding):
// quad_perm [2,3,0,1] 0x4E and [1,0,3,2] 0xB1 (partner lane^2 and lane^1), row_ror:8 0x128
// (lane^8 within the row), row_mirror 0x140 (i <-> 15-i), row_half_mirror 0x141 (i <-> 7-i).
template <int kCtrl>
__device__ inline double dpp_f64(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffu), kCtrl, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), kCtrl, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sum over aligned groups of G lanes (G = 8 or 16), every lane of a group receiving it:
// the mirrors pair lane i with its reflection, the quad permutations finish the group.
template <int G>
__device__ inline double group_sum(double v) {
  if (G >= 16) v += dpp_f64<0x140>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0xB1>(v);
  return v;
}

__device__ inline double wave_sum(double v) {
  v = group_sum<16>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

__device__ inline double readlane_f64(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffu), src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Sums of eight per-lane partials d[0..7] over the 64 lanes of a wave.  Three exchange
// steps (lane offsets 32, 16, 8) each send half of the values a lane still carries to
// its partner and add the half received, so a lane ends with one column, (lane >> 3) & 7;
// offsets 4, 2, 1 finish that column's sum, and the eight totals are read from lanes 8q.
// Three LDS permutes and a few DPP moves instead of the forty-eight shuffles of eight
// separate butterflies.
__device__ inline void wave_sum8(double d[8]) {
  const int lane = threadIdx.x & 63;
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0, h3 = (lane & 8) != 0;
  double e[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double keep = h5 ? d[q + 4] : d[q], send = h5 ? d[q] : d[q + 4];
    e[q] = keep + __shfl_xor(send, 32, 64);
  }
  double f[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double keep = h4 ? e[q + 2] : e[q], send = h4 ? e[q] : e[q + 2];
    f[q] = keep + __shfl_xor(send, 16, 64);
  }
  double g = (h3 ? f[1] : f[0]) + dpp_f64<0x128>(h3 ? f[0] : f[1]);
  g = group_sum<8>(g);
#pragma unroll
  for (int q = 0; q < 8; ++q) d[q] = readlane_f64(g, 8 * q);
}


// col[q][i] -= f[q] * v[i] for q < NQ and the rows i = i0, i0 + 64, ... < nr of one lane:
// one pass over the rows for all columns of a batch, so the loads of different columns
// overlap.
template <int NQ>
__device__ inline void update_batch(double* const* col, const double* f, const double* v, int i0, int nr) {
  for (int i = i0; i < nr; i += 64) {
    const double x = v[i];
    double y[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) y[q] = col[q][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) col[q][i] = y[q] - f[q] * x;
  }
}

__device__ inline void update_batch_n(int nq, double* const* col, const double* f, const double* v, int i0,
                                      int nr) {
  switch (nq) {
    case 1: update_batch<1>(col, f, v, i0, nr); break;
    case 2: update_batch<2>(col, f, v, i0, nr); break;
    case 3: update_batch<3>(col, f, v, i0, nr); break;
    case 4: update_batch<4>(col, f, v, i0, nr); break;
    case 5: update_batch<5>(col, f, v, i0, nr); break;
    case 6: update_batch<6>(col, f, v, i0, nr); break;
    case 7: update_batch<7>(col, f, v, i0, nr); break;
    default: update_batch<8>(col, f, v, i0, nr); break;
  }
}

// d[q] += v[i] col[q][i] for q < NQ over the rows i = i0, i0 + 64, ... < nr of one lane; only
// the batch's real columns are read (a batch of a few columns would otherwise stream the
// aliased ones through LDS as well)
template <int NQ>
__device__ inline void dot_batch(double* const* col, const double* v, int i0, int nr, double* d) {
  for (int i = i0; i < nr; i += 64) {
    const double x = v[i];
    double y[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) y[q] = col[q][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) d[q] += x * y[q];
  }
}

__device__ inline void dot_batch_n(int nq, double* const* col, const double* v, int i0, int nr, double* d) {
  switch (nq) {
    case 1: dot_batch<1>(col, v, i0, nr, d); break;
    case 2: dot_batch<2>(col, v, i0, nr, d); break;
    case 3: dot_batch<3>(col, v, i0, nr, d); break;
    case 4: dot_batch<4>(col, v, i0, nr, d); break;
    case 5: dot_batch<5>(col, v, i0, nr, d); break;
    case 6: dot_batch<6>(col, v, i0, nr, d); break;
    case 7: dot_batch<7>(col, v, i0, nr, d); break;
    default: dot_batch<8>(col, v, i0, nr, d); break;
  }
}

// Column k of the block belongs to wave k % nwaves for the whole factorisation,
// so a reflector needs one barrier: the owner of column j forms v_j and tau_j,
// then every wave applies H_j to the columns it owns.
// (outer, inner) = (e / n_inner, e % n_inner) for e = e0, e0 + step, ...: one division at the
// start instead of a (64-bit) division per element of a flattened copy loop
struct FlatWalk {
  int outer, inner, d_out, d_in, n_in;
  __device__ FlatWalk(int e0, int step, int n_inner) : n_in(n_inner) {
    outer = e0 / n_inner;
    inner = e0 - outer * n_inner;
    d_out = step / n_inner;
    d_in = step - d_out * n_inner;
  }
  __device__ void next() {
    inner += d_in;
    outer += d_out;
    if (inner >= n_in) {
      inner -= n_in;
      ++outer;
    }
  }
};

template <bool kLds>
__global__ __launch_bounds__(1024) void k_hh_factor(int m, int c, const double* __restrict__ A,
                                                    long lda, int trans, int nb, int ldw,
                                                    double* __restrict__ V,
                                                    double* __restrict__ tau,
                                                    double* __restrict__ Rout,
                                                    double* __restrict__ gwork) {
  extern __shared__ double smem[];
  __shared__ double s_tau[1024];
  const int blk = blockIdx.x;
  const long r0 = (long)m * blk / nb, r1 = (long)m * (blk + 1) / nb;
  const int nr = (int)(r1 - r0);
  const int tid = threadIdx.x, lane = tid & 63, nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform within the wave
  // the storage is a template choice so LDS accesses compile to ds_* instructions
  double* W = kLds ? smem : gwork + (long)blk * ldw * c;
  if (trans)
    for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next())
      W[(long)w.outer * ldw + w.inner] = A[(long)w.outer * lda + r0 + w.inner];
  else
    for (FlatWalk w(tid, blockDim.x, c); w.outer < nr; w.next())
      W[(long)w.inner * ldw + w.outer] = A[(r0 + w.outer) * lda + w.inner];
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    double* wj = W + (long)j * ldw;
    if (wave == j % nwaves) {
      double ss = 0.0;
      for (int i = j + 1 + lane; i < nr; i += 64) ss += wj[i] * wj[i];
      ss = wave_sum(ss);
      const double alpha = wj[j];
      double t = 0.0, sc = 0.0, beta = alpha;
      if (ss != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + ss), alpha);
        t = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
      if (t != 0.0)
        for (int i = j + 1 + lane; i < nr; i += 64) wj[i] *= sc;
      if (lane == 0) {
        wj[j] = beta;
        s_tau[j] = t;
      }
    }
    __syncthreads();
    const double t = s_tau[j];
    if (t == 0.0) continue;
    // H_j on the owned columns k > j, eight at a time: the partial dot products are
    // formed first and reduced together.  Columns of a batch past c alias its first column
    // (read, never written), so the row loop has no per-column branches.
    const int k0 = j + 1 + ((wave - (j + 1) % nwaves + nwaves) % nwaves);
    for (int kb = k0; kb < c; kb += 8 * nwaves) {
      const int nq = min(8, (c - kb + nwaves - 1) / nwaves);
      double* col[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) col[q] = W + (long)(kb + (q < nq ? q : 0) * nwaves) * ldw;
      double d[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) d[q] = 0.0;
      dot_batch_n(nq, col, wj, j + 1 + lane, nr, d);
      wave_sum8(d);
      double f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = t * (d[q] + col[q][j]);
      if (lane == 0)
        for (int q = 0; q < nq; ++q) col[q][j] -= f[q];
      update_batch_n(nq, col, f, wj, j + 1 + lane, nr);
    }
  }
  __syncthreads();
  for (int j = tid; j < c; j += blockDim.x) tau[(long)blk * c + j] = s_tau[j];
  for (FlatWalk w(tid, blockDim.x, c); w.outer < c; w.next()) {
    const int j = w.outer, k = w.inner;
    Rout[(long)blk * c * c + (long)j * c + k] = (k >= j) ? W[(long)k * ldw + j] : 0.0;
  }
  double* Vb = V + r0 * c;
  for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next()) {
    const int j = w.outer, i = w.inner;
    Vb[(long)j * nr + i] = (i > j) ? W[(long)j * ldw + i] : (i == j ? 1.0 : 0.0);
  }
}

// Qout (m x c, row-major) = H_0 ... H_{c-1} [Qtop slice (c x c); 0] per block;
// Qtop == nullptr stands for the identity (the root of the tree).  Each wave owns
// columns k = wave, wave + nwaves, ... and applies all reflectors to them with no
// barrier; the reflectors are staged in LDS after the work columns when they fit.
template <bool kLds, bool kVLds>
__global__ __launch_bounds__(1024) void k_hh_apply(int m, int c, int nb, int ldw,
                                                   const double* __restrict__ V,
                                                   const double* __restrict__ tau,
                                                   const double* __restrict__ Qtop,
                                                   double* __restrict__ Qout,
                                                   double* __restrict__ gwork) {
  extern __shared__ double smem[];
  __shared__ double s_tau[1024];
  const int blk = blockIdx.x;
  const long r0 = (long)m * blk / nb, r1 = (long)m * (blk + 1) / nb;
  const int nr = (int)(r1 - r0);
  const int tid = threadIdx.x, lane = tid & 63, nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // uniform within the wave
  double* Y = kLds ? smem : gwork + (long)blk * ldw * c;
  const double* Vg = V + r0 * c;
  double* Vs = smem + (long)ldw * c;
  if (kVLds)
    for (long e = tid; e < (long)nr * c; e += blockDim.x) Vs[e] = Vg[e];
  const double* Vb = kVLds ? Vs : Vg;
  for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next()) {
    const int k = w.outer, i = w.inner;
    double v = 0.0;
    if (i < c) v = Qtop ? Qtop[((long)blk * c + i) * c + k] : (i == k ? 1.0 : 0.0);
    Y[(long)k * ldw + i] = v;
  }
  for (int j = tid; j < c; j += blockDim.x) s_tau[j] = tau[(long)blk * c + j];
  __syncthreads();
  // each wave applies all reflectors to its owned columns, eight columns at a time so the
  // eight dot-product reductions of one reflector overlap
  for (int kb = wave; kb < c; kb += 8 * nwaves) {
    const int nq = min(8, (c - kb + nwaves - 1) / nwaves);
    double* col[8];  // columns past c alias the batch's first (read, never written)
#pragma unroll
    for (int q = 0; q < 8; ++q) col[q] = Y + (long)(kb + (q < nq ? q : 0) * nwaves) * ldw;
    for (int j = c - 1; j >= 0; --j) {
      const double t = s_tau[j];
      if (t == 0.0) continue;
      const double* vj = Vb + (long)j * nr;
      double d[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) d[q] = 0.0;
      dot_batch_n(nq, col, vj, j + 1 + lane, nr, d);
      wave_sum8(d);
      double f[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) f[q] = t * (d[q] + col[q][j]);
      if (lane == 0)
        for (int q = 0; q < nq; ++q) col[q][j] -= f[q];
      update_batch_n(nq, col, f, vj, j + 1 + lane, nr);
    }
  }
  __syncthreads();
  for (FlatWalk w(tid, blockDim.x, c); w.outer < nr; w.next())
    Qout[(r0 + w.outer) * c + w.inner] = Y[(long)w.inner * ldw + w.outer];
}

// col[q][i] -= sum_k v[k][i] X[4 k + q] for q < NQ and the rows i = i0, i0 + 64, ... < nr of
// one lane: the update of a panel of four reflectors in compact WY form.
template <int NQ>
__device__ inline void update_panel(double* const* col, const double* X, const double* const* v, int i0, int nr) {
  for (int i = i0; i < nr; i += 64) {
    double vv[4], y[NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k) vv[k] = v[k][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) y[q] = col[q][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = y[q];
#pragma unroll
      for (int k = 0; k < 4; ++k) s -= vv[k] * X[4 * k + q];
      col[q][i] = s;
    }
  }
}

// w[4 k + q] += v[k][i] col[q][i] for q < NQ over the rows i = i0, i0 + 64, ... < nr of one
// lane: the 4 x NQ dot products of a panel with a batch of owned columns
template <int NQ>
__device__ inline void panel_dots(double* const* col, const double* const* v, int i0, int nr, double* w) {
  for (int i = i0; i < nr; i += 64) {
    double vv[4], x[NQ];
#pragma unroll
    for (int k = 0; k < 4; ++k) vv[k] = v[k][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) x[q] = col[q][i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q) w[4 * k + q] += vv[k] * x[q];
  }
}

__device__ inline void panel_dots_n(int nq, double* const* col, const double* const* v, int i0, int nr, double* w) {
  switch (nq) {
    case 1: panel_dots<1>(col, v, i0, nr, w); break;
    case 2: panel_dots<2>(col, v, i0, nr, w); break;
    case 3: panel_dots<3>(col, v, i0, nr, w); break;
    default: panel_dots<4>(col, v, i0, nr, w); break;
  }
}

__device__ inline void update_panel_n(int nq, double* const* col, const double* X, const double* const* v, int i0,
                                      int nr) {
  switch (nq) {
    case 1: update_panel<1>(col, X, v, i0, nr); break;
    case 2: update_panel<2>(col, X, v, i0, nr); break;
    case 3: update_panel<3>(col, X, v, i0, nr); break;
    default: update_panel<4>(col, X, v, i0, nr); break;
  }
}

// The same product as k_hh_apply with the reflectors taken four at a time in compact WY form
// (Schreiber and Van Loan): H_j0 ... H_j0+3 = I - V_p T_p V_p^T with T_p upper triangular,
// T_mm = tau_m and T[0:m, m] = -tau_m T[0:m, 0:m] (V_p^T V_p)[0:m, m].  A panel costs each
// batch of four owned columns one round of 4 x 4 dot products (rows from the panel's first diagonal on: the
// reflectors vanish above their diagonal), one reduction, a 4 x 4 triangular product and one
// fused update, instead of four dependent reflector steps.  The panel factors are formed
// first, one wave per panel, into Tg (16 doubles per panel, per block), then copied into the
// LDS that held tau (so c <= 256), where the update reads them entry by entry.  Panel columns
// past c alias the panel's first column with tau 0, which T turns into zero updates.
// Per-problem strides of a batched TSQR (blockIdx.y selects the problem; all zero for one).
struct QrStrides {
  long in = 0, v = 0, tau = 0, r = 0, work = 0, qtop = 0, qout = 0, tg = 0;
};

template <bool kLds, bool kVLds>
__global__ __launch_bounds__(1024) void k_hh_apply_wy(int m, int c, int nb, int ldw,
                                                      const double* __restrict__ V,
                                                      const double* __restrict__ tau,
                                                      const double* __restrict__ Qtop,
                                                      double* __restrict__ Qout,
                                                      double* __restrict__ gwork,
                                                      double* __restrict__ Tg, QrStrides bs) {
  extern __shared__ double smem[];
  __shared__ double s_tau[1024];
  const int blk = blockIdx.x;
  {
    const long b = blockIdx.y;
    V += b * bs.v;
    tau += b * bs.tau;
    if (Qtop) Qtop += b * bs.qtop;
    Qout += b * bs.qout;
    if (gwork) gwork += b * bs.work;
    Tg += b * bs.tg;
  }
  const long r0 = (long)m * blk / nb, r1 = (long)m * (blk + 1) / nb;
  const int nr = (int)(r1 - r0);
  const int tid = threadIdx.x, lane = tid & 63, nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* Y = kLds ? smem : gwork + (long)blk * ldw * c;
  const double* Vg = V + r0 * c;
  double* Vs = smem + (long)ldw * c;
  if (kVLds)
    for (long e = tid; e < (long)nr * c; e += blockDim.x) Vs[e] = Vg[e];
  const double* Vb = kVLds ? Vs : Vg;
  for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next()) {
    const int k = w.outer, i = w.inner;
    double v = 0.0;
    if (i < c) v = Qtop ? Qtop[((long)blk * c + i) * c + k] : (i == k ? 1.0 : 0.0);
    Y[(long)k * ldw + i] = v;
  }
  for (int j = tid; j < c; j += blockDim.x) s_tau[j] = tau[(long)blk * c + j];
  __syncthreads();
  const int np = (c + 3) / 4;
  double* Tb = Tg + (long)blk * np * 16;
  // panel factors
  for (int P = wave; P < np; P += nwaves) {
    const int j0 = 4 * P, bp = min(4, c - j0);
    const double* v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = Vb + (long)(j0 + (k < bp ? k : 0)) * nr;
    double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
    for (int i = j0 + lane; i < nr; i += 64) {
      const double x0 = v[0][i], x1 = v[1][i], x2 = v[2][i], x3 = v[3][i];
      g[0] += x0 * x1;
      g[1] += x0 * x2;
      g[2] += x0 * x3;
      g[3] += x1 * x2;
      g[4] += x1 * x3;
      g[5] += x2 * x3;
    }
    wave_sum8(g);
    if (lane == 0) {
      double tp[4], G[4][4] = {{0}}, T[4][4] = {{0}};
      for (int k = 0; k < 4; ++k) tp[k] = k < bp ? s_tau[j0 + k] : 0.0;
      G[0][1] = g[0];
      G[0][2] = g[1];
      G[0][3] = g[2];
      G[1][2] = g[3];
      G[1][3] = g[4];
      G[2][3] = g[5];
      for (int mm = 0; mm < 4; ++mm) {
        T[mm][mm] = tp[mm];
        for (int k = 0; k < mm; ++k) {
          double s = 0.0;
          for (int l = k; l < mm; ++l) s += T[k][l] * G[l][mm];
          T[k][mm] = -tp[mm] * s;
        }
      }
      for (int e = 0; e < 16; ++e) Tb[(long)P * 16 + e] = T[e / 4][e % 4];
    }
  }
  __syncthreads();
  double* Ts = s_tau;  // tau is no longer needed: the panel factors take its place
  for (int e = tid; e < np * 16; e += blockDim.x) Ts[e] = Tb[e];
  __syncthreads();
  // panels from the last to the first on each wave's owned columns, four at a time (sixteen
  // accumulators per lane keep the kernel within the registers of a 1024-thread block)
  for (int kb = wave; kb < c; kb += 4 * nwaves) {
    const int nq = min(4, (c - kb + nwaves - 1) / nwaves);
    double* col[4];  // columns past c alias the batch's first (read, never written)
#pragma unroll
    for (int q = 0; q < 4; ++q) col[q] = Y + (long)(kb + (q < nq ? q : 0) * nwaves) * ldw;
    for (int P = np - 1; P >= 0; --P) {
      const int j0 = 4 * P, bp = min(4, c - j0);
      const double* v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = Vb + (long)(j0 + (k < bp ? k : 0)) * nr;
      double w[16];  // w[4 k + q] = v_k . col_q
#pragma unroll
      for (int e = 0; e < 16; ++e) w[e] = 0.0;
      panel_dots_n(nq, col, v, j0 + lane, nr, w);
      wave_sum8(w);
      wave_sum8(w + 8);
      // X = T W in place (T upper triangular: row k uses rows k.. of W)
      const double* T = Ts + P * 16;
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double s = 0.0;
#pragma unroll
          for (int l = k; l < 4; ++l) s += T[k * 4 + l] * w[4 * l + q];
          w[4 * k + q] = s;
        }
      update_panel_n(nq, col, w, v, j0 + lane, nr);
    }
  }
  __syncthreads();
  for (FlatWalk w(tid, blockDim.x, c); w.outer < nr; w.next())
    Qout[(r0 + w.outer) * c + w.inner] = Y[(long)w.inner * ldw + w.outer];
}

// Orders the LDS accesses of one wave: stores issued before it are complete and visible
// to every lane of the wave (and to the compiler's alias analysis) before later loads.
__device__ inline void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// v_k[i] of a panel's reflectors k = 0..3 as stored in W (below the diagonal, the diagonal
// holding R): 0 above row j0 + k, 1 on it, the stored entry below
__device__ inline void panel_rows(const double* const* v, int j0, int i, double* vv) {
#pragma unroll
  for (int k = 0; k < 4; ++k) vv[k] = v[k][i];
  if (i < j0 + 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) vv[k] = i > j0 + k ? vv[k] : (i == j0 + k ? 1.0 : 0.0);
  }
}

// w[4 k + q] += v_k[i] col[q][i] over rows i = i0, i0 + 64, ... < nr (i0 >= j0)
template <int NQ>
__device__ inline void panel_dots_tri(double* const* col, const double* const* v, int j0, int i0, int nr,
                                      double* w) {
  for (int i = i0; i < nr; i += 64) {
    double vv[4], x[NQ];
    panel_rows(v, j0, i, vv);
#pragma unroll
    for (int q = 0; q < NQ; ++q) x[q] = col[q][i];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int q = 0; q < NQ; ++q) w[4 * k + q] += vv[k] * x[q];
  }
}

// col[q][i] -= sum_k v_k[i] X[4 k + q] over the same rows
template <int NQ>
__device__ inline void panel_update_tri(double* const* col, const double* X, const double* const* v, int j0,
                                        int i0, int nr) {
  for (int i = i0; i < nr; i += 64) {
    double vv[4], y[NQ];
    panel_rows(v, j0, i, vv);
#pragma unroll
    for (int q = 0; q < NQ; ++q) y[q] = col[q][i];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = y[q];
#pragma unroll
      for (int k = 0; k < 4; ++k) s -= vv[k] * X[4 * k + q];
      col[q][i] = s;
    }
  }
}

template <int NQ>
__device__ inline void panel_apply_tri(double* const* col, const double* T, const double* const* v, int j0,
                                       int i0, int nr) {
  double w[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) w[e] = 0.0;
  panel_dots_tri<NQ>(col, v, j0, i0, nr, w);
  wave_sum8(w);
  wave_sum8(w + 8);
  // X = T^T W in place, rows from the last (T^T is lower triangular: row k uses rows 0..k)
#pragma unroll
  for (int k = 3; k >= 0; --k)
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l <= k; ++l) s += T[l * 4 + k] * w[4 * l + q];
      w[4 * k + q] = s;
    }
  panel_update_tri<NQ>(col, w, v, j0, i0, nr);
}

// The Householder QR of each block that k_hh_factor computes (same reflectors, tau, R and V
// layout), blocked by panels of four columns.  Wave 0 factors the panel's columns one after
// another, each reflector applied at once to the panel's remaining columns, with only
// wave-level ordering between the steps, and forms the panel's compact WY factor T
// (H_j0 ... H_j0+3 = I - V T V^T, Schreiber and Van Loan).  After one barrier every wave
// applies H_j0+3 ... H_j0 = I - V T^T V^T to its owned trailing columns, four at a time.
// Two workgroup barriers per four columns instead of one per column: the column-at-a-time
// kernel is bound by the latency of its dependent steps, not by arithmetic or bandwidth.
template <bool kLds>
__global__ __launch_bounds__(1024) void k_hh_factor_wy(int m, int c, const double* __restrict__ A, long lda,
                                                       int trans, int nb, int ldw, double* __restrict__ V,
                                                       double* __restrict__ tau, double* __restrict__ Rout,
                                                       double* __restrict__ gwork, QrStrides bs) {
  extern __shared__ double smem[];
  __shared__ double s_tau[1024];
  __shared__ double s_T[16];
  const int blk = blockIdx.x;
  {
    const long b = blockIdx.y;
    A += b * bs.in;
    V += b * bs.v;
    tau += b * bs.tau;
    Rout += b * bs.r;
    if (gwork) gwork += b * bs.work;
  }
  const long r0 = (long)m * blk / nb, r1 = (long)m * (blk + 1) / nb;
  const int nr = (int)(r1 - r0);
  const int tid = threadIdx.x, lane = tid & 63, nwaves = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* W = kLds ? smem : gwork + (long)blk * ldw * c;
  if (trans)
    for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next())
      W[(long)w.outer * ldw + w.inner] = A[(long)w.outer * lda + r0 + w.inner];
  else
    for (FlatWalk w(tid, blockDim.x, c); w.outer < nr; w.next())
      W[(long)w.inner * ldw + w.outer] = A[(r0 + w.outer) * lda + w.inner];
  __syncthreads();
  for (int j0 = 0; j0 < c; j0 += 4) {
    const int bp = min(4, c - j0), kt = j0 + bp;  // kt: first trailing column
    if (wave == 0) {
      for (int j = j0; j < kt; ++j) {
        double* wj = W + (long)j * ldw;
        double ss = 0.0;
        for (int i = j + 1 + lane; i < nr; i += 64) ss += wj[i] * wj[i];
        ss = wave_sum(ss);
        const double alpha = wj[j];
        double t = 0.0, sc = 0.0, beta = alpha;
        if (ss != 0.0) {
          beta = -copysign(sqrt(alpha * alpha + ss), alpha);
          t = (beta - alpha) / beta;
          sc = 1.0 / (alpha - beta);
        }
        if (t != 0.0)
          for (int i = j + 1 + lane; i < nr; i += 64) wj[i] *= sc;
        if (lane == 0) {
          wj[j] = beta;
          s_tau[j] = t;
        }
        wave_lds_fence();
        const int nq = kt - 1 - j;  // panel columns right of j
        if (t != 0.0 && nq > 0) {
          double* col[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) col[q] = W + (long)(j + 1 + (q < nq ? q : 0)) * ldw;
          double d[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) d[q] = 0.0;
          dot_batch_n(nq, col, wj, j + 1 + lane, nr, d);
          wave_sum8(d);
          double f[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) f[q] = t * (d[q] + col[q][j]);
          if (lane == 0)
            for (int q = 0; q < nq; ++q) col[q][j] -= f[q];
          update_batch_n(nq, col, f, wj, j + 1 + lane, nr);
          wave_lds_fence();
        }
      }
      if (kt < c) {  // T of the panel (bp == 4 whenever trailing columns remain)
        const double* v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = W + (long)(j0 + k) * ldw;
        double g[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // (0,1) (0,2) (0,3) (1,2) (1,3) (2,3)
        for (int i = j0 + lane; i < nr; i += 64) {
          double x[4];
          panel_rows(v, j0, i, x);
          g[0] += x[0] * x[1];
          g[1] += x[0] * x[2];
          g[2] += x[0] * x[3];
          g[3] += x[1] * x[2];
          g[4] += x[1] * x[3];
          g[5] += x[2] * x[3];
        }
        wave_sum8(g);
        if (lane == 0) {
          double G[4][4] = {{0}}, T[4][4] = {{0}};
          G[0][1] = g[0];
          G[0][2] = g[1];
          G[0][3] = g[2];
          G[1][2] = g[3];
          G[1][3] = g[4];
          G[2][3] = g[5];
          for (int mm = 0; mm < 4; ++mm) {
            const double tm = s_tau[j0 + mm];
            T[mm][mm] = tm;
            for (int k = 0; k < mm; ++k) {
              double acc = 0.0;
              for (int l = k; l < mm; ++l) acc += T[k][l] * G[l][mm];
              T[k][mm] = -tm * acc;
            }
          }
          for (int e = 0; e < 16; ++e) s_T[e] = T[e / 4][e % 4];
        }
      }
    }
    __syncthreads();
    if (kt < c) {
      double T[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) T[e] = s_T[e];
      const double* v[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) v[k] = W + (long)(j0 + k) * ldw;
      for (int kb = kt + wave; kb < c; kb += 4 * nwaves) {
        const int nq = min(4, (c - kb + nwaves - 1) / nwaves);
        double* col[4];  // columns past c alias the batch's first (read, never written)
#pragma unroll
        for (int q = 0; q < 4; ++q) col[q] = W + (long)(kb + (q < nq ? q : 0) * nwaves) * ldw;
        switch (nq) {
          case 1: panel_apply_tri<1>(col, T, v, j0, j0 + lane, nr); break;
          case 2: panel_apply_tri<2>(col, T, v, j0, j0 + lane, nr); break;
          case 3: panel_apply_tri<3>(col, T, v, j0, j0 + lane, nr); break;
          default: panel_apply_tri<4>(col, T, v, j0, j0 + lane, nr); break;
        }
      }
      __syncthreads();
    }
  }
  for (int j = tid; j < c; j += blockDim.x) tau[(long)blk * c + j] = s_tau[j];
  for (FlatWalk w(tid, blockDim.x, c); w.outer < c; w.next()) {
    const int j = w.outer, k = w.inner;
    Rout[(long)blk * c * c + (long)j * c + k] = (k >= j) ? W[(long)k * ldw + j] : 0.0;
  }
  double* Vb = V + r0 * c;
  for (FlatWalk w(tid, blockDim.x, nr); w.outer < c; w.next()) {
    const int j = w.outer, i = w.inner;
    Vb[(long)j * nr + i] = (i > j) ? W[(long)j * ldw + i] : (i == j ? 1.0 : 0.0);
  }
}

// Per-problem strides of a batched Jacobi SVD (blockIdx.x selects the problem; LDS mode only).
struct SvdStrides {
  long a = 0, u = 0, s = 0, v = 0;
};

template <int kMode>
__global__ void k_jacobi_svd(int m, int c, const double* __restrict__ A, int transA, long lda,
                             double* __restrict__ gwork, double* __restrict__ U, double* __restrict__ S,
                             double* __restrict__ V, int max_sweeps, int G, SvdStrides bs);

template <bool kLds>
__global__ void k_pchol(int r, const double* __restrict__ G, double tau_rel, double* __restrict__ L,
                        double* __restrict__ gwork, int* __restrict__ rank_out);

// static LDS of k_jacobi_svd (pair flags, permutation, singular values) and of the
// TSQR kernels (reflector scalars), with margin
constexpr int kJacobiStatic = 16384;
constexpr int kTsqrStatic = 8192 + 512;

// Dynamic LDS available to the TSQR kernels, in doubles: the device's per-workgroup
// limit (160 KiB on gfx950) minus their static shared variables; about 56 KiB when
// the larger opt-in is refused.  The Jacobi kernel gets the same budget minus its own
// larger static part.
static int lds_doubles() {
  // computed once (thread-safe static initialisation)
  static const int cap = [] {
    int dev = 0, bytes = 65536;
    TTIGA_HIP(hipGetDevice(&dev));
    if (hipDeviceGetAttribute(&bytes, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      bytes = 65536;
    int dyn = bytes - kJacobiStatic;  // the larger static part bounds both budgets
    if (bytes > 65536) {
      const bool ok =
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_factor<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_factor_wy<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_apply<true, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_apply<true, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_apply_wy<true, true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_hh_apply_wy<true, false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kTsqrStatic) == hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi_svd<2>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kJacobiStatic) ==
              hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_jacobi_svd<1>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kJacobiStatic) ==
              hipSuccess &&
          hipFuncSetAttribute(reinterpret_cast<const void*>(k_pchol<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, bytes - kJacobiStatic) ==
              hipSuccess;
      if (!ok) {
        (void)hipGetLastError();
        dyn = 65536 - kJacobiStatic;
      }
    }
    return dyn / 8;
  }();
  return cap;
}

// Dynamic LDS for a single-workgroup factorisation kernel: with TTIGA_EXCLUSIVE_CU=1 the
// whole budget is requested, so that no workgroup of another stream shares the compute unit
// (measurement switch for concurrent lanes).
static size_t lds_request(size_t need) {
  static const bool exclusive = [] {
    const char* e = std::getenv("TTIGA_EXCLUSIVE_CU");
    return e && e[0] == '1';
  }();
  return exclusive ? std::max(need, sizeof(double) * (size_t)lds_doubles()) : need;
}

// one wave per owned column up to 16 waves
static int qr_threads(int c) { return 64 * std::min(16, std::max(1, c)); }

void qr_tall(Context& ctx, const double* A, bool transA, int m, int c, long lda, double* Q,
             double* R) {
  qr_tall_batched(ctx, 1, A, 0, transA, m, c, lda, Q, 0, R, 0);
}

void qr_tall_batched(Context& ctx, int batch, const double* A, long sA, bool transA, int m, int c, long lda,
                     double* Q, long sQ, double* R, long sR) {
  TTIGA_CHECK(m >= c && c > 0, TTIGA_E_ARG, "qr_tall needs m >= c > 0");
  TTIGA_CHECK(batch >= 1 && batch <= 65535, TTIGA_E_ARG, "qr_tall: batch out of range");
  // TTIGA_QR_TRACE=1 prints the shape of every factorisation (for measurements)
  static const bool trace = std::getenv("TTIGA_QR_TRACE") != nullptr;
  if (trace) std::fprintf(stderr, "[qr-shape] m=%d c=%d batch=%d\n", m, c, batch);
  const int kLdsDoubles = lds_doubles();
  struct Level {
    int m, nb, ldw;
    bool lds, v_lds;
    DBuf V, tau, R, work;
  };
  std::vector<Level> lv;
  const double* in = A;
  long s_in = sA;
  bool tr = transA;
  long ld = lda;
  int mm = m;
  // blocks of at least 2c rows so every level at least halves the rows, as tall as the
  // LDS holds the work columns (each tree level costs a launch of c dependent steps, so
  // fewer, taller blocks win); the apply step keeps the reflectors in LDS only when
  // both fit and otherwise streams them from L2.  A batch of problems of one shape runs
  // every level as one launch (grid.y = problem).
  // panels of four columns (TTIGA_TSQR_FACTOR=column selects the column-at-a-time kernel, for
  // measurements; single problems only)
  static const bool per_column = [] {
    const char* e = std::getenv("TTIGA_TSQR_FACTOR");
    return e && std::strcmp(e, "column") == 0;
  }();
  const int rows_work = kLdsDoubles / c;
  const int rows_target = rows_work >= 2 * c ? rows_work : 4 * c;
  const size_t bt = (size_t)batch;
  while (true) {
    Level L;
    L.m = mm;
    L.nb = std::max(1, (mm + rows_target - 1) / rows_target);
    L.ldw = (mm + L.nb - 1) / L.nb;
    L.lds = (long)L.ldw * c <= kLdsDoubles;
    L.v_lds = 2L * L.ldw * c <= kLdsDoubles;
    L.V = DBuf(ctx.alloc, sizeof(double) * bt * mm * c);
    L.tau = DBuf(ctx.alloc, sizeof(double) * bt * L.nb * c);
    // the root of the tree writes its R straight to the caller's buffer
    if (L.nb > 1) L.R = DBuf(ctx.alloc, sizeof(double) * bt * L.nb * c * c);
    double* Rout = L.nb > 1 ? L.R.d() : R;
    if (!L.lds) L.work = DBuf(ctx.alloc, sizeof(double) * bt * L.nb * L.ldw * c);
    QrStrides bs;
    bs.in = s_in;
    bs.v = (long)mm * c;
    bs.tau = (long)L.nb * c;
    bs.r = L.nb > 1 ? (long)L.nb * c * c : sR;
    bs.work = (long)L.nb * L.ldw * c;
    const size_t shm = L.lds ? sizeof(double) * (size_t)L.ldw * c : 0;
    ProfScope prof(ctx, "tsqr_factor", batch * (2.0 * mm * c * c - L.nb * (2.0 / 3.0) * c * c * c),
                   batch * 8.0 * (2.0 * mm * c + (double)L.nb * c * c), c);
    const dim3 grid(L.nb, batch);
    if (per_column && batch == 1 && L.lds)
      hipLaunchKernelGGL(k_hh_factor<true>, grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream, mm, c, in, ld,
                         tr ? 1 : 0, L.nb, L.ldw, L.V.d(), L.tau.d(), Rout, nullptr);
    else if (per_column && batch == 1)
      hipLaunchKernelGGL(k_hh_factor<false>, grid, dim3(qr_threads(c)), 0, ctx.stream, mm, c, in, ld, tr ? 1 : 0,
                         L.nb, L.ldw, L.V.d(), L.tau.d(), Rout, L.work.d());
    else if (L.lds)
      hipLaunchKernelGGL(k_hh_factor_wy<true>, grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream, mm, c, in,
                         ld, tr ? 1 : 0, L.nb, L.ldw, L.V.d(), L.tau.d(), Rout, nullptr, bs);
    else
      hipLaunchKernelGGL(k_hh_factor_wy<false>, grid, dim3(qr_threads(c)), 0, ctx.stream, mm, c, in, ld, tr ? 1 : 0,
                         L.nb, L.ldw, L.V.d(), L.tau.d(), Rout, L.work.d(), bs);
    TTIGA_HIP(hipGetLastError());
    lv.push_back(std::move(L));
    const Level& last = lv.back();
    if (last.nb == 1) break;
    in = last.R.d();
    s_in = (long)last.nb * c * c;
    tr = false;
    ld = c;
    mm = last.nb * c;
  }
  // thin Q, top-down: reflectors four at a time in compact WY form (TTIGA_TSQR_APPLY=reflector
  // selects the one-reflector-at-a-time kernel, for measurements; single problems only)
  static const bool per_reflector = [] {
    const char* e = std::getenv("TTIGA_TSQR_APPLY");
    return e && std::strcmp(e, "reflector") == 0;
  }();
  TTIGA_CHECK(batch == 1 || c <= 256, TTIGA_E_ARG, "qr_tall: batched factorisations need c <= 256");
  DBuf qprev;
  long s_qprev = 0;
  for (int l = (int)lv.size() - 1; l >= 0; --l) {
    Level& L = lv[l];
    DBuf qout;
    double* dst = (l == 0) ? Q : (qout = DBuf(ctx.alloc, sizeof(double) * bt * L.m * c), qout.d());
    const size_t shm = L.lds ? (L.v_lds ? 2 : 1) * sizeof(double) * (size_t)L.ldw * c : 0;
    ProfScope prof(ctx, "tsqr_apply", batch * (4.0 * c * c * (double)L.m - 2.0 * c * c * c * L.nb),
                   batch * 8.0 * (2.0 * L.m * c + (double)L.nb * c * c), c);
    const dim3 grid(L.nb, batch);
    if ((per_reflector || c > 256) && batch == 1) {
      if (L.v_lds)
        hipLaunchKernelGGL((k_hh_apply<true, true>), grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream, L.m, c,
                           L.nb, L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, nullptr);
      else if (L.lds)
        hipLaunchKernelGGL((k_hh_apply<true, false>), grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream, L.m,
                           c, L.nb, L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, nullptr);
      else
        hipLaunchKernelGGL((k_hh_apply<false, false>), grid, dim3(qr_threads(c)), 0, ctx.stream, L.m, c, L.nb,
                           L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, L.work.d());
    } else {
      const long tg = (long)L.nb * ((c + 3) / 4) * 16;
      DBuf Tg(ctx.alloc, sizeof(double) * bt * tg);
      QrStrides bs;
      bs.v = (long)L.m * c;
      bs.tau = (long)L.nb * c;
      bs.qtop = s_qprev;
      bs.qout = l == 0 ? sQ : (long)L.m * c;
      bs.work = (long)L.nb * L.ldw * c;
      bs.tg = tg;
      if (L.v_lds)
        hipLaunchKernelGGL((k_hh_apply_wy<true, true>), grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream, L.m,
                           c, L.nb, L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, nullptr, Tg.d(), bs);
      else if (L.lds)
        hipLaunchKernelGGL((k_hh_apply_wy<true, false>), grid, dim3(qr_threads(c)), lds_request(shm), ctx.stream,
                           L.m, c, L.nb, L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, nullptr, Tg.d(), bs);
      else
        hipLaunchKernelGGL((k_hh_apply_wy<false, false>), grid, dim3(qr_threads(c)), 0, ctx.stream, L.m, c, L.nb,
                           L.ldw, L.V.d(), L.tau.d(), qprev.d(), dst, L.work.d(), Tg.d(), bs);
    }
    TTIGA_HIP(hipGetLastError());
    qprev = std::move(qout);
    s_qprev = (long)L.m * c;
  }
}

// ------------------------------------------------------------------ Cholesky
// One workgroup: upper Cholesky factor R of an SPD matrix G (c x c, row-major),
// R^T R = G, and its inverse Rinv (upper).  Used for the 1-D mass matrices of the
// preconditioner (a few hundred rows: the work arrays in global memory) and for the small
// frame matrices of the AMEn local preconditioner (kLds: R and Rinv built in LDS, c <= 56,
// then copied out; every step is a barrier, so LDS instead of global memory is most of the
// cost of a small factorisation).
template <bool kLds>
__global__ __launch_bounds__(256) void k_chol_inv(int c, const double* __restrict__ G,
                                                  double* __restrict__ Rg, double* __restrict__ Rinvg,
                                                  double* __restrict__ status) {
  extern __shared__ double sm[];
  double* R = kLds ? sm : Rg;
  double* Rinv = kLds ? sm + (long)c * c : Rinvg;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (long e = tid; e < (long)c * c; e += nt) {
    const int i = e / c, k = e % c;
    R[e] = (k < i) ? 0.0 : G[e];
  }
  __syncthreads();
  for (int j = 0; j < c; ++j) {
    if (tid == 0) {
      const double d = R[(long)j * c + j];
      if (!(d > 0.0)) status[0] = 1.0;  // not positive definite
      R[(long)j * c + j] = sqrt(fmax(d, 1e-300));
    }
    __syncthreads();
    const double d = R[(long)j * c + j];
    for (int k = j + 1 + tid; k < c; k += nt) R[(long)j * c + k] /= d;
    __syncthreads();
    const int rem = c - j - 1;
    for (long e = tid; e < (long)rem * rem; e += nt) {
      const int i = j + 1 + e / rem, k = j + 1 + e % rem;
      if (k >= i) R[(long)i * c + k] -= R[(long)j * c + i] * R[(long)j * c + k];
    }
    __syncthreads();
  }
  for (int j = tid; j < c; j += nt) {
    for (int i = j + 1; i < c; ++i) Rinv[(long)i * c + j] = 0.0;
    Rinv[(long)j * c + j] = 1.0 / R[(long)j * c + j];
    for (int i = j - 1; i >= 0; --i) {
      double acc = 0.0;
      for (int k = i + 1; k <= j; ++k) acc += R[(long)i * c + k] * Rinv[(long)k * c + j];
      Rinv[(long)i * c + j] = -acc / R[(long)i * c + i];
    }
  }
  if (kLds) {
    __syncthreads();
    for (long e = tid; e < (long)c * c; e += nt) {
      Rg[e] = R[e];
      Rinvg[e] = Rinv[e];
    }
  }
}

bool cholesky_inverse(Context& ctx, const double* G, int c, double* R, double* Rinv) {
  DBuf st(ctx.alloc, sizeof(double));
  fill(ctx, st.d(), 1, 0.0);
  if (c <= 56)
    hipLaunchKernelGGL(k_chol_inv<true>, dim3(1), dim3(256), 2 * sizeof(double) * c * c, ctx.stream, c, G, R, Rinv,
                       st.d());
  else
    hipLaunchKernelGGL(k_chol_inv<false>, dim3(1), dim3(256), 0, ctx.stream, c, G, R, Rinv, st.d());
  TTIGA_HIP(hipGetLastError());
  double* h = ctx.host(1);
  TTIGA_HIP(hipMemcpyAsync(h, st.d(), sizeof(double), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  return h[0] == 0.0;
}

// ------------------------------------------------- pivoted Cholesky (Gram route)
// G = L L^T for a symmetric positive semi-definite G (r x r, row-major), with L (r x k,
// row-major, leading dimension r) in the original index order: step j takes the largest
// remaining diagonal entry of the Schur complement as pivot p_j, so column j vanishes on
// the rows pivoted before it and no permutation has to be undone.  The factorisation stops
// at the first pivot at most tau_rel max_i G_ii (rank k = that step; every diagonal entry
// of the Schur complement left out is then below that level).  One workgroup: the working
// copy W in LDS (kLds) or in gwork; diagonal, pivot column and the list of remaining
// indices in LDS after W.
template <bool kLds>
__global__ __launch_bounds__(1024) void k_pchol(int r, const double* __restrict__ G, double tau_rel,
                                               double* __restrict__ L, double* __restrict__ gwork,
                                               int* __restrict__ rank_out) {
  extern __shared__ double sm[];
  double* W = kLds ? sm : gwork;
  double* dg = sm + (kLds ? (long)r * r : 0);
  double* lcol = dg + r;
  int* rem = reinterpret_cast<int*>(lcol + r);
  __shared__ double s_best[16];
  __shared__ int s_bi[16];
  __shared__ int s_p, s_stop;
  __shared__ double s_ljj, s_tau;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (long e = tid; e < (long)r * r; e += nt) {
    W[e] = G[e];
    L[e] = 0.0;
  }
  for (int i = tid; i < r; i += nt) rem[i] = i;
  __syncthreads();
  for (int i = tid; i < r; i += nt) dg[i] = W[(long)i * r + i];
  __syncthreads();
  // largest entry among dg[rem[0 .. nr)] (ties: the first position), into s_best / s_bi
  auto pick = [&](int nr) {
    double best = -INFINITY;
    int bi = nr;
    for (int t = tid; t < nr; t += nt) {
      const double v = dg[rem[t]];
      if (v > best) {
        best = v;
        bi = t;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) {
        best = ob;
        bi = oi;
      }
    }
    if (lane == 0) {
      s_best[wave] = best;
      s_bi[wave] = bi;
    }
  };
  int nr = r, k = r;
  for (int j = 0; j < r; ++j) {
    pick(nr);
    __syncthreads();
    if (tid == 0) {
      double best = s_best[0];
      int bi = s_bi[0];
      for (int w = 1; w < nw; ++w)
        if (s_best[w] > best || (s_best[w] == best && s_bi[w] < bi)) {
          best = s_best[w];
          bi = s_bi[w];
        }
      if (j == 0) s_tau = tau_rel * fmax(best, 0.0);
      if (!(best > s_tau) || bi >= nr) {
        s_stop = 1;
      } else {
        s_stop = 0;
        s_p = rem[bi];
        rem[bi] = rem[nr - 1];
        s_ljj = sqrt(best);
      }
    }
    __syncthreads();
    if (s_stop) {
      k = j;
      break;
    }
    const int p = s_p;
    const double ljj = s_ljj;
    nr -= 1;
    if (tid == 0) L[(long)p * r + j] = ljj;
    for (int t = tid; t < nr; t += nt) {
      const int a = rem[t];
      const double l = W[(long)a * r + p] / ljj;
      lcol[a] = l;
      L[(long)a * r + j] = l;
    }
    __syncthreads();
    // Schur complement on the remaining indices (a wave per row, lanes along the row)
    for (int ia = wave; ia < nr; ia += nw) {
      const int a = rem[ia];
      const double la = lcol[a];
      double* wa = W + (long)a * r;
      for (int ib = lane; ib < nr; ib += 64) {
        const int b = rem[ib];
        const double v = wa[b] - la * lcol[b];
        wa[b] = v;
        if (a == b) dg[a] = v;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    *rank_out = k;
    __threadfence_system();  // rank_out is host-mapped memory
  }
}

static bool pchol_lds_fit(int r) {
  return (long)r * r + 2L * r + (r + 1) / 2 <= (long)lds_doubles();
}

int pivoted_cholesky(Context& ctx, const double* G, int r, double* L, double tau_rel) {
  TTIGA_CHECK(r > 0 && r <= 1024, TTIGA_E_ARG, "pivoted_cholesky needs 0 < r <= 1024");
  const bool lds = pchol_lds_fit(r);
  DBuf work;
  if (!lds) work = DBuf(ctx.alloc, sizeof(double) * (size_t)r * r);
  int* rk = reinterpret_cast<int*>(ctx.host_device(1));
  const int* h = reinterpret_cast<const int*>(ctx.host_scratch);
  const size_t shm = sizeof(double) * ((lds ? (size_t)r * r : 0) + 2 * (size_t)r) + sizeof(int) * (size_t)r;
  ProfScope prof(ctx, "gram_cholesky", (double)r * r * r / 3.0, 8.0 * 2.0 * r * r, r);
  const int threads = 64 * std::min(16, std::max(1, (r + 63) / 64 * 4));
  if (lds)
    hipLaunchKernelGGL(k_pchol<true>, dim3(1), dim3(threads), lds_request(shm), ctx.stream, r, G, tau_rel, L, nullptr,
                       rk);
  else
    hipLaunchKernelGGL(k_pchol<false>, dim3(1), dim3(threads), shm, ctx.stream, r, G, tau_rel, L, work.d(),
                       rk);
  TTIGA_HIP(hipGetLastError());
  ctx.sync();
  return *h;
}

// ------------------------------------------------------------- Jacobi SVD

// One workgroup.  Ucol [c][m] and Vcol [c][c] are column-major work arrays.  kMode 2:
// both in LDS (dynamic shared memory of (m + c) c doubles); 1: Ucol in LDS (m c doubles),
// Vcol in gwork (the dot products of a round read only Ucol, so the critical path stays in
// LDS); 0: both in gwork.  With V null the right vectors are not accumulated.
template <int kMode>
__global__ __launch_bounds__(1024) void k_jacobi_svd(int m, int c, const double* __restrict__ A,
                                                     int transA, long lda, double* __restrict__ gwork,
                                                     double* __restrict__ U, double* __restrict__ S,
                                                     double* __restrict__ V, int max_sweeps, int G,
                                                     SvdStrides bs) {
  extern __shared__ double smem[];
  {
    const long b = blockIdx.x;
    A += b * bs.a;
    U += b * bs.u;
    S += b * bs.s;
    if (V) V += b * bs.v;
  }
  double* Ucol = kMode >= 1 ? smem : gwork;
  double* Vcol = kMode == 2 ? smem + (long)m * c : (kMode == 1 ? gwork : gwork + (long)m * c);
  const bool want_v = V != nullptr;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int nwaves = nt >> 6;
  __shared__ int s_rot;
  __shared__ int s_perm[1024];
  __shared__ double s_sig[1024];
  if (transA)
    for (FlatWalk w(tid, nt, m); w.outer < c; w.next())
      Ucol[(long)w.outer * m + w.inner] = A[(long)w.outer * lda + w.inner];
  else
    for (FlatWalk w(tid, nt, c); w.outer < m; w.next())
      Ucol[(long)w.inner * m + w.outer] = A[(long)w.outer * lda + w.inner];
  if (want_v)
    for (FlatWalk w(tid, nt, c); w.outer < c; w.next())
      Vcol[(long)w.outer * c + w.inner] = w.outer == w.inner ? 1.0 : 0.0;
  __shared__ double s_f2[16];
  {
    double f = 0.0;
    for (long e = tid; e < (long)m * c; e += nt) f += Ucol[e] * Ucol[e];
    f = wave_sum(f);
    if (lane == 0) s_f2[wave] = f;
  }
  __syncthreads();
  double f2 = 0.0;
  for (int w = 0; w < nwaves; ++w) f2 += s_f2[w];
  const int cp = (c + 1) & ~1;
  // a column pair is handled by a group of G lanes (8, 16, 32 or 64)
  const int gl = lane % G, grp = wave * (64 / G) + lane / G, ngroups = nwaves * (64 / G);
  // rotate a pair unless it is orthogonal to working accuracy (m u, the rounding level
  // of a length-m dot product), or both columns are below 1e-15 of the Frobenius norm
  // (they cannot affect any truncation decision)
  const double tol = 2.220446049250313e-16 * m, floor2 = 1e-30 * f2;
  // columns of at most kRegs G entries stay in registers from the dot products to the
  // rotation (one LDS read per round instead of two)
  constexpr int kRegs = 8;
  const bool in_regs = m <= G * kRegs;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int rnd = 0; rnd < cp - 1; ++rnd) {
      for (int k = grp; k < cp / 2; k += ngroups) {
        // circle method: slot 0 fixed, slots 1..cp-1 rotate by rnd (a - 1 + rnd and
        // b - 1 + rnd stay below 2 (cp - 1), so one subtraction wraps them)
        const int a = k, b = cp - 1 - k;
        int pa = 0;
        if (a != 0) {
          pa = a - 1 + rnd;
          if (pa >= cp - 1) pa -= cp - 1;
          pa += 1;
        }
        int pb = b - 1 + rnd;
        if (pb >= cp - 1) pb -= cp - 1;
        pb += 1;
        const int p = min(pa, pb), q = max(pa, pb);
        if (q >= c) continue;
        double* up = Ucol + (long)p * m;
        double* uq = Ucol + (long)q * m;
        double al = 0.0, be = 0.0, ga = 0.0;
        double xr[kRegs], yr[kRegs];
        if (in_regs) {
#pragma unroll
          for (int r = 0; r < kRegs; ++r) {
            const int i = gl + r * G;
            xr[r] = i < m ? up[i] : 0.0;
            yr[r] = i < m ? uq[i] : 0.0;
          }
#pragma unroll
          for (int r = 0; r < kRegs; ++r) {
            al += xr[r] * xr[r];
            be += yr[r] * yr[r];
            ga += xr[r] * yr[r];
          }
        } else {
#pragma unroll 4
          for (int i = gl; i < m; i += G) {
            const double x = up[i], y = uq[i];
            al += x * x;
            be += y * y;
            ga += x * y;
          }
        }
        if (G == 8) {
          al = group_sum<8>(al);
          be = group_sum<8>(be);
          ga = group_sum<8>(ga);
        } else {
          al = group_sum<16>(al);
          be = group_sum<16>(be);
          ga = group_sum<16>(ga);
          for (int off = 16; off < G; off <<= 1) {
            al += __shfl_xor(al, off, 64);
            be += __shfl_xor(be, off, 64);
            ga += __shfl_xor(ga, off, 64);
          }
        }
        const double pq = sqrt(al) * sqrt(be);
        if (ga == 0.0 || !(fabs(ga) > tol * pq) || pq <= floor2) continue;
        // the rotation annihilating ga: with d = be - al, h = sqrt(d^2 + 4 ga^2) and
        // u = |d| + h, tan = sign(d) 2 ga / u and 1 + tan^2 = 2 h u / u^2, so
        // cos = u / sqrt(2 h u) and sin = sign(d) 2 ga / sqrt(2 h u) (three dependent
        // roots/reciprocals); d and 2 ga are first scaled by a power of two (exactly)
        // so that their squares cannot overflow
        double d = be - al, g2 = 2.0 * ga;
        const int ex = ilogb(fmax(fabs(d), fabs(g2)));
        d = ldexp(d, -ex);
        g2 = ldexp(g2, -ex);
        const double h = sqrt(d * d + g2 * g2);
        const double u = fabs(d) + h;
        const double rw = rsqrt(2.0 * h * u);
        const double cs = u * rw, sn = copysign(1.0, d) * g2 * rw;
        if (in_regs) {
#pragma unroll
          for (int r = 0; r < kRegs; ++r) {
            const int i = gl + r * G;
            if (i < m) {
              up[i] = cs * xr[r] - sn * yr[r];
              uq[i] = sn * xr[r] + cs * yr[r];
            }
          }
        } else {
          for (int i = gl; i < m; i += G) {
            const double x = up[i], y = uq[i];
            up[i] = cs * x - sn * y;
            uq[i] = sn * x + cs * y;
          }
        }
        if (want_v) {
          double* vp = Vcol + (long)p * c;
          double* vq = Vcol + (long)q * c;
          for (int i = gl; i < c; i += G) {
            const double x = vp[i], y = vq[i];
            vp[i] = cs * x - sn * y;
            vq[i] = sn * x + cs * y;
          }
        }
        if (gl == 0) s_rot = 1;
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
    __syncthreads();
  }
  // singular values = column norms
  for (int j = wave; j < c; j += nwaves) {
    double s = 0.0;
    for (int i = lane; i < m; i += 64) s += Ucol[(long)j * m + i] * Ucol[(long)j * m + i];
    s = wave_sum(s);
    if (lane == 0) s_sig[j] = sqrt(s);
  }
  __syncthreads();
  // descending order by ranking (ties keep index order): column j goes to the slot
  // counting the columns before it in that order
  for (int j = tid; j < c; j += nt) {
    const double sj = s_sig[j];
    int rank = 0;
    for (int k = 0; k < c; ++k) {
      const double sk = s_sig[k];
      rank += (sk > sj || (sk == sj && k < j)) ? 1 : 0;
    }
    s_perm[rank] = j;
  }
  __syncthreads();
  for (int j = tid; j < c; j += nt) S[j] = s_sig[s_perm[j]];
  for (FlatWalk w(tid, nt, c); w.outer < m; w.next()) {
    const int i = w.outer, jj = w.inner;
    const long e = (long)i * c + jj;
    const int j = s_perm[jj];
    const double sg = s_sig[j];
    U[e] = (sg > 0.0) ? Ucol[(long)j * m + i] / sg : 0.0;
  }
  if (want_v)
    for (FlatWalk w(tid, nt, c); w.outer < c; w.next())
      V[(long)w.outer * c + w.inner] = Vcol[(long)s_perm[w.inner] * c + w.outer];
}

// Interpolation rows of an n x k matrix Q with orthonormal columns: column-pivoted
// Gram-Schmidt on the rows of Q (QR with column pivoting of Q^T): step l takes the row
// with the largest residual norm and removes its direction from every row, so the k rows
// chosen span the column space as well as any greedy choice can (the selection of
// Q-DEIM).  One workgroup; W (n x k) is a global work copy; norms live in LDS.
__global__ __launch_bounds__(1024) void k_pivot_rows(int n, int k, const double* __restrict__ Q,
                                                     double* __restrict__ W, int* __restrict__ rows) {
  extern __shared__ double nrm[];  // n residual norms (negative once chosen)
  __shared__ double s_v[256];
  __shared__ double s_best[32];
  __shared__ int s_bi[32];
  __shared__ int s_p;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
  for (long e = tid; e < (long)n * k; e += nt) W[e] = Q[e];
  __syncthreads();
  for (int i = tid; i < n; i += nt) {
    double ss = 0.0;
    for (int j = 0; j < k; ++j) ss += W[(long)i * k + j] * W[(long)i * k + j];
    nrm[i] = ss;
  }
  __syncthreads();
  for (int l = 0; l < k; ++l) {
    // pivot: largest residual norm (ties: smallest index)
    double best = -1.0;
    int bi = n;
    for (int i = tid; i < n; i += nt)
      if (nrm[i] > best) { best = nrm[i]; bi = i; }
    for (int off = 32; off > 0; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { s_best[wave] = best; s_bi[wave] = bi; }
    __syncthreads();
    if (tid == 0) {
      double b = s_best[0];
      int p = s_bi[0];
      for (int w = 1; w < nw; ++w)
        if (s_best[w] > b || (s_best[w] == b && s_bi[w] < p)) { b = s_best[w]; p = s_bi[w]; }
      s_p = p;
      rows[l] = p;
    }
    __syncthreads();
    const int p = s_p;
    const double np_ = sqrt(fmax(nrm[p], 0.0));
    for (int j = tid; j < k; j += nt) s_v[j] = np_ > 0.0 ? W[(long)p * k + j] / np_ : 0.0;
    __syncthreads();
    for (int i = tid; i < n; i += nt) {
      if (nrm[i] < 0.0) continue;
      double cf = 0.0;
      for (int j = 0; j < k; ++j) cf += W[(long)i * k + j] * s_v[j];
      double ss = 0.0;
      for (int j = 0; j < k; ++j) {
        const double w = W[(long)i * k + j] - cf * s_v[j];
        W[(long)i * k + j] = w;
        ss += w * w;
      }
      nrm[i] = (i == p) ? -1.0 : ss;
    }
    __syncthreads();
  }
}

// The same selection for long bases (n > 6144 rows), spread over the device: one step is a
// launch that finds each block's largest residual norm, a one-block launch that takes the
// largest of those (ties: smallest index), records it and normalises its row into v, and a
// launch that removes v from every remaining row.  Each row is updated with the arithmetic of
// k_pivot_rows, so both pick the same rows.
__global__ void __launch_bounds__(256) k_piv_init(int n, int k, const double* __restrict__ Q, double* __restrict__ W,
                                                  double* __restrict__ nrm) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    double ss = 0.0;
    for (int j = 0; j < k; ++j) {
      const double w = Q[(long)i * k + j];
      W[(long)i * k + j] = w;
      ss += w * w;
    }
    nrm[i] = ss;
  }
}

__global__ void __launch_bounds__(256) k_piv_partial(int n, const double* __restrict__ nrm, double* __restrict__ pbest,
                                                     int* __restrict__ pidx) {
  __shared__ double s_b[4];
  __shared__ int s_i[4];
  double best = -1.0;
  int bi = n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256)
    if (nrm[i] > best) { best = nrm[i]; bi = i; }
  for (int off = 32; off > 0; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if ((threadIdx.x & 63) == 0) { s_b[threadIdx.x >> 6] = best; s_i[threadIdx.x >> 6] = bi; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < 4; ++w)
      if (s_b[w] > best || (s_b[w] == best && s_i[w] < bi)) { best = s_b[w]; bi = s_i[w]; }
    pbest[blockIdx.x] = best;
    pidx[blockIdx.x] = bi;
  }
}

__global__ void __launch_bounds__(256) k_piv_select(int nb, const double* __restrict__ pbest,
                                                    const int* __restrict__ pidx, int k, const double* __restrict__ W,
                                                    double* __restrict__ v, double* __restrict__ nrm,
                                                    int* __restrict__ rows, int l) {
  __shared__ int s_p;
  if (threadIdx.x == 0) {
    double b = -1.0;
    int p = 0x7fffffff;
    for (int q = 0; q < nb; ++q)
      if (pbest[q] > b || (pbest[q] == b && pidx[q] < p)) { b = pbest[q]; p = pidx[q]; }
    s_p = p;
    rows[l] = p;
  }
  __syncthreads();
  const int p = s_p;
  const double np_ = sqrt(fmax(nrm[p], 0.0));
  for (int j = threadIdx.x; j < k; j += 256) v[j] = np_ > 0.0 ? W[(long)p * k + j] / np_ : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) nrm[p] = -1.0;
}

__global__ void __launch_bounds__(256) k_piv_update(int n, int k, const double* __restrict__ v, double* __restrict__ W,
                                                    double* __restrict__ nrm) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    if (nrm[i] < 0.0) continue;
    double cf = 0.0;
    for (int j = 0; j < k; ++j) cf += W[(long)i * k + j] * v[j];
    double ss = 0.0;
    for (int j = 0; j < k; ++j) {
      const double w = W[(long)i * k + j] - cf * v[j];
      W[(long)i * k + j] = w;
      ss += w * w;
    }
    nrm[i] = ss;
  }
}

void pivot_rows(Context& ctx, const double* Q, int n, int k, int* rows) {
  TTIGA_CHECK(n > 0 && k > 0 && k <= 256 && k <= n, TTIGA_E_ARG, "pivot_rows: bad shape");
  DBuf W(ctx.alloc, sizeof(double) * (size_t)n * k);
  ProfScope prof(ctx, "pivot_rows", 4.0 * n * (double)k * k, 16.0 * n * (double)k * k);
  if (n <= 6144) {
    hipLaunchKernelGGL(k_pivot_rows, dim3(1), dim3(1024), sizeof(double) * n, ctx.stream, n, k, Q, W.d(), rows);
    TTIGA_HIP(hipGetLastError());
    return;
  }
  const int nb = std::min(1024, (n + 255) / 256);
  DBuf nrm(ctx.alloc, sizeof(double) * (size_t)n), v(ctx.alloc, sizeof(double) * k),
      pbest(ctx.alloc, sizeof(double) * nb), pidx(ctx.alloc, sizeof(int) * nb);
  hipLaunchKernelGGL(k_piv_init, dim3(nb), dim3(256), 0, ctx.stream, n, k, Q, W.d(), nrm.d());
  for (int l = 0; l < k; ++l) {
    hipLaunchKernelGGL(k_piv_partial, dim3(nb), dim3(256), 0, ctx.stream, n, nrm.d(), pbest.d(), pidx.as<int>());
    hipLaunchKernelGGL(k_piv_select, dim3(1), dim3(256), 0, ctx.stream, nb, pbest.d(), pidx.as<int>(), k, W.d(),
                       v.d(), nrm.d(), rows, l);
    hipLaunchKernelGGL(k_piv_update, dim3(nb), dim3(256), 0, ctx.stream, n, k, v.d(), W.d(), nrm.d());
  }
  TTIGA_HIP(hipGetLastError());
}

// Lanes per column pair of a Jacobi round: 16 (a DPP row) was fastest for every size
// measured (c = m = 24..256; 8, 32 and 64 lose up to 1.1x, 1.3x and 2.7x), 8 for columns
// of at most 16.  TTIGA_JACOBI_G (8, 16, 32 or 64) overrides the choice for measurements.
static int jacobi_group(int m) {
  static const int forced = [] {
    const char* e = std::getenv("TTIGA_JACOBI_G");
    const int g = e ? std::atoi(e) : 0;
    return (g == 8 || g == 16 || g == 32 || g == 64) ? g : 0;
  }();
  if (forced) return forced;
  return m <= 16 ? 8 : 16;
}

// Device results handed to the host through host-mapped memory: the system-scope fence
// writes them back past the device caches before the wave ends, so that they are in host
// memory by the time the host sees the kernel complete (a plain store need not be).
__global__ void k_publish(const double* __restrict__ src, double* __restrict__ dst, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
  __threadfence_system();
}

void publish_to_host(Context& ctx, const double* src, double* dst_mapped, int n) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, ctx.stream, src, dst_mapped, n);
  TTIGA_HIP(hipGetLastError());
}

// ---- one-sided Jacobi over the whole device, for matrices whose columns do not fit in LDS
// (c > 135: the 1-D eigenbases of long directions, wide R factors).  The columns of W = op(A)
// and of V live in global memory, column-major; one round of the circle ordering (c - 1 rounds
// of c / 2 disjoint pairs per sweep) is one launch with a workgroup per pair, which forms the
// pair's three inner products by a block reduction, rotates both columns of W and of V, and
// folds |w_i . w_j| / (|w_i| |w_j|) into the sweep's maximum, rotating when that exceeds u m (the
// tolerance of the single-workgroup kernel).  After each sweep one host read of that maximum ends
// the iteration once a sweep made no rotation (or after 40 sweeps).  A ranking kernel then writes
// s = |w_j| in descending order (ties by index), U = w_j / s_j and V in that order.
__global__ void k_jr_load(int m, int c, int cp, const double* __restrict__ A, int transA, long lda,
                          double* __restrict__ W, double* __restrict__ V) {
  const long total = (long)cp * m;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int j = (int)(e / m), i = (int)(e % m);
    W[e] = j < c ? (transA ? A[(long)j * lda + i] : A[(long)i * lda + j]) : 0.0;
  }
  if (V)
    for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)cp * cp; e += (long)gridDim.x * blockDim.x)
      V[e] = (e / cp == e % cp) ? 1.0 : 0.0;
}

// ||W||_F^2 into f2[0] (one workgroup): pairs whose norm product lies below 1e-30 of it are left
// alone, as in the single-workgroup kernel
__global__ void k_jr_frob(long total, const double* __restrict__ W, double* __restrict__ f2) {
  __shared__ double sh[256];
  double v = 0.0;
  for (long e = threadIdx.x; e < total; e += 256) v += W[e] * W[e];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) f2[0] = sh[0];
}

__global__ __launch_bounds__(256) void k_jr_round(int m, int cp, int r, double* __restrict__ W,
                                                  double* __restrict__ V, const double* __restrict__ f2,
                                                  unsigned long long* __restrict__ mx) {
  __shared__ double sh[3][256];
  __shared__ double cs_sn[2];
  const int pair = blockIdx.x;
  int i, j;
  if (pair == 0) {
    i = r;
    j = cp - 1;
  } else {
    i = (r + pair) % (cp - 1);
    j = (r - pair + cp - 1) % (cp - 1);
  }
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
  double* wi = W + (long)i * m;
  double* wj = W + (long)j * m;
  double a = 0.0, b = 0.0, g = 0.0;
  for (int e = threadIdx.x; e < m; e += 256) {
    const double x = wi[e], y = wj[e];
    a += x * x;
    b += y * y;
    g += x * y;
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = b;
  sh[2][threadIdx.x] = g;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o)
      for (int q = 0; q < 3; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a = sh[0][0];
    b = sh[1][0];
    g = sh[2][0];
    double cs = 1.0, sn = 0.0, meas = 0.0;
    const double pq = sqrt(a) * sqrt(b);
    if (g != 0.0 && pq > 1e-30 * f2[0]) meas = fabs(g) / pq;
    // rotate only above the tolerance of the single-workgroup kernel, u m
    if (meas > 2.220446049250313e-16 * m) {
      const double zeta = (b - a) / (2.0 * g);
      const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
      cs = 1.0 / sqrt(1.0 + t * t);
      sn = cs * t;
    }
    cs_sn[0] = cs;
    cs_sn[1] = sn;
    // non-negative doubles order as their bit patterns: the sweep's largest measure
    atomicMax(mx, (unsigned long long)__double_as_longlong(meas));
  }
  __syncthreads();
  const double cs = cs_sn[0], sn = cs_sn[1];
  if (sn == 0.0) return;
  for (int e = threadIdx.x; e < m; e += 256) {
    const double x = wi[e], y = wj[e];
    wi[e] = cs * x - sn * y;
    wj[e] = sn * x + cs * y;
  }
  if (V) {
    double* vi = V + (long)i * cp;
    double* vj = V + (long)j * cp;
    for (int e = threadIdx.x; e < cp; e += 256) {
      const double x = vi[e], y = vj[e];
      vi[e] = cs * x - sn * y;
      vj[e] = sn * x + cs * y;
    }
  }
}

__global__ void k_jr_norms(int m, int c, const double* __restrict__ W, double* __restrict__ nrm) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  double v = 0.0;
  for (int e = threadIdx.x; e < m; e += 256) v += W[(long)j * m + e] * W[(long)j * m + e];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) nrm[j] = sqrt(sh[0]);
}

// position of column j in descending order of the norms (ties: smaller index first), then
// s, U (m x c row-major) and V (c x c row-major) in that order
__global__ void k_jr_store(int m, int c, int cp, const double* __restrict__ W, const double* __restrict__ Vw,
                           const double* __restrict__ nrm, double* __restrict__ U, double* __restrict__ s,
                           double* __restrict__ V) {
  const int j = blockIdx.x;
  __shared__ int s_rank;
  if (threadIdx.x == 0) {
    int rk = 0;
    const double x = nrm[j];
    for (int k = 0; k < c; ++k) rk += (nrm[k] > x || (nrm[k] == x && k < j)) ? 1 : 0;
    s_rank = rk;
    s[rk] = x;
  }
  __syncthreads();
  const int rk = s_rank;
  const double x = nrm[j];
  const double inv = x > 0.0 ? 1.0 / x : 0.0;
  for (int e = threadIdx.x; e < m; e += blockDim.x) U[(long)e * c + rk] = W[(long)j * m + e] * inv;
  if (V)
    for (int e = threadIdx.x; e < c; e += blockDim.x) V[(long)e * c + rk] = Vw[(long)j * cp + e];
}

static void svd_rounds(Context& ctx, const double* A, bool transA, int m, int c, long lda, double* U, double* s,
                       double* V) {
  const int cp = c + (c & 1);  // an even count of columns (a zero column pads an odd one)
  const int pairs = cp / 2;
  DBuf W(ctx.alloc, sizeof(double) * (size_t)cp * m), Vw(ctx.alloc, V ? sizeof(double) * (size_t)cp * cp : 0),
      mx(ctx.alloc, sizeof(double)), f2(ctx.alloc, sizeof(double)), nrm(ctx.alloc, sizeof(double) * cp);
  hipLaunchKernelGGL(k_jr_load, dim3(grid_for((long)cp * m)), dim3(256), 0, ctx.stream, m, c, cp, A, transA ? 1 : 0,
                     lda, W.d(), V ? Vw.d() : nullptr);
  hipLaunchKernelGGL(k_jr_frob, dim3(1), dim3(256), 0, ctx.stream, (long)cp * m, W.d(), f2.d());
  double* h = ctx.host_device(1);
  for (int sweep = 0; sweep < 40; ++sweep) {
    fill(ctx, mx.d(), 1, 0.0);
    for (int r = 0; r < cp - 1; ++r) {
      hipLaunchKernelGGL(k_jr_round, dim3(pairs), dim3(256), 0, ctx.stream, m, cp, r, W.d(), V ? Vw.d() : nullptr,
                         f2.d(), reinterpret_cast<unsigned long long*>(mx.d()));
    }
    TTIGA_HIP(hipGetLastError());
    publish_to_host(ctx, mx.d(), h, 1);
    ctx.sync();
    if (!(ctx.host_scratch[0] > 2.220446049250313e-16 * m)) break;  // a sweep without rotations
  }
  hipLaunchKernelGGL(k_jr_norms, dim3(c), dim3(256), 0, ctx.stream, m, c, W.d(), nrm.d());
  hipLaunchKernelGGL(k_jr_store, dim3(c), dim3(256), 0, ctx.stream, m, c, cp, W.d(), V ? Vw.d() : nullptr, nrm.d(),
                     U, s, V);
  TTIGA_HIP(hipGetLastError());
}

void svd_small(Context& ctx, const double* A, bool transA, int m, int c, long lda, double* U,
               double* s, double* V, const char* prof_name) {
  TTIGA_CHECK(c > 0 && m >= c && c <= 1024, TTIGA_E_ARG, "svd_small needs 0 < c <= m, c <= 1024");
  static const bool trace = std::getenv("TTIGA_QR_TRACE") != nullptr;
  if (trace) std::fprintf(stderr, "[svd-shape] m=%d c=%d v=%d\n", m, c, V ? 1 : 0);
  const long uc = (long)m * c, vc = V ? (long)c * c : 0;
  const long cap = lds_doubles();
  const int mode = (uc + vc <= cap) ? 2 : (uc <= cap ? 1 : 0);
  if (mode == 0 && c > 135) {
    ProfScope prof(ctx, prof_name, 8.0 * 0.5 * c * (c - 1.0) * (12.0 * m + (V ? 6.0 * c : 0.0)),
                   8.0 * (2.0 * m * c + (V ? 2.0 * c * c : 0.0) + c), c);
    svd_rounds(ctx, A, transA, m, c, lda, U, s, V);
    return;
  }
  DBuf work;
  const long gneed = mode == 2 ? 0 : (mode == 1 ? vc : uc + vc);
  if (gneed > 0) work = DBuf(ctx.alloc, sizeof(double) * gneed);
  const int pairs = (c + 1) / 2;
  const int G = jacobi_group(m);
  // enough lane groups for all column pairs of a round, up to 16 waves
  const int threads = 64 * std::min(16, std::max(1, (pairs * G + 63) / 64));
  // counted at a nominal 8 sweeps of c(c-1)/2 pair rotations: 3 dots, U (and V) updates
  const double per_rot = 12.0 * m + (V ? 6.0 * c : 0.0);
  ProfScope prof(ctx, prof_name, 8.0 * 0.5 * c * (c - 1.0) * per_rot,
                 8.0 * (2.0 * m * c + (V ? 2.0 * c * c : 0.0) + c), c);
  const size_t lds_bytes = sizeof(double) * (mode == 2 ? uc + vc : (mode == 1 ? uc : 0));
  if (mode == 2)
    hipLaunchKernelGGL(k_jacobi_svd<2>, dim3(1), dim3(threads), lds_request(lds_bytes), ctx.stream, m, c, A,
                       transA ? 1 : 0, lda, nullptr, U, s, V, 40, G, SvdStrides());
  else if (mode == 1)
    hipLaunchKernelGGL(k_jacobi_svd<1>, dim3(1), dim3(threads), lds_request(lds_bytes), ctx.stream, m, c, A,
                       transA ? 1 : 0, lda, work.d(), U, s, V, 40, G, SvdStrides());
  else
    hipLaunchKernelGGL(k_jacobi_svd<0>, dim3(1), dim3(threads), 0, ctx.stream, m, c, A, transA ? 1 : 0, lda,
                       work.d(), U, s, V, 40, G, SvdStrides());
  TTIGA_HIP(hipGetLastError());
}

void svd_small_batched(Context& ctx, int batch, const double* A, long sA, bool transA, int m, int c, long lda,
                       double* U, long sU, double* s, long sS, double* V, long sV, const char* prof_name) {
  TTIGA_CHECK(c > 0 && m >= c && c <= 1024 && batch >= 1 && batch <= 65535, TTIGA_E_ARG,
              "svd_small_batched: bad shape");
  const long uc = (long)m * c, vc = V ? (long)c * c : 0;
  if (batch == 1 || uc + vc > lds_doubles()) {
    // one problem, or columns that do not fit in LDS: one launch per problem
    for (int b = 0; b < batch; ++b)
      svd_small(ctx, A + b * sA, transA, m, c, lda, U + b * sU, s + b * sS, V ? V + b * sV : nullptr, prof_name);
    return;
  }
  const int pairs = (c + 1) / 2;
  const int G = jacobi_group(m);
  const int threads = 64 * std::min(16, std::max(1, (pairs * G + 63) / 64));
  const double per_rot = 12.0 * m + (V ? 6.0 * c : 0.0);
  ProfScope prof(ctx, prof_name, batch * 8.0 * 0.5 * c * (c - 1.0) * per_rot,
                 batch * 8.0 * (2.0 * m * c + (V ? 2.0 * c * c : 0.0) + c), c);
  SvdStrides bs;
  bs.a = sA;
  bs.u = sU;
  bs.s = sS;
  bs.v = sV;
  hipLaunchKernelGGL(k_jacobi_svd<2>, dim3(batch), dim3(threads), lds_request(sizeof(double) * (uc + vc)), ctx.stream,
                     m, c, A, transA ? 1 : 0, lda, nullptr, U, s, V, 40, G, bs);
  TTIGA_HIP(hipGetLastError());
}

// ------------------------------------------------------------ small utilities
__global__ void k_trunc_rank(const double* __restrict__ s, int c, double eps_rel, double delta_abs,
                             double* __restrict__ out, long ss) {
  // one problem per block: problem b reads s + b ss and writes out[3 b .. 3 b + 2]
  if (threadIdx.x != 0) return;
  s += blockIdx.x * ss;
  out += 3L * blockIdx.x;
  double tot = 0.0;
  for (int i = 0; i < c; ++i) tot += s[i] * s[i];
  const double nrm = sqrt(tot);
  const double delta = (delta_abs >= 0.0) ? delta_abs : eps_rel * nrm / sqrt(2.0);
  // smallest r with ||s[r:]|| <= delta, accumulating the tail from the end
  int r = c;
  double tail = 0.0;
  for (int i = c - 1; i >= 0; --i) {
    const double t2 = tail + s[i] * s[i];
    if (sqrt(t2) <= delta) {
      tail = t2;
      r = i;
    } else {
      break;
    }
  }
  out[0] = (double)r;
  out[1] = nrm;
  out[2] = delta;
  __threadfence_system();  // out is host-mapped memory when the host reads the rank
}

int trunc_rank_sync(Context& ctx, const double* s, int c, double delta, double* norm_out) {
  // delta >= 0: absolute threshold; delta < 0: relative eps = -delta.
  double* hd = ctx.host_device(3);
  double* h = ctx.host_scratch;
  hipLaunchKernelGGL(k_trunc_rank, dim3(1), dim3(64), 0, ctx.stream, s, c,
                     delta < 0 ? -delta : 0.0, delta < 0 ? -1.0 : delta, hd, 0L);
  TTIGA_HIP(hipGetLastError());
  ctx.sync();
  if (norm_out) {
    norm_out[0] = h[1];
    norm_out[1] = h[2];
  }
  return (int)h[0];
}

void trunc_ranks_sync(Context& ctx, int batch, const double* s, long ss, int c, const double* delta, int* ranks,
                      double* norms) {
  double* hd = ctx.host_device(3 * (size_t)batch);
  double* h = ctx.host_scratch;
  // one launch per problem (the thresholds differ), one host round trip for all
  for (int b = 0; b < batch; ++b)
    hipLaunchKernelGGL(k_trunc_rank, dim3(1), dim3(64), 0, ctx.stream, s + b * ss, c,
                       delta[b] < 0 ? -delta[b] : 0.0, delta[b] < 0 ? -1.0 : delta[b], hd + 3L * b, 0L);
  TTIGA_HIP(hipGetLastError());
  ctx.sync();
  for (int b = 0; b < batch; ++b) {
    ranks[b] = (int)h[3 * b];
    if (norms) norms[b] = h[3 * b + 1];
  }
}

__global__ void k_fill(double* p, size_t n, double v) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    p[e] = v;
}

void fill(Context& ctx, double* p, size_t n, double v) {
  if (!n) return;
  hipLaunchKernelGGL(k_fill, dim3(grid_for((long)n)), dim3(256), 0, ctx.stream, p, n, v);
  TTIGA_HIP(hipGetLastError());
}

// A copy kernel rather than hipMemcpyAsync: one plain dispatch, no runtime memory-object
// lookups on the host (which serialise concurrent lanes), and the destination may be the
// device address of host staging memory.
__global__ void k_copy(double* __restrict__ dst, const double* __restrict__ src, size_t n) {
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n; e += (size_t)gridDim.x * blockDim.x)
    dst[e] = src[e];
}

void copy(Context& ctx, double* dst, const double* src, size_t n) {
  if (!n || dst == src) return;
  hipLaunchKernelGGL(k_copy, dim3(grid_for((long)n)), dim3(256), 0, ctx.stream, dst, src, n);
  TTIGA_HIP(hipGetLastError());
}

__global__ void k_sumsq_partial(const double* __restrict__ x, size_t n, double* __restrict__ part) {
  __shared__ double sh[256];
  double s = 0.0;
  for (size_t e = blockIdx.x * (size_t)blockDim.x + threadIdx.x; e < n;
       e += (size_t)gridDim.x * blockDim.x)
    s += x[e] * x[e];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ void k_sum_final(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[256];
  double s = 0.0;
  for (int e = threadIdx.x; e < n; e += blockDim.x) s += part[e];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

void sumsq_reduce(Context& ctx, const double* x, size_t n, double* out_dev) {
  const int blocks = (int)std::max<size_t>(1, std::min<size_t>((n + 255) / 256, 1024));
  DBuf part(ctx.alloc, sizeof(double) * blocks);
  hipLaunchKernelGGL(k_sumsq_partial, dim3(blocks), dim3(256), 0, ctx.stream, x, n, part.d());
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, ctx.stream, part.d(), blocks, out_dev);
  TTIGA_HIP(hipGetLastError());
}

}  // namespace ttiga
