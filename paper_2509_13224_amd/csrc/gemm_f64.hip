// FP64 GEMM for the TT contractions and TT-rounding products on gfx950.
//
// C[b] = alpha op(A[b]) op(B[b]) + beta C[b] with row-major operands.  One kernel,
// v_mfma_f64_16x16x4 on tiles of BM x BN (64x64, 128x64, 64x128, or the skinny 64x16 and
// 16x64) per workgroup of four 64-wide waves (2 x 2 on the square and wide tiles, 4 x 1 or
// 1 x 4 on the skinny ones, each wave owning a sub-tile of 16 x 16 blocks), the contraction staged
// through LDS 32 at a time.  The next K step's global loads are issued before the current
// step's MFMAs, so a workgroup keeps one step of loads in flight while it computes (the
// products here are mostly short contractions over a few hundred, where one exposed
// global round trip per step would dominate).  LDS layouts follow the global layout of
// each operand (row-major A is staged m-major, transposed A k-major, and the same for B),
// so the staging writes and the MFMA operand reads both hit distinct banks.
//
// Which tile and how many K splits a product takes is a pure function of its shape
// (gemm_plan: a table measured offline by tune_gemm.py, else a fixed rule): the same product
// runs the same code, with the same summation order, in every problem, process and mix.  K
// splits write partial tiles that a second kernel adds in a fixed order; there are no atomics.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdint>
#include <cstdlib>

#include "runtime.hpp"

namespace ttiga {

typedef double d4_t __attribute__((ext_vector_type(4)));

constexpr int kGK = 32;  // contraction step staged in LDS

// LDS row lengths: an m-major (n-major) tile has rows of kGK + 2 doubles; a k-major tile rows
// of BM + 16 (BN + 16).  Both make the 16-lane groups of an MFMA operand read (and a staging
// write) fall on distinct banks.
template <bool KMajor, int BX>
struct TileLds {
  static constexpr int kRows = KMajor ? kGK : BX;
  static constexpr int kLd = KMajor ? BX + 16 : kGK + 2;
  static constexpr int kElems = kRows * kLd;
  // element (x, k) of the tile, x along M (or N)
  __device__ static int at(int x, int k) { return KMajor ? k * kLd + x : x * kLd + k; }
};

template <bool TA, bool TB, int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_f64(int M, int N, int K, double alpha,
                                                  const double* __restrict__ A, long lda, long sA,
                                                  const double* __restrict__ B, long ldb, long sB,
                                                  double beta, double* __restrict__ C, long ldc,
                                                  long sC, int splits, int kchunk,
                                                  double* __restrict__ Cpart) {
  // A is staged k-major when it is stored transposed (K x M), m-major otherwise; B k-major
  // when stored K x N, n-major when transposed
  using LA = TileLds<TA, BM>;
  using LB = TileLds<!TB, BN>;
  constexpr int kLoadA = BM * kGK / 256;
  constexpr int kLoadB = BN * kGK / 256;
  // four waves: 2 x 2 on the square and wide tiles, stacked along the long side of the
  // skinny ones (64 x 16: four along M; 16 x 64: four along N), each owning MI x NI blocks
  // of 16 x 16
  constexpr int WN = BN == 16 ? 1 : (BM == 16 ? 4 : 2);
  constexpr int WM = 4 / WN;
  constexpr int MI = BM / (16 * WM), NI = BN / (16 * WN);
  static_assert(MI >= 1 && NI >= 1 && MI * 16 * WM == BM && NI * 16 * WN == BN, "tile shape");
  __shared__ double As[LA::kElems];
  __shared__ double Bs[LB::kElems];

  const int bz = blockIdx.z;
  const int batch = bz / splits, split = bz % splits;
  A += batch * sA;
  B += batch * sB;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave / WN) * (BM / WM), wn = (wave % WN) * (BN / WN);

  // (x, k) of the e-th element a thread stages: consecutive threads along the operand's
  // contiguous global index
  auto a_xk = [&](int e, int& x, int& k) {
    if (TA) { x = e % BM; k = e / BM; } else { k = e % kGK; x = e / kGK; }
  };
  auto b_xk = [&](int e, int& x, int& k) {
    if (TB) { k = e % kGK; x = e / kGK; } else { x = e % BN; k = e / BN; }
  };
  double ra[kLoadA], rb[kLoadB];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kLoadA; ++i) {
      int x, k;
      a_xk(tid + 256 * i, x, k);
      const int gm = m0 + x, gk = k0 + k;
      ra[i] = (gm < M && gk < kend) ? (TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kLoadB; ++i) {
      int x, k;
      b_xk(tid + 256 * i, x, k);
      const int gn = n0 + x, gk = k0 + k;
      rb[i] = (gn < N && gk < kend) ? (TB ? B[(long)gn * ldb + gk] : B[(long)gk * ldb + gn]) : 0.0;
    }
  };

  d4_t acc[MI][NI];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j) acc[i][j] = d4_t{0.0, 0.0, 0.0, 0.0};

  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    __syncthreads();  // the previous step's operand reads are done
#pragma unroll
    for (int i = 0; i < kLoadA; ++i) {
      int x, k;
      a_xk(tid + 256 * i, x, k);
      As[LA::at(x, k)] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < kLoadB; ++i) {
      int x, k;
      b_xk(tid + 256 * i, x, k);
      Bs[LB::at(x, k)] = rb[i];
    }
    __syncthreads();
    if (k0 + kGK < kend) load(k0 + kGK);  // in flight during this step's MFMAs
#pragma unroll
    for (int kk = 0; kk < kGK; kk += 4) {
      // operand layout of the 16x16x4 f64 MFMA: lane holds row (lane & 15) of A and column
      // (lane & 15) of B at contraction index lane >> 4
      const int kr = kk + (lane >> 4);
      double a[MI], b[NI];
#pragma unroll
      for (int i = 0; i < MI; ++i) a[i] = As[LA::at(wm + 16 * i + (lane & 15), kr)];
#pragma unroll
      for (int j = 0; j < NI; ++j) b[j] = Bs[LB::at(wn + 16 * j + (lane & 15), kr)];
#pragma unroll
      for (int i = 0; i < MI; ++i)
#pragma unroll
        for (int j = 0; j < NI; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // D layout of the 16x16x4 f64 MFMA: lane holds column (lane & 15) of rows (lane >> 4) + 4 v
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int j = 0; j < NI; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + 16 * i + (lane >> 4) + 4 * v;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (row < M && col < N) {
          const double s = acc[i][j][v];
          if (splits == 1) {
            double* c = C + batch * sC + (long)row * ldc + col;
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
          } else {
            Cpart[((long)bz * M + row) * N + col] = s;
          }
        }
      }
}

// ------------------------------------------------------------------ low precision
// The same product with the operands rounded to FP32 or BF16 (round to nearest even; BF16
// through FP32) as they are staged, MFMA in that type with FP32 accumulation
// (v_mfma_f32_16x16x4_f32, or v_mfma_f32_16x16x16_bf16 with four contraction indices per
// lane), FP64 in and out: the contractions of a mixed-precision solve whose FP64 result only
// needs the low type's accuracy.  64x64 tiles of four waves, the contraction staged 32 at a
// time with the next step's loads in flight, LDS in FP32 (BF16 values are exact in it).
__device__ inline float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return f;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

typedef float f4_t __attribute__((ext_vector_type(4)));
typedef short s4_t __attribute__((ext_vector_type(4)));

template <bool KMajor>
struct TileLdsF {
  static constexpr int kLd = KMajor ? 64 + 16 : kGK + 2;
  static constexpr int kElems = (KMajor ? kGK : 64) * kLd;
  __device__ static int at(int x, int k) { return KMajor ? k * kLd + x : x * kLd + k; }
};

template <bool TA, bool TB, int PREC>
__global__ __launch_bounds__(256) void k_gemm_lowp(int M, int N, int K, double alpha,
                                                   const double* __restrict__ A, long lda, long sA,
                                                   const double* __restrict__ B, long ldb, long sB,
                                                   double beta, double* __restrict__ C, long ldc, long sC,
                                                   int splits, int kchunk, double* __restrict__ Cpart) {
  using LA = TileLdsF<TA>;
  using LB = TileLdsF<!TB>;
  constexpr int kLoad = 64 * kGK / 256;
  __shared__ float As[LA::kElems];
  __shared__ float Bs[LB::kElems];
  const int bz = blockIdx.z;
  const int batch = bz / splits, split = bz % splits;
  A += batch * sA;
  B += batch * sB;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
  auto a_xk = [&](int e, int& x, int& k) {
    if (TA) { x = e % 64; k = e / 64; } else { k = e % kGK; x = e / kGK; }
  };
  auto b_xk = [&](int e, int& x, int& k) {
    if (TB) { k = e % kGK; x = e / kGK; } else { x = e % 64; k = e / 64; }
  };
  auto lowp = [](double v) {
    const float f = (float)v;
    return PREC == TTIGA_BF16 ? round_bf16(f) : f;
  };
  float ra[kLoad], rb[kLoad];
  auto load = [&](int k0) {
#pragma unroll
    for (int i = 0; i < kLoad; ++i) {
      int x, k;
      a_xk(tid + 256 * i, x, k);
      const int gm = m0 + x, gk = k0 + k;
      ra[i] = (gm < M && gk < kend) ? lowp(TA ? A[(long)gk * lda + gm] : A[(long)gm * lda + gk]) : 0.0f;
      b_xk(tid + 256 * i, x, k);
      const int gn = n0 + x, gk2 = k0 + k;
      rb[i] = (gn < N && gk2 < kend) ? lowp(TB ? B[(long)gn * ldb + gk2] : B[(long)gk2 * ldb + gn]) : 0.0f;
    }
  };
  f4_t acc[2][2];
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) acc[i][j] = f4_t{0.f, 0.f, 0.f, 0.f};
  if (kbeg < kend) load(kbeg);
  for (int k0 = kbeg; k0 < kend; k0 += kGK) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kLoad; ++i) {
      int x, k;
      a_xk(tid + 256 * i, x, k);
      As[LA::at(x, k)] = ra[i];
      b_xk(tid + 256 * i, x, k);
      Bs[LB::at(x, k)] = rb[i];
    }
    __syncthreads();
    if (k0 + kGK < kend) load(k0 + kGK);
    if constexpr (PREC == TTIGA_BF16) {
      // 16 contraction indices per MFMA: lane holds indices 4 (lane >> 4) + j, j = 0..3
#pragma unroll
      for (int kk = 0; kk < kGK; kk += 16) {
        s4_t a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            const int kr = kk + 4 * (lane >> 4) + j;
            a[i][j] = (short)(__float_as_uint(As[LA::at(wm + 16 * i + (lane & 15), kr)]) >> 16);
            b[i][j] = (short)(__float_as_uint(Bs[LB::at(wn + 16 * i + (lane & 15), kr)]) >> 16);
          }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kk = 0; kk < kGK; kk += 4) {
        const int kr = kk + (lane >> 4);
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a[i] = As[LA::at(wm + 16 * i + (lane & 15), kr)];
          b[i] = Bs[LB::at(wn + 16 * i + (lane & 15), kr)];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
  }
  // D layout of the FP32-accumulating 16x16 MFMAs: lane holds column (lane & 15) of rows
  // 4 (lane >> 4) + v
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + v;
        const int col = n0 + wn + 16 * j + (lane & 15);
        if (row < M && col < N) {
          const double s = (double)acc[i][j][v];
          if (splits == 1) {
            double* c = C + batch * sC + (long)row * ldc + col;
            *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
          } else {
            Cpart[((long)bz * M + row) * N + col] = s;
          }
        }
      }
}

// C = alpha * (sum of the K-split partial tiles, in split order) + beta C
__global__ void k_splitk_reduce(int M, int N, int splits, int batches, double alpha,
                                const double* __restrict__ Cpart, double beta, double* C, long ldc,
                                long sC) {
  const long total = (long)batches * M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e / ((long)M * N);
    const long rc = e % ((long)M * N);
    const int row = rc / N, col = rc % N;
    double s = 0.0;
    for (int k = 0; k < splits; ++k) s += Cpart[((long)(b * splits + k) * M + row) * N + col];
    double* c = C + b * sC + (long)row * ldc + col;
    *c = (beta == 0.0) ? alpha * s : alpha * s + beta * (*c);
  }
}

// Tuned plans: one entry per shape bucket that measured faster than the rule below, written
// by tune_gemm.py (offline, on the target GPU) and compiled in, so the choice is the same in
// every run and process.
namespace {
struct GemmEntry {
  int ta, tb, lm, ln, lk, batched, bm, bn, kchunk;
};
const GemmEntry kGemmTable[] = {
#include "gemm_table.inc"
    {-1, 0, 0, 0, 0, 0, 0, 0, 0}};
int ceil_log2(long v) {
  int b = 0;
  while ((1L << b) < v) ++b;
  return b;
}
}  // namespace

GemmPlan gemm_plan(bool ta, bool tb, int M, int N, int K, int batch) {
  GemmPlan g;
  const std::array<int, 6> key = {ta ? 1 : 0, tb ? 1 : 0, ceil_log2(M), ceil_log2(N), ceil_log2(K), batch > 1 ? 1 : 0};
  // the table is sorted by key (the tuner writes it so): binary search
  auto key_of = [](const GemmEntry& e) { return std::array<int, 6>{e.ta, e.tb, e.lm, e.ln, e.lk, e.batched}; };
  constexpr size_t kEntries = sizeof(kGemmTable) / sizeof(kGemmTable[0]) - 1;
  const GemmEntry* hit = std::lower_bound(kGemmTable, kGemmTable + kEntries, key,
                                          [&](const GemmEntry& e, const std::array<int, 6>& k) { return key_of(e) < k; });
  if (hit != kGemmTable + kEntries && key_of(*hit) == key) {
    const GemmEntry* e = hit;
    g.bm = e->bm;
    g.bn = e->bn;
    if (e->kchunk > 0 && e->kchunk < K) {
      g.kchunk = e->kchunk;
      g.splits = (K + g.kchunk - 1) / g.kchunk;
    } else {
      g.kchunk = K;
      g.splits = 1;
    }
    if (batch * g.splits <= 65535) return g;
    g = GemmPlan();
  }
  // otherwise a skinny 64 x 16 (16 x 64) tile when N (M) is at most 16, where a square tile
  // would spend almost all of its MFMA work on padding, or when 64 x 64 tiles would give fewer
  // than 512 workgroups (four times as many workgroups, each with a quarter of the MFMA work
  // per contraction step: on such grids the products are bound by latency, not by MFMA
  // throughput); else 64 x 64 (measured: the 128-wide tiles win only on a few shapes, which
  // the table lists).  Long contractions on grids below 256 workgroups are split (partials
  // summed by a second kernel in split order), at most 256 rows of K per split, about 512
  // workgroups.
  const long square_tiles = (long)((M + 63) / 64) * ((N + 63) / 64) * batch;
  if (N <= 16 && (M > 16 || M >= N)) {
    g.bm = 64;
    g.bn = 16;
  } else if (M <= 16) {
    g.bm = 16;
    g.bn = 64;
  } else if (square_tiles < 512) {
    g.bm = M >= N ? 64 : 16;
    g.bn = M >= N ? 16 : 64;
  }
  const long tiles = (long)((M + g.bm - 1) / g.bm) * ((N + g.bn - 1) / g.bn) * batch;
  if (tiles < 256 && K >= 320) {
    long s = std::min<long>((K + 255) / 256, std::max<long>(1, 512 / tiles));
    int kchunk = (int)((K + s - 1) / s);
    kchunk = (kchunk + kGK - 1) / kGK * kGK;
    g.splits = (K + kchunk - 1) / kchunk;
    g.kchunk = kchunk;
  } else {
    g.splits = 1;
    g.kchunk = K;
  }
  return g;
}

template <int BM, int BN>
static void launch_tile(Context& ctx, ProfScope& prof, const GemmPlan& g, bool ta, bool tb, int M, int N, int K,
                        double alpha, const double* A, long lda, long sA, const double* B, long ldb,
                        long sB, double beta, double* C, long ldc, long sC, int batch, double* part) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, batch * g.splits);
  dim3 block(256);
  hipEvent_t e0, e1;
  prof.kernel_events(&e0, &e1);
  // the plain launch unless timed (a stream under graph capture is never timed)
#define TTIGA_GEMM_LAUNCH(TA, TB)                                                                               \
  do {                                                                                                          \
    if (e0)                                                                                                     \
      hipExtLaunchKernelGGL((k_gemm_f64<TA, TB, BM, BN>), grid, block, 0, ctx.stream, e0, e1, 0, M, N, K, alpha, \
                            A, lda, sA, B, ldb, sB, beta, C, ldc, sC, g.splits, g.kchunk, part);                  \
    else                                                                                                        \
      hipLaunchKernelGGL((k_gemm_f64<TA, TB, BM, BN>), grid, block, 0, ctx.stream, M, N, K, alpha, A, lda, sA, B, \
                         ldb, sB, beta, C, ldc, sC, g.splits, g.kchunk, part);                                     \
  } while (0)
  if (!ta && !tb) TTIGA_GEMM_LAUNCH(false, false);
  else if (ta && !tb) TTIGA_GEMM_LAUNCH(true, false);
  else if (!ta && tb) TTIGA_GEMM_LAUNCH(false, true);
  else TTIGA_GEMM_LAUNCH(true, true);
#undef TTIGA_GEMM_LAUNCH
  TTIGA_HIP(hipGetLastError());
}

void gemm_planned(Context& ctx, const GemmPlan& g, bool ta, bool tb, int M, int N, int K, double alpha,
                  const double* A, long lda, long sA, const double* B, long ldb, long sB, double beta,
                  double* C, long ldc, long sC, int batch, double* part) {
  TTIGA_CHECK(batch <= 65535 / std::max(1, g.splits), TTIGA_E_ARG, "gemm: batch too large");
  // TTIGA_GEMM_TRACE=1 prints the shape of every product (the input of the offline tile tuner)
  static const bool trace = std::getenv("TTIGA_GEMM_TRACE") != nullptr;
  if (trace) std::fprintf(stderr, "[gemm-shape] ta=%d tb=%d M=%d N=%d K=%d batch=%d\n", ta, tb, M, N, K, batch);
  TTIGA_CHECK((M + g.bm - 1) / g.bm <= 65535, TTIGA_E_ARG, "gemm: M too large for the grid");
  // timed per kernel: most products here take a few microseconds
  ProfScope prof(ctx, "gemm_f64", 2.0 * M * N * (double)K * batch,
                 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N), -1, true);
  if (g.bm == 128) launch_tile<128, 64>(ctx, prof, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part);
  else if (g.bn == 128) launch_tile<64, 128>(ctx, prof, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part);
  else if (g.bn == 16) launch_tile<64, 16>(ctx, prof, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part);
  else if (g.bm == 16) launch_tile<16, 64>(ctx, prof, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part);
  else launch_tile<64, 64>(ctx, prof, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part);
  if (g.splits > 1) {
    const long total = (long)batch * M * N;
    hipEvent_t e0, e1;
    prof.kernel_events(&e0, &e1);
    if (e0)
      hipExtLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(total)), dim3(256), 0, ctx.stream, e0, e1, 0, M, N,
                            g.splits, batch, alpha, (const double*)part, beta, C, ldc, sC);
    else
      hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(total)), dim3(256), 0, ctx.stream, M, N, g.splits, batch,
                         alpha, (const double*)part, beta, C, ldc, sC);
    TTIGA_HIP(hipGetLastError());
  }
}

void gemm_lowp(Context& ctx, int dtype, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
               long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC,
               int batch) {
  TTIGA_CHECK(dtype == TTIGA_FP32 || dtype == TTIGA_BF16, TTIGA_E_ARG, "low-precision GEMM is FP32 or BF16");
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {
    gemm(ctx, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
    return;
  }
  GemmPlan g = gemm_plan(ta, tb, M, N, K, batch);
  g.bm = g.bn = 64;  // the low-precision kernel has one tile shape
  TTIGA_CHECK(batch <= 65535 / std::max(1, g.splits), TTIGA_E_ARG, "gemm: batch too large");
  // TTIGA_GEMM_TRACE=1 prints the shape of every product (the input of the offline tile tuner)
  static const bool trace = std::getenv("TTIGA_GEMM_TRACE") != nullptr;
  if (trace) std::fprintf(stderr, "[gemm-shape] ta=%d tb=%d M=%d N=%d K=%d batch=%d\n", ta, tb, M, N, K, batch);
  DBuf part;
  if (g.splits > 1) part = DBuf(ctx.alloc, sizeof(double) * gemm_part_doubles(g, M, N, batch));
  ProfScope prof(ctx, dtype == TTIGA_BF16 ? "gemm_bf16" : "gemm_fp32", 2.0 * M * N * (double)K * batch,
                 8.0 * batch * ((double)M * K + (double)K * N + (double)M * N));
  dim3 grid((N + 63) / 64, (M + 63) / 64, batch * g.splits);
#define TTIGA_LP_LAUNCH(TA, TB, PR)                                                                      \
  hipLaunchKernelGGL((k_gemm_lowp<TA, TB, PR>), grid, dim3(256), 0, ctx.stream, M, N, K, alpha, A, lda, sA, B, \
                     ldb, sB, beta, C, ldc, sC, g.splits, g.kchunk, part.d())
#define TTIGA_LP_PREC(PR)                                     \
  if (!ta && !tb) TTIGA_LP_LAUNCH(false, false, PR);          \
  else if (ta && !tb) TTIGA_LP_LAUNCH(true, false, PR);       \
  else if (!ta && tb) TTIGA_LP_LAUNCH(false, true, PR);       \
  else TTIGA_LP_LAUNCH(true, true, PR)
  if (dtype == TTIGA_BF16) {
    TTIGA_LP_PREC(TTIGA_BF16);
  } else {
    TTIGA_LP_PREC(TTIGA_FP32);
  }
#undef TTIGA_LP_PREC
#undef TTIGA_LP_LAUNCH
  TTIGA_HIP(hipGetLastError());
  if (g.splits > 1) {
    const long total = (long)batch * M * N;
    hipLaunchKernelGGL(k_splitk_reduce, dim3(grid_for(total)), dim3(256), 0, ctx.stream, M, N, g.splits, batch,
                       alpha, part.d(), beta, C, ldc, sC);
    TTIGA_HIP(hipGetLastError());
  }
}

void gemm_c(Context& ctx, bool operator_, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
            long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC,
            int batch) {
  if (ctx.lowp == 0)
    gemm(ctx, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
  else
    gemm_lowp(ctx, operator_ ? ctx.lowp : TTIGA_FP32, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc,
              sC, batch);
}

size_t gemm_part_doubles(const GemmPlan& g, int M, int N, int batch) {
  return g.splits > 1 ? (size_t)batch * g.splits * M * N : 0;
}

__global__ void k_scale_matrix(int M, int N, double beta, double* C, long ldc, long sC, int batch) {
  const long total = (long)batch * M * N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e / ((long)M * N);
    const long rc = e % ((long)M * N);
    double* c = C + b * sC + (rc / N) * ldc + rc % N;
    *c = (beta == 0.0) ? 0.0 : beta * (*c);
  }
}

void gemm(Context& ctx, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
          long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
          long sC, int batch) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  if (K <= 0) {  // C = beta C
    hipLaunchKernelGGL(k_scale_matrix, dim3(grid_for((long)batch * M * N)), dim3(256), 0, ctx.stream, M, N,
                       beta, C, ldc, sC, batch);
    TTIGA_HIP(hipGetLastError());
    return;
  }
  const GemmPlan g = gemm_plan(ta, tb, M, N, K, batch);
  DBuf part;
  if (g.splits > 1) part = DBuf(ctx.alloc, sizeof(double) * gemm_part_doubles(g, M, N, batch));
  gemm_planned(ctx, g, ta, tb, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch, part.d());
}

}  // namespace ttiga
