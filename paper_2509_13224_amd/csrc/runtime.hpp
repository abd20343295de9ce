// Internal runtime of the TT-IGA library: context, device allocator, TT handles,
// and the host-side drivers that sequence the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <condition_variable>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ttiga.h"

struct ttiga_ctx;

namespace ttiga {

// Errors travel as exceptions inside the library and become status codes at the C ABI.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define TTIGA_HIP(call)                                                                      \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      throw ::ttiga::Error(TTIGA_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define TTIGA_CHECK(cond, code, msg) \
  do {                               \
    if (!(cond)) throw ::ttiga::Error((code), (msg)); \
  } while (0)

// First-fit sub-allocator over one device buffer, or direct hipMalloc when no
// workspace was given.  All blocks are 256-byte aligned.  Calls are serialised by a
// mutex, so one allocator can feed several per-job arenas on other threads.  An
// arena may name a spill parent: requests it cannot place are taken from the parent,
// and their release is deferred until flush_deferred() (called once the arena's
// stream has drained), so another stream cannot reuse memory still being read.
class DeviceAllocator {
 public:
  ~DeviceAllocator();
  void set_workspace(void* base, size_t bytes);
  void set_spill_parent(DeviceAllocator* parent) { spill_parent_ = parent; }
  void* alloc(size_t bytes);
  void* try_alloc(size_t bytes);  // nullptr instead of E_OOM
  void release(void* p);
  void flush_deferred();
  size_t in_use() const { return in_use_; }
  size_t high_water() const { return high_water_; }
  size_t capacity() const { return size_; }
  size_t largest_free() const;

 private:
  void* alloc_locked(size_t bytes);
  mutable std::mutex mu_;
  char* base_ = nullptr;
  size_t size_ = 0;
  std::map<size_t, size_t> free_;   // offset -> size
  std::map<size_t, size_t> used_;   // offset -> size
  std::map<void*, size_t> direct_;  // hipMalloc'd blocks when no workspace
  DeviceAllocator* spill_parent_ = nullptr;
  std::map<void*, size_t> spilled_;  // live blocks taken from the parent
  std::vector<void*> deferred_;      // released spills awaiting flush_deferred()
  size_t in_use_ = 0, high_water_ = 0;
};

// A device buffer owned by the allocator; freed when the handle dies.
struct DBuf {
  DeviceAllocator* a = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(DeviceAllocator* al, size_t b) : a(al), bytes(b) { p = b ? al->alloc(b) : nullptr; }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept { *this = std::move(o); }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      reset();
      a = o.a; p = o.p; bytes = o.bytes;
      o.a = nullptr; o.p = nullptr; o.bytes = 0;
    }
    return *this;
  }
  ~DBuf() { reset(); }
  void reset() {
    if (a && p) a->release(p);
    p = nullptr; bytes = 0;
  }
  double* d() const { return static_cast<double*>(p); }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

// Opt-in per-kernel-class timing with HIP events on the context stream, with the
// algorithmic flops and bytes of each launch (for roofline fractions).
struct KernelStat {
  long launches = 0;
  double ms = 0.0, flops = 0.0, bytes = 0.0;
};

struct Profiler {
  std::mutex mu;  // guards stats while per-job profilers merge into this one
  bool on = false;
  bool detail = false;  // append a size bucket to kernel names (diagnostics)
  std::map<std::string, KernelStat> stats;
  struct Pending {
    std::string name;
    hipEvent_t a, b;
    double flops, bytes;
    int count;  // launches this entry stands for (0: a further kernel of the same call)
  };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  hipEvent_t get();
  void flush();  // waits for recorded events and folds them into stats
  void merge_into(Profiler& dst);  // flush, then add the stats to dst and clear them
  ~Profiler();
};

struct Context;

// Records events around the launches issued while it lives (when profiling is on).
class ProfScope {
 public:
  // size >= 0 is bucketed into the name when detailed profiling is on.  per_kernel: the time is
  // that of the kernels launched with the events of kernel_events (hipExtLaunchKernelGGL stamps
  // them at each kernel's own start and end) instead of the span between two stream markers,
  // which for kernels of a few microseconds also holds the host's launch latency whenever the
  // stream had run dry before the launch.
  ProfScope(Context& c, const char* name, double flops, double bytes, int size = -1, bool per_kernel = false);
  ~ProfScope();
  // start and stop events for one kernel of a per-kernel scope (both null when profiling is off)
  void kernel_events(hipEvent_t* start, hipEvent_t* stop);

 private:
  Context* c_;
  std::string name_;
  double flops_, bytes_;
  hipEvent_t a_ = nullptr;
  bool per_kernel_ = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> kev_;
};

// Discretisation-level plans reused across problems (the 1-D eigenbases of the
// preconditioner), keyed by (n, p, g, lo, hi).  Shared by the per-job contexts of an
// executor, so lookups and inserts take the mutex; a plan is inserted only after the
// stream that computed it has drained.
// Per-discretisation data (1-D eigenbases of the preconditioner), computed once and shared
// by every problem of a context and of the executors built on it.  A plan being computed
// is listed in `busy`; others asking for it wait on `cv` instead of computing it again.
struct PlanCache {
  std::mutex mu;
  std::condition_variable cv;
  std::map<std::array<int, 5>, std::shared_ptr<void>> map;
  std::set<std::array<int, 5>> busy;
};

struct Context {
  Profiler prof;
  int device = 0;
  hipStream_t stream = nullptr;
  // device memory: the context's own allocator, or a per-job arena of an executor
  DeviceAllocator own_alloc;
  DeviceAllocator* alloc = &own_alloc;
  // where plans are allocated: memory that lives as long as the plan cache; plan_stream is
  // the stream that releases plan_alloc's memory (null: this context's own stream), which
  // work on a plan's buffers must follow
  DeviceAllocator* plan_alloc = &own_alloc;
  hipStream_t plan_stream = nullptr;
  // declared after the allocator so that cached plans are released before it
  PlanCache own_plans;
  PlanCache* plans = &own_plans;
  // pinned, coherent host staging for small readbacks (ranks, scalars); kernels write
  // results straight to host_dev (its device address), so a readback needs no copy
  double* host_scratch = nullptr;
  double* host_dev = nullptr;
  size_t host_scratch_doubles = 0;
  // a second, fixed host-mapped array of kHostSmall doubles that never moves (host_scratch
  // is reallocated when a larger readback needs it): the AMEn local CG's dot results, whose
  // device address its captured graphs hold
  static constexpr int kHostSmall = 64;
  double* host_small = nullptr;
  double* host_small_dev = nullptr;
  double* small(double** dev);
  // executor lanes take their stream and pinned host memory from here and give them back
  // when the executor ends, so that a batch does not pay for creating streams (milliseconds
  // each) or for freeing pinned memory, which waits for the whole device to go idle
  struct LaneRes {
    hipStream_t stream = nullptr;
    double* host = nullptr;
    double* host_dev = nullptr;
    size_t host_doubles = 0;
    double* small = nullptr;
    double* small_dev = nullptr;
  };
  std::mutex lane_mu;
  std::vector<LaneRes> lane_cache;
  // set on an executor lane's context: its stream and host arrays belong to lane_cache
  bool borrowed = false;
  // TTIGA_FP32 / TTIGA_BF16 while the inner corrections of a mixed-precision solve run: the
  // contractions routed through gemm_c then use the low-precision MFMA product (0: FP64)
  int lowp = 0;
  // sketch seeds; reset at the start of every assembly and solve, so a problem's
  // results do not depend on what ran before it on the context
  uint64_t rng_counter = 0x5eed;
  // problems and TT handles alive on this context; ttiga_destroy defers the
  // deletion until the last of them is destroyed
  int live_objects = 0;
  bool closing = false;
  void (*on_last_release)(Context*) = nullptr;  // frees the owning C handle
  struct ::ttiga_ctx* owner = nullptr;
  ~Context();
  double* host(size_t n);
  // host(n) and the device address of the same memory
  double* host_device(size_t n) {
    host(n);
    return host_dev;
  }
  // waits for the stream; with TTIGA_BLOCKING_SYNC=1 the host thread sleeps on a
  // blocking-sync event instead of polling (measurement switch for many lanes)
  void sync();
  hipEvent_t sync_event = nullptr;
};

// TT tensor with d = 3 cores in paper order [r_k][n_k][r_{k+1}] (FP64, device).
struct TT {
  int n[3] = {0, 0, 0};
  int r[4] = {0, 0, 0, 0};  // all zero: the exact zero tensor
  DBuf c[3];
  bool zero() const { return r[1] == 0; }
  size_t core_elems(int k) const { return (size_t)r[k] * n[k] * r[k + 1]; }
  size_t total_elems() const { return core_elems(0) + core_elems(1) + core_elems(2); }
  void alloc(Context& ctx, const int* nn, const int* rr);
  void set_zero(const int* nn) {
    for (int k = 0; k < 3; ++k) { n[k] = nn[k]; c[k].reset(); }
    for (int k = 0; k < 4; ++k) r[k] = 0;
  }
};

// TT-matrix cores stored in FP32 or BF16 (raw 16-bit) for low-precision products.
struct LowpTT {
  int dtype = TTIGA_FP32;
  int n[3] = {0, 0, 0};
  int r[4] = {0, 0, 0, 0};
  DBuf c[3];
};

// Library-owned TT tensor returned through the C ABI.
}  // namespace ttiga

struct ttiga_tt {
  ttiga::Context* ctx;
  ttiga::TT t;
};

namespace ttiga {

// ----------------------------------------------------------------- kernel API
// Dense linear algebra on the stream (kernels_linalg.hip).
// C[b] = alpha * op(A[b]) * op(B[b]) + beta * C[b]; row-major operands, hand-written MFMA
// kernel (gemm_f64.hip).  The tile and the K splits are a function of the shape alone.
struct GemmPlan {
  int bm = 64, bn = 64;  // workgroup tile
  int splits = 1;        // K splits (partials summed in split order by a second kernel)
  int kchunk = 0;        // contraction length per split
};
GemmPlan gemm_plan(bool ta, bool tb, int M, int N, int K, int batch);
// doubles of partial-tile workspace a plan needs (0 without K splits)
size_t gemm_part_doubles(const GemmPlan& g, int M, int N, int batch);
// the product with a given plan and caller-provided partial-tile workspace (K > 0)
void gemm_planned(Context& ctx, const GemmPlan& g, bool ta, bool tb, int M, int N, int K, double alpha,
                  const double* A, long lda, long sA, const double* B, long ldb, long sB, double beta,
                  double* C, long ldc, long sC, int batch, double* part);
void gemm(Context& ctx, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
          long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
          long sC, int batch = 1);
// the contraction of a TT operation that may run in low precision: gemm, or while ctx.lowp is
// set gemm_lowp in ctx.lowp (operator = true: a product with the operator's cores) or FP32
// (the preconditioner's transforms, which need about two digits)
void gemm_c(Context& ctx, bool operator_, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
            long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC,
            int batch = 1);
// the same product with the operands rounded to dtype (TTIGA_FP32 / TTIGA_BF16) as they are
// staged, MFMA in that type with FP32 accumulation, FP64 in and out
void gemm_lowp(Context& ctx, int dtype, bool ta, bool tb, int M, int N, int K, double alpha, const double* A,
               long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc, long sC,
               int batch = 1);
// Blocks of 256 threads for a grid-stride elementwise kernel over `total` elements: four or
// more elements per thread and at most 2048 blocks (eight per compute unit), enough to stream
// HBM on an idle device without holding every wave slot while the kernels of other streams
// wait for room (short workgroups of one element per thread mostly wait for memory).
inline int grid_for(long total) { return (int)std::max<long>(1, std::min<long>((total + 1023) / 1024, 2048)); }
// Q (m x c, row-major, orthonormal columns) and R (c x c, upper) with op(A) = Q R (Householder TSQR).
void qr_tall(Context& ctx, const double* A, bool transA, int m, int c, long lda, double* Q,
             double* R);
// qr_tall of `batch` problems of one shape in the same launches: problem b reads A + b sA and
// writes Q + b sQ, R + b sR (c <= 256).
void qr_tall_batched(Context& ctx, int batch, const double* A, long sA, bool transA, int m, int c, long lda,
                     double* Q, long sQ, double* R, long sR);
// One-sided Jacobi SVD of op(A) (m x c, m >= c): U (m x c), s (c, descending), V (c x c);
// V may be null when the right vectors are not needed.  prof_name labels the launch in
// the profile.
void svd_small(Context& ctx, const double* A, bool transA, int m, int c, long lda, double* U,
               double* s, double* V, const char* prof_name = "jacobi_svd");
// k interpolation rows of an n x k matrix with orthonormal columns (column-pivoted QR of
// Q^T), written to the device array rows.
void pivot_rows(Context& ctx, const double* Q, int n, int k, int* rows);
// Upper Cholesky factor R (R^T R = G) and R^-1 of an SPD c x c matrix; false if G is not SPD.
bool cholesky_inverse(Context& ctx, const double* G, int c, double* R, double* Rinv);
// Pivoted Cholesky G = L L^T of a symmetric positive semi-definite G (r x r, row-major):
// L (r x r buffer, row-major; columns >= k are zero) in the original index order, stopped
// at the first pivot at most tau_rel max_i G_ii; returns k (host synchronisation).
int pivoted_cholesky(Context& ctx, const double* G, int r, double* L, double tau_rel);
// Smallest r with ||s[r:]|| <= delta (delta < 0: -delta * ||s|| / sqrt(2) relative).
int trunc_rank_sync(Context& ctx, const double* s, int c, double delta, double* norm_out);
// truncation ranks of `batch` singular value lists (s + b ss, thresholds as trunc_rank_sync's
// delta, one per list) with one host round trip; norms (optional) receives each list's norm
void trunc_ranks_sync(Context& ctx, int batch, const double* s, long ss, int c, const double* delta, int* ranks,
                      double* norms);
// svd_small of `batch` problems of one shape (problem b: A + b sA, U + b sU, s + b sS, V + b sV):
// one launch when a problem's columns fit in LDS, else one launch per problem
void svd_small_batched(Context& ctx, int batch, const double* A, long sA, bool transA, int m, int c, long lda,
                       double* U, long sU, double* s, long sS, double* V, long sV, const char* prof_name = "jacobi_svd");
void fill(Context& ctx, double* p, size_t n, double v);
void copy(Context& ctx, double* dst, const double* src, size_t n);
void sumsq_reduce(Context& ctx, const double* x, size_t n, double* out_dev);

// TT algebra (tt_ops.cpp / kernels_tt.hip).
void tt_from_view(Context& ctx, const ttiga_tt_view& v, TT& out);
void tt_round(Context& ctx, TT& x, double eps_rel, double delta_abs, int max_rank,
              double* norm_out = nullptr, bool left_orthogonal = false);
// Rounding that first projects high-rank trains onto a Gaussian sketch of width
// hint + 10 (randomised TT-rounding) and then truncates deterministically; hint
// is updated to the resulting rank.
void tt_round_auto(Context& ctx, TT& x, double eps_rel, int max_rank, int& hint);
// out[0..n) = standard normal numbers from the context's sketch counter (advanced by one).
void gaussian_fill(Context& ctx, double* out, long n);
// Randomised rounding of y = alpha K x + beta z (K banded with half-bandwidth p, z optional)
// at relative eps without forming the product cores (sketch width hint + 10, widened by 12
// while the rounded rank saturates it; hint receives the rank).  The sketch is drawn as
// tt_round_auto draws it for an explicit train.
void tt_matvec_round(Context& ctx, const TT& K, int p, const TT& x, double alpha, const TT* z, double beta,
                     double eps_rel, int max_rank, int& hint, TT& out);
// Bytes of the explicit product cores of K x.
size_t matvec_product_bytes(const TT& K, const TT& x);
// out core d of x multiplied along mode d by op(Mat) (n x n row-major).
void tt_mode_product(Context& ctx, TT& x, int d, const double* Mat, bool trans);
void tt_axpby(Context& ctx, double alpha, const TT& x, double beta, const TT& y, TT& out);
void tt_axpby_dev(Context& ctx, const double* alpha, const TT& x, const double* beta, const TT& y,
                  TT& out);
// copies n device doubles into host-mapped memory (a Context::host_device address) with a
// system-scope fence, so that they are in host memory once the stream has drained
void publish_to_host(Context& ctx, const double* src, double* dst_mapped, int n);
double tt_dot_sync(Context& ctx, const TT& x, const TT& y);
// out[i] = x_i . y_i for count pairs (count <= 8) with one host synchronisation
void tt_dots_sync(Context& ctx, const TT* const* x, const TT* const* y, int count, double* out);
void tt_dot_dev(Context& ctx, const TT& x, const TT& y, double* out_dev);
// <x, y> from raw device cores (ranks rx, ry with rx[0] = ry[0] = rx[3] = ry[3] = 1) into
// out_dev, all temporaries in `scratch` of tt_dot_scratch_doubles(n, rx, ry) doubles
size_t tt_dot_scratch_doubles(const int* n, const int* rx, const int* ry);
// sum_q W_q E_q^2 over the grid of two TTs with the same mode sizes (errors.hip)
double tt_weighted_sqnorm(Context& ctx, const TT& E, const TT& W);
// the allocation-free variant (noalloc.hip): the same chain with its temporaries in a fixed
// per-device array; noalloc_scratch looks the array's address up (once per device, with
// that device current)
double* noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
void tt_dot_noalloc(Context& ctx, const ttiga_tt_view& x, const ttiga_tt_view& y, double* out_dev);
void tt_dot_cores(Context& ctx, const int* n, const int* rx, const double* const* xc, const int* ry,
                  const double* const* yc, double* out_dev, double* scratch);
void tt_matvec_banded(Context& ctx, const TT& K, int p, const TT& x, TT& y);
// FP64 cores -> FP32 or BF16 cores (round to nearest even, BF16 through FP32).
void tt_to_lowp(Context& ctx, const TT& src, int dtype, LowpTT& dst);
// y = K x with K in FP32/BF16, x rounded to FP32, FP32 products and band sums, y in FP64.
void tt_matvec_banded_lp(Context& ctx, const LowpTT& K, int p, const TT& x, TT& y);
void tt_compress_dense(Context& ctx, const double* A, const int* n, double delta, TT& out,
                       int max_rank);
void tt_copy(Context& ctx, const TT& src, TT& dst);
// Streamed TT-SVD of nt tensors of shape n produced in chunks of second-direction slabs:
// produce(b, c, buf) writes slabs b .. b+c-1 of every tensor into buf[t][n0][c][n2];
// thresholds(delta) is called once, after the first pass, and sets the absolute
// per-unfolding thresholds (negative: the tensor is zero).
using ChunkFn = std::function<void(int a, int c, double* buf)>;
using ThresholdFn = std::function<void(std::vector<double>& delta)>;
void tt_compress_streamed(Context& ctx, int nt, const int* n, int chunk, const ChunkFn& produce,
                          const ThresholdFn& thresholds, TT* out, int max_rank);
// TT of A from an orthonormal basis Qb (n0 x L) of its first unfolding and B (L x n1 n2)
// with A_(0) ~= Qb B: truncated SVD of B at delta, first core Qb U_s, the rest factored like
// a dense tensor.  With spare > 0 it returns false (out untouched) when the truncated rank
// leaves fewer than spare columns of L.
bool tt_from_first_unfolding(Context& ctx, const double* Qb, int L, const double* B, const int* n, double delta,
                             int spare, TT& out, int max_rank);
// Orthonormal basis U (m x k) of the columns of C (m x L, m >= L) from its truncated SVD
// with tail delta (Frobenius; delta < 0: relative to ||C||); returns k (0: C is below it).
int column_basis(Context& ctx, const double* C, int m, int L, double delta, DBuf& U);
// column_basis of `count` m x L matrices C + t stride (m > L) at thresholds delta[t]: ranks into
// k[t], bases into U[t] (left empty at rank 0), with the factorisations batched
void column_basis_batched(Context& ctx, int count, const double* C, long stride, int m, int L, const double* delta,
                          int* k, DBuf* U);
// out[i][j] = A[i][j] / S[j] for an m x cols row-major A.
void scale_cols_inv(Context& ctx, const double* A, int m, int cols, const double* S, double* out);
// out (nr x k) = rows `rows` (device) of A (n x k), row-major.
void gather_rows(Context& ctx, const double* A, int k, const int* rows, int nr, double* out);
// Values of x at grid points (device index arrays, count entries) into out.
void tt_eval_points(Context& ctx, const TT& x, long count, const int* i0, const int* i1, const int* i2,
                    double* out);
// Sizes at or below which TT-SVD unfoldings are factored exactly instead of sketched.
constexpr int kExactSvdSize = 64;

}  // namespace ttiga
