// extern "C" entry points: argument checks, exception -> status code, and the
// device allocator / context plumbing.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <cstring>
#include <string>

#include "engine.hpp"

namespace ttiga {

static thread_local std::string g_last_error;

DeviceAllocator::~DeviceAllocator() {
  for (auto& kv : direct_) (void)hipFree(kv.first);
  if (spill_parent_) {
    for (void* p : deferred_) spill_parent_->release(p);
    for (auto& kv : spilled_) spill_parent_->release(kv.first);
  }
}

void DeviceAllocator::set_workspace(void* base, size_t bytes) {
  std::lock_guard<std::mutex> lk(mu_);
  TTIGA_CHECK(base_ == nullptr && direct_.empty(), TTIGA_E_STATE,
              "workspace must be set before the first allocation");
  TTIGA_CHECK(base && bytes >= 4096, TTIGA_E_ARG, "workspace too small");
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t a = (b + 255) & ~uintptr_t(255);
  base_ = reinterpret_cast<char*>(a);
  size_ = (bytes - (a - b)) & ~size_t(255);
  free_.clear();
  free_[0] = size_;
}

void* DeviceAllocator::alloc_locked(size_t bytes) {
  if (!base_ && spill_parent_) return nullptr;  // an arena without a region of its own
  if (!base_) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    direct_[p] = bytes;
    in_use_ += bytes;
    high_water_ = std::max(high_water_, in_use_);
    return p;
  }
  for (auto it = free_.begin(); it != free_.end(); ++it) {
    if (it->second >= bytes) {
      const size_t off = it->first, sz = it->second;
      free_.erase(it);
      if (sz > bytes) free_[off + bytes] = sz - bytes;
      used_[off] = bytes;
      in_use_ += bytes;
      high_water_ = std::max(high_water_, in_use_);
      return base_ + off;
    }
  }
  return nullptr;
}

void* DeviceAllocator::try_alloc(size_t bytes) {
  bytes = (std::max<size_t>(bytes, 1) + 255) & ~size_t(255);
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (void* p = alloc_locked(bytes)) return p;
  }
  if (!spill_parent_) return nullptr;
  void* p = spill_parent_->try_alloc(bytes);
  if (p) {
    std::lock_guard<std::mutex> lk(mu_);
    spilled_[p] = bytes;
    in_use_ += bytes;
    high_water_ = std::max(high_water_, in_use_);
  }
  return p;
}

void* DeviceAllocator::alloc(size_t bytes) {
  void* p = try_alloc(bytes);
  if (!p) {
    std::lock_guard<std::mutex> lk(mu_);
    throw Error(TTIGA_E_OOM, "device memory exhausted: need " + std::to_string(bytes) + " bytes, " +
                                 std::to_string(size_ - std::min(size_, in_use_)) +
                                 " free in the arena (fragmented or spilled)");
  }
  return p;
}

size_t DeviceAllocator::largest_free() const {
  std::lock_guard<std::mutex> lk(mu_);
  size_t m = 0;
  for (auto& kv : free_) m = std::max(m, kv.second);
  return m;
}

void DeviceAllocator::flush_deferred() {
  std::vector<void*> d;
  {
    std::lock_guard<std::mutex> lk(mu_);
    d.swap(deferred_);
  }
  for (void* p : d) spill_parent_->release(p);
}

void DeviceAllocator::release(void* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(mu_);
  if (!spilled_.empty()) {
    auto sp = spilled_.find(p);
    if (sp != spilled_.end()) {
      in_use_ -= sp->second;
      spilled_.erase(sp);
      deferred_.push_back(p);
      return;
    }
  }
  if (!base_) {
    auto it = direct_.find(p);
    if (it != direct_.end()) {
      in_use_ -= it->second;
      (void)hipFree(p);
      direct_.erase(it);
    }
    return;
  }
  const size_t off = static_cast<char*>(p) - base_;
  auto it = used_.find(off);
  if (it == used_.end()) return;
  size_t sz = it->second;
  used_.erase(it);
  in_use_ -= sz;
  size_t start = off;
  auto nx = free_.lower_bound(off);
  if (nx != free_.end() && nx->first == off + sz) {
    sz += nx->second;
    free_.erase(nx);
  }
  auto pv = free_.lower_bound(off);
  if (pv != free_.begin()) {
    --pv;
    if (pv->first + pv->second == off) {
      start = pv->first;
      sz += pv->second;
      free_.erase(pv);
    }
  }
  free_[start] = sz;
}

Context::~Context() {
  if (sync_event) (void)hipEventDestroy(sync_event);
  if (!borrowed) {
    if (host_scratch) (void)hipHostFree(host_scratch);
    if (host_small) (void)hipHostFree(host_small);
  }
  for (LaneRes& r : lane_cache) {
    if (r.stream) {
      (void)hipStreamSynchronize(r.stream);
      (void)hipStreamDestroy(r.stream);
    }
    if (r.host) (void)hipHostFree(r.host);
    if (r.small) (void)hipHostFree(r.small);
  }
}

double* Context::small(double** dev) {
  if (!host_small) {
    TTIGA_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_small), sizeof(double) * kHostSmall,
                            hipHostMallocCoherent));
    TTIGA_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&host_small_dev), host_small, 0));
  }
  *dev = host_small_dev;
  return host_small;
}

void Context::sync() {
  static const bool blocking = [] {
    const char* e = std::getenv("TTIGA_BLOCKING_SYNC");
    return e && e[0] == '1';
  }();
  if (!blocking) {
    TTIGA_HIP(hipStreamSynchronize(stream));
    return;
  }
  if (!sync_event) TTIGA_HIP(hipEventCreateWithFlags(&sync_event, hipEventBlockingSync | hipEventDisableTiming));
  TTIGA_HIP(hipEventRecord(sync_event, stream));
  TTIGA_HIP(hipEventSynchronize(sync_event));
}

hipEvent_t Profiler::get() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  TTIGA_HIP(hipEventCreate(&e));
  return e;
}

void Profiler::flush() {
  std::lock_guard<std::mutex> lk(mu);
  for (auto& p : pending) {
    TTIGA_HIP(hipEventSynchronize(p.b));
    float ms = 0.f;
    TTIGA_HIP(hipEventElapsedTime(&ms, p.a, p.b));
    KernelStat& k = stats[p.name];
    k.launches += p.count;
    k.ms += ms;
    k.flops += p.flops;
    k.bytes += p.bytes;
    pool.push_back(p.a);
    pool.push_back(p.b);
  }
  pending.clear();
}

void Profiler::merge_into(Profiler& dst) {
  flush();
  std::lock_guard<std::mutex> lk(dst.mu);
  std::lock_guard<std::mutex> lk_own(mu);
  for (auto& kv : stats) {
    KernelStat& k = dst.stats[kv.first];
    k.launches += kv.second.launches;
    k.ms += kv.second.ms;
    k.flops += kv.second.flops;
    k.bytes += kv.second.bytes;
  }
  stats.clear();
}

Profiler::~Profiler() {
  for (auto& p : pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : pool) (void)hipEventDestroy(e);
}

ProfScope::ProfScope(Context& c, const char* name, double flops, double bytes, int size, bool per_kernel)
    : c_(&c), name_(name), flops_(flops), bytes_(bytes) {
  if (!c.prof.on) return;
  if (c.prof.detail && size >= 0) {
    static const int edges[] = {16, 32, 48, 64, 96, 128, 160, 192, 256, 384, 512, 1024};
    int b = 1 << 30;
    for (int e : edges)
      if (size <= e) {
        b = e;
        break;
      }
    name_ += "_c" + std::to_string(b);
  }
  if (per_kernel) {
    per_kernel_ = true;
    return;
  }
  a_ = c.prof.get();
  TTIGA_HIP(hipEventRecord(a_, c.stream));
}

void ProfScope::kernel_events(hipEvent_t* start, hipEvent_t* stop) {
  *start = *stop = nullptr;
  if (!per_kernel_) return;
  *start = c_->prof.get();
  *stop = c_->prof.get();
  kev_.emplace_back(*start, *stop);
}

ProfScope::~ProfScope() {
  if (per_kernel_) {
    for (size_t i = 0; i < kev_.size(); ++i)
      c_->prof.pending.push_back({name_, kev_[i].first, kev_[i].second, i == 0 ? flops_ : 0.0, i == 0 ? bytes_ : 0.0,
                                  i == 0 ? 1 : 0});
    if (c_->prof.pending.size() > 4096) c_->prof.flush();
    return;
  }
  if (!a_) return;
  hipEvent_t b = c_->prof.get();
  if (hipEventRecord(b, c_->stream) != hipSuccess) {
    (void)hipGetLastError();
    c_->prof.pool.push_back(b);
    c_->prof.pool.push_back(a_);
    return;
  }
  c_->prof.pending.push_back({name_, a_, b, flops_, bytes_, 1});
  if (c_->prof.pending.size() > 4096) c_->prof.flush();
}

double* Context::host(size_t n) {
  if (n > host_scratch_doubles) {
    if (host_scratch) TTIGA_HIP(hipHostFree(host_scratch));
    host_scratch = nullptr;
    host_dev = nullptr;
    TTIGA_HIP(hipHostMalloc(reinterpret_cast<void**>(&host_scratch), sizeof(double) * std::max<size_t>(n, 64),
                            hipHostMallocCoherent));
    TTIGA_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&host_dev), host_scratch, 0));
    host_scratch_doubles = std::max<size_t>(n, 64);
  }
  return host_scratch;
}

template <class F>
static int guard(F&& f) {
  try {
    f();
    return TTIGA_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return TTIGA_E_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return TTIGA_E_ARG;
  } catch (...) {
    g_last_error = "unknown error";
    return TTIGA_E_ARG;
  }
}

static void copy_tt_to_host(Context& c, const TT& t, double* dst, size_t count) {
  const size_t need = t.total_elems();
  TTIGA_CHECK(dst != nullptr || need == 0, TTIGA_E_ARG, "null destination");
  TTIGA_CHECK(count >= need, TTIGA_E_ARG, "destination too small: need " + std::to_string(need));
  size_t off = 0;
  for (int k = 0; k < 3; ++k) {
    const size_t ne = t.core_elems(k);
    if (ne) TTIGA_HIP(hipMemcpyAsync(dst + off, t.c[k].d(), sizeof(double) * ne, hipMemcpyDeviceToHost, c.stream));
    off += ne;
  }
  c.sync();
}

}  // namespace ttiga

struct ttiga_ctx {
  ttiga::Context impl;
};

using namespace ttiga;

// Objects created on a context keep it alive: ttiga_destroy on a context with
// live problems or TT handles only marks it, and the last object frees it.
static void ctx_retain(Context* c) { ++c->live_objects; }
static void ctx_release(Context* c) {
  if (--c->live_objects == 0 && c->closing && c->on_last_release) c->on_last_release(c);
}

extern "C" {

int ttiga_version(int* major, int* minor) {
  if (major) *major = TTIGA_VERSION_MAJOR;
  if (minor) *minor = TTIGA_VERSION_MINOR;
  return TTIGA_OK;
}

const char* ttiga_last_error(void) { return g_last_error.c_str(); }

int ttiga_create(int device, void* hip_stream, ttiga_ctx** out) {
  return guard([&] {
    TTIGA_CHECK(out != nullptr, TTIGA_E_ARG, "null output");
    int count = 0;
    TTIGA_HIP(hipGetDeviceCount(&count));
    TTIGA_CHECK(device >= 0 && device < count, TTIGA_E_ARG, "no such HIP device");
    TTIGA_HIP(hipSetDevice(device));
    auto* c = new ttiga_ctx();
    c->impl.on_last_release = [](Context* ic) {
      (void)hipStreamSynchronize(ic->stream);
      delete ic->owner;
    };
    c->impl.owner = c;
    c->impl.device = device;
    c->impl.stream = static_cast<hipStream_t>(hip_stream);
    // the device address of the allocation-free entry point's scratch, once per device
    (void)noalloc_scratch(device);
    *out = c;
  });
}

int ttiga_destroy(ttiga_ctx* ctx) {
  return guard([&] {
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->impl.stream);
    if (ctx->impl.live_objects > 0) {
      ctx->impl.closing = true;
      return;
    }
    delete ctx;
  });
}

int ttiga_set_workspace(ttiga_ctx* ctx, void* dev_ptr, size_t bytes) {
  return guard([&] {
    TTIGA_CHECK(ctx != nullptr, TTIGA_E_ARG, "null context");
    ctx->impl.alloc->set_workspace(dev_ptr, bytes);
  });
}

int ttiga_problem_create(ttiga_ctx* ctx, const ttiga_geometry* geo, const ttiga_discretization* disc,
                         const ttiga_source* src, const ttiga_dirichlet* bc, const ttiga_options* opt,
                         ttiga_problem** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && out, TTIGA_E_ARG, "null context or output");
    TTIGA_HIP(hipSetDevice(ctx->impl.device));
    auto* p = new Problem(&ctx->impl, geo, disc, src, bc, opt);
    try {
      p->upload();
    } catch (...) {
      delete p;
      throw;
    }
    *out = new ttiga_problem{p};
    ctx_retain(&ctx->impl);
  });
}

int ttiga_validate(const ttiga_geometry* geo, const ttiga_discretization* disc, const ttiga_source* src,
                   const ttiga_dirichlet* bc, const ttiga_options* opt) {
  return guard([&] { Problem probe(nullptr, geo, disc, src, bc, opt); });
}

int ttiga_problem_destroy(ttiga_problem* prob) {
  return guard([&] {
    if (!prob) return;
    Context* c = prob->impl->ctx;
    (void)hipStreamSynchronize(c->stream);
    delete prob->impl;
    delete prob;
    ctx_release(c);
  });
}

int ttiga_assemble(ttiga_problem* prob, ttiga_assembly_stats* stats) {
  int code = guard([&] {
    TTIGA_CHECK(prob != nullptr, TTIGA_E_ARG, "null problem");
    TTIGA_HIP(hipSetDevice(prob->impl->ctx->device));
    prob->impl->assemble(stats);
  });
  if (stats) stats->status = code;
  return code;
}

int ttiga_solve(ttiga_problem* prob, ttiga_solve_stats* stats) {
  int code = guard([&] {
    TTIGA_CHECK(prob != nullptr, TTIGA_E_ARG, "null problem");
    TTIGA_HIP(hipSetDevice(prob->impl->ctx->device));
    prob->impl->solve(stats);
  });
  if (stats && prob && prob->impl->solved) {
    *stats = prob->impl->last_solve;
    stats->status = code;
  } else if (stats) {
    stats->status = code;
  }
  return code;
}

int ttiga_solution_ranks(const ttiga_problem* prob, int ranks[4], int n[3]) {
  return guard([&] {
    TTIGA_CHECK(prob && ranks && n, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(prob->impl->solved, TTIGA_E_STATE, "no solution yet");
    const TT& u = prob->impl->u;
    for (int k = 0; k < 4; ++k) ranks[k] = u.r[k];
    for (int k = 0; k < 3; ++k) n[k] = u.n[k];
  });
}

int ttiga_get_solution(const ttiga_problem* prob, double* dst, size_t count) {
  return guard([&] {
    TTIGA_CHECK(prob != nullptr, TTIGA_E_ARG, "null problem");
    TTIGA_CHECK(prob->impl->solved, TTIGA_E_STATE, "no solution yet");
    copy_tt_to_host(*prob->impl->ctx, prob->impl->u, dst, count);
  });
}

int ttiga_l2_error(ttiga_problem* prob, int exact_kind, const double* params, int extra_gauss, double out[3]) {
  return guard([&] {
    TTIGA_CHECK(prob && out, TTIGA_E_ARG, "null argument");
    Problem& P = *prob->impl;
    TTIGA_HIP(hipSetDevice(P.ctx->device));
    P.l2_error(exact_kind, params, extra_gauss, out);
  });
}

int ttiga_compression_ratios(ttiga_problem* prob, double out[4]) {
  return guard([&] {
    TTIGA_CHECK(prob && out, TTIGA_E_ARG, "null argument");
    prob->impl->compression_ratios(out);
  });
}

int ttiga_problem_tt_info(const ttiga_problem* prob, int which, int ranks[4], int n[3], int* band) {
  return guard([&] {
    TTIGA_CHECK(prob && ranks && n, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(prob->impl->assembled, TTIGA_E_STATE, "problem not assembled");
    const TT* t = prob->impl->which(which);
    TTIGA_CHECK(t != nullptr, TTIGA_E_ARG, "unknown TT selector");
    const bool banded = (which == TTIGA_WHICH_K || which == TTIGA_WHICH_KII);
    const int bw = banded ? 2 * prob->impl->p + 1 : 1;
    for (int k = 0; k < 4; ++k) ranks[k] = t->r[k];
    for (int k = 0; k < 3; ++k) n[k] = t->n[k] / bw;
    if (band) *band = bw;
  });
}

int ttiga_problem_tt_copy(const ttiga_problem* prob, int which, double* dst, size_t count) {
  return guard([&] {
    TTIGA_CHECK(prob != nullptr, TTIGA_E_ARG, "null problem");
    TTIGA_CHECK(prob->impl->assembled, TTIGA_E_STATE, "problem not assembled");
    const TT* t = prob->impl->which(which);
    TTIGA_CHECK(t != nullptr, TTIGA_E_ARG, "unknown TT selector");
    copy_tt_to_host(*prob->impl->ctx, *t, dst, count);
  });
}

int ttiga_sample_factors(ttiga_problem* prob, const double* pts, size_t count, double* out,
                         double* det_out) {
  return guard([&] {
    TTIGA_CHECK(prob != nullptr, TTIGA_E_ARG, "null problem");
    TTIGA_HIP(hipSetDevice(prob->impl->ctx->device));
    prob->impl->sample_points(pts, count, out, det_out);
  });
}

int ttiga_gemm_f64(ttiga_ctx* ctx, int ta, int tb, int M, int N, int K, double alpha, const double* A,
                   long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
                   long sC, int batch, const int* plan) {
  return guard([&] {
    TTIGA_CHECK(ctx && A && B && C, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(M >= 1 && N >= 1 && K >= 1 && batch >= 1, TTIGA_E_ARG, "gemm: sizes must be positive");
    TTIGA_CHECK(lda >= (ta ? M : K) && ldb >= (tb ? K : N) && ldc >= N, TTIGA_E_ARG,
                "gemm: leading dimension shorter than a row");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    GemmPlan g = gemm_plan(ta != 0, tb != 0, M, N, K, batch);
    if (plan) {
      const bool tile_ok = (plan[0] == 64 && plan[1] == 64) || (plan[0] == 128 && plan[1] == 64) ||
                           (plan[0] == 64 && plan[1] == 128) || (plan[0] == 64 && plan[1] == 16) ||
                           (plan[0] == 16 && plan[1] == 64);
      TTIGA_CHECK(tile_ok && plan[2] >= 0 && plan[2] % 32 == 0, TTIGA_E_ARG, "gemm: unknown plan");
      g.bm = plan[0];
      g.bn = plan[1];
      g.kchunk = (plan[2] == 0 || plan[2] >= K) ? K : plan[2];
      g.splits = (K + g.kchunk - 1) / g.kchunk;
      TTIGA_CHECK((long)batch * g.splits <= 65535, TTIGA_E_ARG, "gemm: batch times splits above 65535");
    }
    DBuf part;
    if (g.splits > 1) part = DBuf(c.alloc, sizeof(double) * gemm_part_doubles(g, M, N, batch));
    gemm_planned(c, g, ta != 0, tb != 0, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch,
                 part.d());
    c.sync();
  });
}

int ttiga_gemm_lowp(ttiga_ctx* ctx, int dtype, int ta, int tb, int M, int N, int K, double alpha, const double* A,
                    long lda, long sA, const double* B, long ldb, long sB, double beta, double* C, long ldc,
                    long sC, int batch) {
  return guard([&] {
    TTIGA_CHECK(ctx && A && B && C, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(M >= 1 && N >= 1 && K >= 1 && batch >= 1, TTIGA_E_ARG, "gemm: sizes must be positive");
    TTIGA_CHECK(lda >= (ta ? M : K) && ldb >= (tb ? K : N) && ldc >= N, TTIGA_E_ARG,
                "gemm: leading dimension shorter than a row");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    gemm_lowp(c, dtype, ta != 0, tb != 0, M, N, K, alpha, A, lda, sA, B, ldb, sB, beta, C, ldc, sC, batch);
    c.sync();
  });
}

int ttiga_tt_matvec(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, ttiga_tt** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && K && x && out, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(K->p >= 0 && K->p <= 16, TTIGA_E_ARG, "bad band half-width");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    ttiga_tt_view kv{};
    const int band = 2 * K->p + 1;
    for (int k = 0; k < 3; ++k) {
      TTIGA_CHECK(K->n[k] == x->n[k], TTIGA_E_ARG, "matvec: mode sizes differ");
      kv.n[k] = K->n[k] * band;
      kv.core[k] = K->core[k];
    }
    for (int k = 0; k < 4; ++k) kv.r[k] = K->r[k];
    TT Kt, xt;
    tt_from_view(c, kv, Kt);
    tt_from_view(c, *x, xt);
    auto* res = new ttiga_tt{&c, TT()};
    try {
      tt_matvec_banded(c, Kt, K->p, xt, res->t);
      c.sync();
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
    ctx_retain(&c);
  });
}

int ttiga_tt_matvec_round(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, double alpha,
                          const ttiga_tt_view* z, double beta, double eps, int sketch_rank, ttiga_tt** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && K && x && out, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(K->p >= 0 && K->p <= 16, TTIGA_E_ARG, "bad band half-width");
    TTIGA_CHECK(eps > 0.0 && eps < 1.0, TTIGA_E_ARG, "eps must lie in (0, 1)");
    TTIGA_CHECK(sketch_rank >= 1, TTIGA_E_ARG, "sketch_rank must be positive");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    ttiga_tt_view kv{};
    const int band = 2 * K->p + 1;
    for (int k = 0; k < 3; ++k) {
      TTIGA_CHECK(K->n[k] == x->n[k], TTIGA_E_ARG, "matvec: mode sizes differ");
      if (z) TTIGA_CHECK(z->n[k] == x->n[k], TTIGA_E_ARG, "z: mode sizes differ");
      kv.n[k] = K->n[k] * band;
      kv.core[k] = K->core[k];
    }
    for (int k = 0; k < 4; ++k) kv.r[k] = K->r[k];
    TT Kt, xt, zt;
    tt_from_view(c, kv, Kt);
    tt_from_view(c, *x, xt);
    if (z) tt_from_view(c, *z, zt);
    auto* res = new ttiga_tt{&c, TT()};
    try {
      int hint = sketch_rank;
      tt_matvec_round(c, Kt, K->p, xt, alpha, z ? &zt : nullptr, beta, eps, 0, hint, res->t);
      c.sync();
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
    ctx_retain(&c);
  });
}

int ttiga_tt_matvec_lowp(ttiga_ctx* ctx, const ttiga_ttm_view* K, const ttiga_tt_view* x, int dtype,
                         ttiga_tt** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && K && x && out, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(K->p >= 0 && K->p <= 16, TTIGA_E_ARG, "bad band half-width");
    TTIGA_CHECK(dtype == TTIGA_FP32 || dtype == TTIGA_BF16, TTIGA_E_ARG, "dtype must be TTIGA_FP32 or TTIGA_BF16");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    ttiga_tt_view kv{};
    const int band = 2 * K->p + 1;
    for (int k = 0; k < 3; ++k) {
      TTIGA_CHECK(K->n[k] == x->n[k], TTIGA_E_ARG, "matvec: mode sizes differ");
      kv.n[k] = K->n[k] * band;
      kv.core[k] = K->core[k];
    }
    for (int k = 0; k < 4; ++k) kv.r[k] = K->r[k];
    TT Kt, xt;
    tt_from_view(c, kv, Kt);
    tt_from_view(c, *x, xt);
    LowpTT Kl;
    tt_to_lowp(c, Kt, dtype, Kl);
    auto* res = new ttiga_tt{&c, TT()};
    try {
      tt_matvec_banded_lp(c, Kl, K->p, xt, res->t);
      c.sync();
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
    ctx_retain(&c);
  });
}

int ttiga_tt_round(ttiga_ctx* ctx, const ttiga_tt_view* x, double eps, ttiga_tt** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && x && out, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(eps > 0.0 && eps < 1.0, TTIGA_E_ARG, "eps must be in (0, 1)");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    auto* res = new ttiga_tt{&c, TT()};
    try {
      tt_from_view(c, *x, res->t);
      tt_round(c, res->t, eps, -1.0, 0);
      c.sync();
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
    ctx_retain(&c);
  });
}

int ttiga_tt_dot(ttiga_ctx* ctx, const ttiga_tt_view* x, const ttiga_tt_view* y, double* out) {
  return guard([&] {
    TTIGA_CHECK(ctx && x && y && out, TTIGA_E_ARG, "null argument");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    for (int k = 0; k < 3; ++k) TTIGA_CHECK(x->n[k] == y->n[k], TTIGA_E_ARG, "dot: mode sizes differ");
    TT xt, yt;
    tt_from_view(c, *x, xt);
    tt_from_view(c, *y, yt);
    *out = tt_dot_sync(c, xt, yt);
  });
}

int ttiga_tt_dot_noalloc(ttiga_ctx* ctx, const ttiga_tt_view* x, const ttiga_tt_view* y, double* out_dev) {
  return guard([&] {
    TTIGA_CHECK(ctx && x && y && out_dev, TTIGA_E_ARG, "null argument");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    tt_dot_noalloc(c, *x, *y, out_dev);
  });
}

int ttiga_tt_compress(ttiga_ctx* ctx, const double* A, const int n[3], double delta, ttiga_tt** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && A && n && out, TTIGA_E_ARG, "null argument");
    TTIGA_CHECK(delta >= 0.0, TTIGA_E_ARG, "delta must be >= 0");
    for (int k = 0; k < 3; ++k) TTIGA_CHECK(n[k] > 0, TTIGA_E_ARG, "bad mode size");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    auto* res = new ttiga_tt{&c, TT()};
    try {
      tt_compress_dense(c, A, n, delta, res->t, 0);
      c.sync();
    } catch (...) {
      delete res;
      throw;
    }
    *out = res;
    ctx_retain(&c);
  });
}

int ttiga_profile(ttiga_ctx* ctx, int enable) {
  return guard([&] {
    TTIGA_CHECK(ctx != nullptr, TTIGA_E_ARG, "null context");
    Profiler& pr = ctx->impl.prof;
    if (enable < 0) {  // reset
      pr.flush();
      std::lock_guard<std::mutex> lk(pr.mu);
      pr.stats.clear();
      return;
    }
    if (!enable) pr.flush();
    pr.on = enable != 0;
    const char* env = std::getenv("TTIGA_PROF_DETAIL");
    pr.detail = env && env[0] == '1';
  });
}

int ttiga_profile_read(ttiga_ctx* ctx, ttiga_kernel_stat* out, int capacity, int* count) {
  return guard([&] {
    TTIGA_CHECK(ctx && count, TTIGA_E_ARG, "null argument");
    Profiler& pr = ctx->impl.prof;
    pr.flush();
    std::lock_guard<std::mutex> lk(pr.mu);
    int i = 0;
    for (auto& kv : pr.stats) {
      if (out && i < capacity) {
        ttiga_kernel_stat& o = out[i];
        std::memset(&o, 0, sizeof(o));
        std::strncpy(o.name, kv.first.c_str(), sizeof(o.name) - 1);
        o.launches = kv.second.launches;
        o.total_ms = kv.second.ms;
        o.flops = kv.second.flops;
        o.bytes = kv.second.bytes;
      }
      ++i;
    }
    *count = i;
  });
}

int ttiga_tt_info(const ttiga_tt* t, int ranks[4], int n[3]) {
  return guard([&] {
    TTIGA_CHECK(t && ranks && n, TTIGA_E_ARG, "null argument");
    for (int k = 0; k < 4; ++k) ranks[k] = t->t.r[k];
    for (int k = 0; k < 3; ++k) n[k] = t->t.n[k];
  });
}

int ttiga_tt_copy(const ttiga_tt* t, double* dst, size_t count) {
  return guard([&] {
    TTIGA_CHECK(t != nullptr, TTIGA_E_ARG, "null TT");
    copy_tt_to_host(*t->ctx, t->t, dst, count);
  });
}

int ttiga_tt_view_of(const ttiga_tt* t, ttiga_tt_view* view) {
  return guard([&] {
    TTIGA_CHECK(t && view, TTIGA_E_ARG, "null argument");
    for (int k = 0; k < 3; ++k) view->n[k] = t->t.n[k];
    for (int k = 0; k < 4; ++k) view->r[k] = t->t.r[k];
    for (int k = 0; k < 3; ++k) view->core[k] = t->t.c[k].d();
  });
}

static std::unique_ptr<Problem> problem_from_request(const ttiga_request* req) {
  TTIGA_CHECK(req != nullptr, TTIGA_E_ARG, "null request");
  return std::make_unique<Problem>(nullptr, req->geo, req->disc, req->src, req->bc, req->opt);
}

int ttiga_footprint(const ttiga_request* req, size_t* bytes) {
  return guard([&] {
    TTIGA_CHECK(bytes != nullptr, TTIGA_E_ARG, "null output");
    *bytes = problem_from_request(req)->footprint_estimate();
  });
}

// Default pool: the largest free block of the workspace (or of the device) less 1 GiB.
static size_t default_budget(Context& c) {
  size_t avail = c.alloc->largest_free();
  if (c.alloc->capacity() == 0) {
    size_t free_b = 0, total_b = 0;
    TTIGA_HIP(hipMemGetInfo(&free_b, &total_b));
    avail = free_b;
  }
  const size_t reserve = size_t(1) << 30;
  TTIGA_CHECK(avail > reserve + (size_t(64) << 20), TTIGA_E_OOM, "no device memory left for a pool");
  return avail - reserve;
}

int ttiga_solve_batch(ttiga_ctx* ctx, int count, const ttiga_request* reqs, int lanes,
                      size_t hbm_budget, ttiga_tt** solutions, ttiga_result* results) {
  return guard([&] {
    TTIGA_CHECK(ctx && count >= 0 && (count == 0 || (reqs && solutions && results)), TTIGA_E_ARG,
                "null argument");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    for (int i = 0; i < count; ++i) {
      solutions[i] = nullptr;
      std::memset(&results[i], 0, sizeof(ttiga_result));
    }
    if (count == 0) return;
    std::vector<std::unique_ptr<Problem>> probs(count);
    std::vector<size_t> fp(count, 0);
    for (int i = 0; i < count; ++i) {
      const int code = guard([&] {
        probs[i] = problem_from_request(&reqs[i]);
        fp[i] = probs[i]->footprint_estimate();
      });
      if (code != TTIGA_OK) {
        results[i].status = code;
        std::strncpy(results[i].error, g_last_error.c_str(), sizeof(results[i].error) - 1);
      }
    }
    const size_t budget = hbm_budget ? hbm_budget : default_budget(c);
    Engine eng(&c, budget, lanes, count);
    // largest footprint first: the big problems overlap with the many small ones
    std::vector<int> order;
    for (int i = 0; i < count; ++i)
      if (probs[i]) order.push_back(i);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return fp[a] > fp[b]; });
    std::vector<unsigned long long> ticket(count, 0);
    for (int i : order) {
      const int code = guard([&] { ticket[i] = eng.submit(std::move(probs[i])); });
      if (code != TTIGA_OK) {
        results[i].status = code;
        std::strncpy(results[i].error, g_last_error.c_str(), sizeof(results[i].error) - 1);
      }
    }
    eng.wait_all();
    for (int i = 0; i < count; ++i) {
      if (!ticket[i]) continue;
      eng.poll(ticket[i], 0, &results[i]);
      if (results[i].status != TTIGA_OK && results[i].status != TTIGA_E_NOTCONV) continue;
      const TT& u = eng.solution(ticket[i]);
      auto* res = new ttiga_tt{&c, TT{}};
      const int code = guard([&] { tt_copy(c, u, res->t); });
      if (code != TTIGA_OK) {
        delete res;
        results[i].status = code;
        std::strncpy(results[i].error, g_last_error.c_str(), sizeof(results[i].error) - 1);
        continue;
      }
      solutions[i] = res;
      ctx_retain(&c);
    }
    c.sync();
  });
}

int ttiga_server_create(ttiga_ctx* ctx, size_t hbm_budget, int lanes, int max_queue,
                        ttiga_server** out) {
  return guard([&] {
    TTIGA_CHECK(ctx && out, TTIGA_E_ARG, "null argument");
    Context& c = ctx->impl;
    TTIGA_HIP(hipSetDevice(c.device));
    const size_t budget = hbm_budget ? hbm_budget : default_budget(c);
    auto* s = new ttiga_server{nullptr};
    try {
      s->engine = new Engine(&c, budget, lanes, max_queue > 0 ? max_queue : 1024);
    } catch (...) {
      delete s;
      throw;
    }
    *out = s;
    ctx_retain(&c);
  });
}

int ttiga_server_submit(ttiga_server* srv, const ttiga_request* req, unsigned long long* ticket) {
  return guard([&] {
    TTIGA_CHECK(srv && ticket, TTIGA_E_ARG, "null argument");
    *ticket = srv->engine->submit(problem_from_request(req));
  });
}

int ttiga_server_poll(ttiga_server* srv, unsigned long long ticket, int wait_ms, ttiga_result* out) {
  int st = TTIGA_OK;
  const int code = guard([&] {
    TTIGA_CHECK(srv != nullptr, TTIGA_E_ARG, "null server");
    st = srv->engine->poll(ticket, wait_ms, out);
  });
  return code != TTIGA_OK ? code : st;
}

int ttiga_server_solution(ttiga_server* srv, unsigned long long ticket, ttiga_tt_view* view) {
  return guard([&] {
    TTIGA_CHECK(srv && view, TTIGA_E_ARG, "null argument");
    const TT& u = srv->engine->solution(ticket);
    for (int k = 0; k < 3; ++k) view->n[k] = u.n[k];
    for (int k = 0; k < 4; ++k) view->r[k] = u.r[k];
    for (int k = 0; k < 3; ++k) view->core[k] = u.c[k].d();
  });
}

int ttiga_server_copy_solution(ttiga_server* srv, unsigned long long ticket, double* dst, size_t count) {
  return guard([&] {
    TTIGA_CHECK(srv != nullptr, TTIGA_E_ARG, "null server");
    Engine& e = *srv->engine;
    TTIGA_HIP(hipSetDevice(e.root()->device));
    copy_tt_to_host(*e.root(), e.solution(ticket), dst, count);
  });
}

int ttiga_server_release(ttiga_server* srv, unsigned long long ticket) {
  return guard([&] {
    TTIGA_CHECK(srv != nullptr, TTIGA_E_ARG, "null server");
    srv->engine->release(ticket);
  });
}

int ttiga_server_destroy(ttiga_server* srv) {
  return guard([&] {
    if (!srv) return;
    Context* c = srv->engine->root();
    delete srv->engine;
    delete srv;
    ctx_release(c);
  });
}

int ttiga_tt_free(ttiga_tt* t) {
  return guard([&] {
    if (!t) return;
    Context* c = t->ctx;
    delete t;
    ctx_release(c);
  });
}

}  // extern "C"
