// Executor for many independent TT-IGA problems (batched and serving modes).
//
// Every step of one problem is a chain of small dependent launches with host-side rank
// decisions in between (QR and SVD sweeps of TT-rounding on ranks of tens to a few
// hundred), so one problem occupies a few compute units at a time.  The executor runs
// several problems at once, one per lane; a lane is a host worker thread with its own
// HIP stream, so the launches and host synchronisations of different problems overlap.
//
// Memory: the pool is one block of the context's workspace.  A problem is admitted when
// its footprint estimate fits beside the estimates of the running problems; it then runs
// in an arena cut from the pool to that size.  Allocations that overrun the arena are
// taken from the pool and handed back only after the lane's stream has drained, and an
// arena returns to the pool only after its problem's work is complete, so memory never
// moves between streams while in use.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "engine.hpp"

namespace ttiga {

static double clock_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// Head-of-line rule: a waiting problem lets at most this many later ones start before it.
static constexpr int kMaxBypass = 8;

Engine::Engine(Context* root, size_t budget, int lanes, int max_queue) : root_(root) {
  TTIGA_CHECK(lanes >= 1 && lanes <= 64, TTIGA_E_ARG, "lanes must be in 1..64");
  TTIGA_CHECK(budget >= (size_t(64) << 20), TTIGA_E_ARG, "pool budget below 64 MiB");
  root->sync();  // memory the root stream released is idle before it changes hands
  region_ = DBuf(root->alloc, budget);
  pool_.set_workspace(region_.p, region_.bytes);
  budget_ = pool_.capacity();
  max_queue_ = std::max(1, max_queue);
  for (int i = 0; i < lanes; ++i) {
    auto ln = std::make_unique<Lane>();
    ln->ctx.device = root->device;
    ln->ctx.borrowed = true;
    Context::LaneRes r;
    {
      std::lock_guard<std::mutex> lk(root->lane_mu);
      if (!root->lane_cache.empty()) {
        r = root->lane_cache.back();
        root->lane_cache.pop_back();
      }
    }
    if (!r.stream) {
      const hipError_t e = hipStreamCreateWithFlags(&r.stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        give_back();
        TTIGA_HIP(e);
      }
    }
    ln->ctx.stream = r.stream;
    ln->ctx.host_scratch = r.host;
    ln->ctx.host_dev = r.host_dev;
    ln->ctx.host_scratch_doubles = r.host_doubles;
    ln->ctx.host_small = r.small;
    ln->ctx.host_small_dev = r.small_dev;
    lanes_.push_back(std::move(ln));
  }
  for (int i = 0; i < lanes; ++i) threads_.emplace_back([this, i] { worker(i); });
}

Engine::~Engine() {
  {
    std::lock_guard<std::mutex> lk(mu_);
    stop_ = true;
  }
  cv_work_.notify_all();
  for (auto& t : threads_) t.join();
  give_back();
}

// the lanes' streams and host arrays back to the root context (after their work has drained)
void Engine::give_back() {
  for (auto& ln : lanes_) {
    Context& c = ln->ctx;
    if (c.stream) (void)hipStreamSynchronize(c.stream);
    Context::LaneRes r{c.stream, c.host_scratch, c.host_dev, c.host_scratch_doubles, c.host_small, c.host_small_dev};
    c.stream = nullptr;
    c.host_scratch = c.host_dev = c.host_small = c.host_small_dev = nullptr;
    c.host_scratch_doubles = 0;
    if (r.stream || r.host || r.small) {
      std::lock_guard<std::mutex> lk(root_->lane_mu);
      root_->lane_cache.push_back(r);
    }
  }
  lanes_.clear();
}

Job* Engine::find_locked(unsigned long long ticket) {
  auto it = jobs_.find(ticket);
  return it == jobs_.end() ? nullptr : it->second.get();
}

Job* Engine::pick_locked() {
  if (queue_.empty()) return nullptr;
  const size_t free_bytes = budget_ - std::min(budget_, reserved_);
  auto take = [&](std::deque<Job*>::iterator it) {
    Job* j = *it;
    queue_.erase(it);
    return j;
  };
  // with nothing running the head always starts: only resident solutions can hold the
  // pool then, and waiting would wait for a release that may never come
  if (queue_.front()->footprint <= free_bytes || running_ == 0) return take(queue_.begin());
  if (queue_.front()->bypassed >= kMaxBypass) return nullptr;
  for (auto it = queue_.begin() + 1; it != queue_.end(); ++it) {
    if ((*it)->footprint <= free_bytes) {
      queue_.front()->bypassed += 1;
      return take(it);
    }
  }
  return nullptr;
}

unsigned long long Engine::submit(std::unique_ptr<Problem> p) {
  TTIGA_CHECK(p != nullptr, TTIGA_E_ARG, "null problem");
  const size_t fp = p->footprint_estimate();
  std::lock_guard<std::mutex> lk(mu_);
  TTIGA_CHECK(!stop_, TTIGA_E_STATE, "executor is shutting down");
  if (fp > budget_)
    throw Error(TTIGA_E_ADMISSION, "footprint estimate " + std::to_string(fp) + " bytes exceeds the pool (" +
                                       std::to_string(budget_) + " bytes)");
  if ((int)queue_.size() >= max_queue_) throw Error(TTIGA_E_ADMISSION, "request queue is full");
  auto j = std::make_unique<Job>();
  j->ticket = next_ticket_++;
  j->prob = std::move(p);
  j->footprint = fp;
  j->t_submit = clock_ms();
  const unsigned long long t = j->ticket;
  queue_.push_back(j.get());
  jobs_[t] = std::move(j);
  cv_work_.notify_one();
  return t;
}

void Engine::worker(int index) {
  (void)hipSetDevice(root_->device);
  Lane& lane = *lanes_[index];
  while (true) {
    Job* j = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu_);
      cv_work_.wait(lk, [&] {
        j = pick_locked();
        return j != nullptr || (stop_ && queue_.empty());
      });
      if (!j) return;
      reserved_ += j->footprint;
      running_ += 1;
      j->state = 1;
      j->t_start = clock_ms();
    }
    run(*j, lane, index);
    {
      std::lock_guard<std::mutex> lk(mu_);
      // the arena is back in the pool; the resident solution stays charged until release
      reserved_ -= j->footprint;
      reserved_ += j->resident_bytes;
      running_ -= 1;
      j->state = 2;
    }
    cv_done_.notify_all();
    cv_work_.notify_all();
  }
}

void Engine::run(Job& j, Lane& lane, int index) {
  Context& c = lane.ctx;
  ttiga_result& r = j.res;
  std::memset(&r, 0, sizeof(r));
  r.lane = index;
  r.footprint_bytes = j.footprint;
  int code = TTIGA_OK;
  std::string msg;
  {
    // the arena: when the pool is too fragmented, wait for a running problem that is not
    // itself waiting to hand memory back (a finished problem or a released solution wakes
    // the waiters); with no such problem, run on spills from the pool (E_OOM if they fail)
    DBuf chunk;
    {
      std::unique_lock<std::mutex> lk(mu_);
      void* p = nullptr;
      while (!(p = pool_.try_alloc(j.footprint)) && running_ - arena_waiters_ > 1) {
        arena_waiters_ += 1;
        cv_done_.wait(lk);
        arena_waiters_ -= 1;
      }
      if (p) {
        chunk.a = &pool_;
        chunk.p = p;
        chunk.bytes = j.footprint;
      }
    }
    DeviceAllocator arena;
    if (chunk.p) arena.set_workspace(chunk.p, chunk.bytes);
    arena.set_spill_parent(&pool_);
    c.alloc = &arena;
    // plans live in the root context: computed once, kept across batches and servers
    c.plan_alloc = root_->plan_alloc;
    c.plan_stream = root_->stream;
    c.plans = root_->plans;
    c.prof.on = root_->prof.on;
    c.prof.detail = root_->prof.detail;
    Problem& P = *j.prob;
    P.ctx = &c;
    try {
      P.upload();
      P.assemble(&r.assembly);
      try {
        P.solve(&r.solve);
      } catch (const Error& e) {
        if (e.code != TTIGA_E_NOTCONV) throw;
        code = e.code;
        msg = e.what();
      }
      const TT& u = P.u;
      TT& s = j.solution;
      for (int k = 0; k < 3; ++k) s.n[k] = u.n[k];
      for (int k = 0; k < 4; ++k) s.r[k] = u.r[k];
      for (int k = 0; k < 3; ++k) {
        const size_t bytes = sizeof(double) * u.core_elems(k);
        if (!bytes) continue;
        s.c[k] = DBuf(&pool_, bytes);
        j.resident_bytes += bytes;
        TTIGA_HIP(hipMemcpyAsync(s.c[k].p, u.c[k].p, bytes, hipMemcpyDeviceToDevice, c.stream));
      }
      c.sync();
    } catch (const Error& e) {
      code = e.code;
      msg = e.what();
    } catch (const std::bad_alloc&) {
      code = TTIGA_E_OOM;
      msg = "host allocation failed";
    } catch (const std::exception& e) {
      code = TTIGA_E_ARG;
      msg = e.what();
    }
    (void)hipStreamSynchronize(c.stream);
    if (code != TTIGA_OK && code != TTIGA_E_NOTCONV) {
      j.solution.set_zero(j.solution.n);
      j.resident_bytes = 0;
    }
    r.assembly.status = P.assembled ? TTIGA_OK : code;
    r.peak_bytes = arena.high_water();
    j.prob.reset();  // its buffers go back to the arena (the stream has drained)
    arena.flush_deferred();
    c.alloc = &c.own_alloc;
    c.plan_alloc = &c.own_alloc;
    c.plan_stream = nullptr;
    c.plans = &c.own_plans;
    if (c.prof.on) {
      try {
        c.prof.merge_into(root_->prof);
      } catch (const Error&) {
      }
    }
  }  // the arena, then its chunk, return to the pool
  const double t_end = clock_ms();
  r.status = code;
  std::strncpy(r.error, msg.c_str(), sizeof(r.error) - 1);
  for (int k = 0; k < 4; ++k) r.rank_u[k] = j.solution.r[k];
  for (int k = 0; k < 3; ++k) r.n[k] = j.solution.n[k];
  r.queue_ms = j.t_start - j.t_submit;
  r.run_ms = t_end - j.t_start;
  r.latency_ms = t_end - j.t_submit;
  r.solve.status = code;
}

int Engine::poll(unsigned long long ticket, int wait_ms, ttiga_result* out) {
  std::unique_lock<std::mutex> lk(mu_);
  Job* j = find_locked(ticket);
  TTIGA_CHECK(j != nullptr, TTIGA_E_ARG, "unknown ticket");
  if (j->state != 2 && wait_ms != 0) {
    auto done = [&] { return j->state == 2; };
    if (wait_ms < 0)
      cv_done_.wait(lk, done);
    else
      cv_done_.wait_for(lk, std::chrono::milliseconds(wait_ms), done);
  }
  if (j->state != 2) return TTIGA_PENDING;
  if (out) *out = j->res;
  return TTIGA_OK;
}

const TT& Engine::solution(unsigned long long ticket) {
  std::lock_guard<std::mutex> lk(mu_);
  Job* j = find_locked(ticket);
  TTIGA_CHECK(j != nullptr, TTIGA_E_ARG, "unknown ticket");
  TTIGA_CHECK(j->state == 2, TTIGA_E_STATE, "request still pending");
  TTIGA_CHECK(!j->solution.zero() || j->res.status == TTIGA_OK, TTIGA_E_STATE,
              "request failed: no solution");
  return j->solution;
}

void Engine::release(unsigned long long ticket) {
  std::unique_ptr<Job> dead;
  size_t dead_bytes = 0;
  {
    std::lock_guard<std::mutex> lk(mu_);
    auto it = jobs_.find(ticket);
    TTIGA_CHECK(it != jobs_.end(), TTIGA_E_ARG, "unknown ticket");
    TTIGA_CHECK(it->second->state == 2, TTIGA_E_STATE, "request still pending");
    dead_bytes = it->second->resident_bytes;
    dead = std::move(it->second);
    jobs_.erase(it);
  }
  // copies of the solution on the root stream are complete before its memory is reused
  root_->sync();
  dead.reset();
  {
    std::lock_guard<std::mutex> lk(mu_);
    reserved_ -= std::min(reserved_, dead_bytes);
  }
  // the solution's memory is back in the pool: waiting arenas and queued problems retry
  cv_done_.notify_all();
  cv_work_.notify_all();
}

void Engine::wait_all() {
  std::unique_lock<std::mutex> lk(mu_);
  cv_done_.wait(lk, [&] { return queue_.empty() && running_ == 0; });
}

}  // namespace ttiga
