// Executor for many independent TT-IGA problems: lanes (a host worker thread and a
// HIP stream each), a device pool carved from the context's workspace, admission by
// footprint, and per-problem arenas.  Used by the batched and the serving entry points.
#pragma once

#include <condition_variable>
#include <deque>
#include <thread>

#include "problem.hpp"

namespace ttiga {

struct Job {
  unsigned long long ticket = 0;
  std::unique_ptr<Problem> prob;  // host description; bound to a lane context while it runs
  size_t footprint = 0;
  int state = 0;  // 0 queued, 1 running, 2 done
  int bypassed = 0;  // later problems that started while this one waited at the head
  ttiga_result res{};
  TT solution;  // in the pool, resident until the job is released
  size_t resident_bytes = 0;  // the solution's bytes, charged to admission until release
  double t_submit = 0.0, t_start = 0.0;
};

class Engine {
 public:
  // budget bytes of the root context's allocator become the pool; lanes >= 1
  Engine(Context* root, size_t budget, int lanes, int max_queue);
  ~Engine();  // drains the queue, joins the lanes
  Engine(const Engine&) = delete;
  Engine& operator=(const Engine&) = delete;

  // takes ownership of a validated host description; E_ADMISSION when it can never fit
  // or the queue is full
  unsigned long long submit(std::unique_ptr<Problem> p);
  // TTIGA_PENDING or TTIGA_OK (result copied to out)
  int poll(unsigned long long ticket, int wait_ms, ttiga_result* out);
  // the finished job's solution (throws E_STATE while pending); the engine keeps it
  const TT& solution(unsigned long long ticket);
  void release(unsigned long long ticket);
  void wait_all();
  size_t budget() const { return budget_; }
  Context* root() const { return root_; }

 private:
  struct Lane {
    Context ctx;  // stream, host scratch and profiler of the lane; arena set per job
  };
  void worker(int lane);
  void give_back();
  void run(Job& j, Lane& lane, int index);
  Job* pick_locked();
  Job* find_locked(unsigned long long ticket);

  Context* root_;
  DBuf region_;           // the pool's memory in the root allocator
  DeviceAllocator pool_;  // arenas, spills and resident solutions
  std::map<unsigned long long, std::unique_ptr<Job>> jobs_;  // destroyed before the pool
  std::vector<std::unique_ptr<Lane>> lanes_;
  std::vector<std::thread> threads_;
  std::mutex mu_;
  std::condition_variable cv_work_, cv_done_;
  std::deque<Job*> queue_;
  // reserved_: footprints of running problems plus the bytes of resident solutions
  size_t budget_ = 0, reserved_ = 0;
  unsigned long long next_ticket_ = 1;
  // running_: problems started and not finished; arena_waiters_: those of them blocked
  // until memory comes back to the pool
  int max_queue_ = 0, running_ = 0, arena_waiters_ = 0;
  bool stop_ = false;
};

}  // namespace ttiga

struct ttiga_server {
  ttiga::Engine* engine;
};
