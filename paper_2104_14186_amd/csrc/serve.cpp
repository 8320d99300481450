// Continuous-batching request server for EIG / SVD solves.
//
// Requests enter a FIFO.  A request is admitted when a lane is idle and its
// workspace (the library's own size query, i.e. its HBM footprint) fits in
// a free range of the server's arena; lanes are host threads, each with its
// own HIP stream, so admitted requests run concurrently and their kernels
// overlap on the device.  Requests that arrive while others run are admitted
// as lanes and memory free up; the head of the queue is never overtaken, so
// a large request cannot starve.  Iteration state lives in the request's
// arena range on the device for the whole solve.
//
// A request computes exactly what a standalone call computes (same kernels,
// launch shapes independent of what else runs, no order-dependent atomics),
// so its results do not depend on the mix it was served in.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"

namespace qdwhp {
size_t problem_workspace(const qdwhp_problem& p, const qdwhp_opts* o);
int run_problem(const qdwhp_problem& p, void* work, size_t lwork, const qdwhp_opts* o,
                hipStream_t s, qdwhp_info* info, Deferred* df);
}  // namespace qdwhp

using namespace qdwhp;
using Clock = std::chrono::steady_clock;

namespace {

// First-fit allocator over [0, cap) with coalescing of freed ranges.
struct RangeAlloc {
  std::map<size_t, size_t> free_;   // offset -> size
  explicit RangeAlloc(size_t cap) { if (cap) free_[0] = cap; }
  bool take(size_t bytes, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      *off = it->first;
      const size_t rest = it->second - bytes, o = it->first + bytes;
      free_.erase(it);
      if (rest) free_[o] = rest;
      return true;
    }
    return false;
  }
  void give(size_t off, size_t bytes) {
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Request {
  qdwhp_problem p;
  size_t bytes = 0;
  Clock::time_point t_submit, t_start, t_done;
  int status = QDWHP_PENDING;
  qdwhp_info info{};
};

}  // namespace

struct qdwhp_server {
  int dev = 0;
  char* arena = nullptr;
  size_t cap = 0;
  RangeAlloc alloc{0};
  qdwhp_opts opts;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;
  std::map<int64_t, Request> reqs;
  int64_t next_id = 1;
  bool stop = false;
  int running = 0;
  int peak_running = 0;
  size_t in_use = 0, peak_bytes = 0;
  std::vector<std::thread> lanes;

  std::vector<hipStream_t> streams;

  void lane_loop(int l) {
    if (hipSetDevice(dev) != hipSuccess) return;
    hipStream_t s = streams[l];
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
      if (stop && queue.empty()) return;
      size_t off = 0;
      if (queue.empty() || !alloc.take(reqs[queue.front()].bytes, &off)) {
        cv_work.wait(lk);
        continue;
      }
      const int64_t id = queue.front();
      queue.pop_front();
      Request& r = reqs[id];
      r.t_start = Clock::now();
      ++running;
      in_use += r.bytes;
      peak_bytes = std::max(peak_bytes, in_use);
      peak_running = std::max(peak_running, running);
      const qdwhp_problem p = r.p;
      const size_t bytes = r.bytes;
      lk.unlock();
      qdwhp_info info{};
      int st = run_problem(p, arena + off, bytes, &opts, s, &info, nullptr);
      if (hipStreamSynchronize(s) != hipSuccess && st == QDWHP_OK) st = QDWHP_ERR_HIP;
      lk.lock();
      Request& q = reqs[id];
      q.t_done = Clock::now();
      q.status = st;
      q.info = info;
      --running;
      in_use -= bytes;
      alloc.give(off, bytes);
      cv_done.notify_all();
      cv_work.notify_all();
    }
  }
};

extern "C" int qdwhp_serve_create(size_t arena_bytes, int lanes, const qdwhp_opts* opts,
                                  qdwhp_server** out) {
  if (!out) return -4;
  *out = nullptr;
  if (arena_bytes == 0) return -1;
  if (lanes < 0) return -2;
  auto* srv = new qdwhp_server();
  if (opts) srv->opts = *opts; else qdwhp_opts_default(&srv->opts);
  if (hipGetDevice(&srv->dev) != hipSuccess ||
      hipMalloc((void**)&srv->arena, arena_bytes) != hipSuccess) {
    delete srv;
    return QDWHP_ERR_HIP;
  }
  srv->cap = arena_bytes;
  srv->alloc = RangeAlloc(arena_bytes);
  const int L = lanes > 0 ? lanes : (int)std::max<int64_t>(1, qdwhp_tune_get("serve.lanes", 8));
  for (int l = 0; l < L; ++l) {
    hipStream_t st;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (auto x : srv->streams) (void)hipStreamDestroy(x);
      (void)hipFree(srv->arena);
      delete srv;
      return QDWHP_ERR_HIP;
    }
    srv->streams.push_back(st);
  }
  for (int l = 0; l < L; ++l) srv->lanes.emplace_back(&qdwhp_server::lane_loop, srv, l);
  *out = srv;
  return QDWHP_OK;
}

extern "C" int qdwhp_serve_submit(qdwhp_server* srv, const qdwhp_problem* p, int64_t* ticket) {
  if (!srv) return -1;
  if (!p || (p->type != QDWHP_PROBLEM_EIG && p->type != QDWHP_PROBLEM_SVD)) return -2;
  if (!ticket) return -3;
  const size_t b = (problem_workspace(*p, &srv->opts) + 255) / 256 * 256;
  if (b == 0) return -2;
  std::lock_guard<std::mutex> g(srv->mu);
  if (srv->stop) return -1;
  const int64_t id = srv->next_id++;
  Request& r = srv->reqs[id];
  r.p = *p;
  r.bytes = b;
  r.t_submit = Clock::now();
  if (b > srv->cap) {   // can never be admitted
    r.status = QDWHP_ERR_WORKSPACE;
    r.t_start = r.t_done = r.t_submit;
  } else {
    srv->queue.push_back(id);
    srv->cv_work.notify_all();
  }
  *ticket = id;
  return QDWHP_OK;
}

extern "C" int qdwhp_serve_poll(qdwhp_server* srv, int64_t ticket, int wait, qdwhp_info* info,
                                double* latency_ms, double* queue_ms) {
  if (!srv) return -1;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto it = srv->reqs.find(ticket);
  if (it == srv->reqs.end()) return -2;
  if (wait)
    srv->cv_done.wait(lk, [&] { return srv->reqs[ticket].status != QDWHP_PENDING; });
  Request& r = srv->reqs[ticket];
  if (r.status == QDWHP_PENDING) return QDWHP_PENDING;
  if (info) *info = r.info;
  if (latency_ms) *latency_ms = std::chrono::duration<double, std::milli>(r.t_done - r.t_submit).count();
  if (queue_ms) *queue_ms = std::chrono::duration<double, std::milli>(r.t_start - r.t_submit).count();
  const int st = r.status;
  srv->reqs.erase(ticket);
  return st;
}

extern "C" int qdwhp_serve_stats(qdwhp_server* srv, size_t* peak_bytes, size_t* arena_bytes, int* peak_running,
                                 int reset) {
  if (!srv) return -1;
  std::lock_guard<std::mutex> g(srv->mu);
  if (peak_bytes) *peak_bytes = srv->peak_bytes;
  if (arena_bytes) *arena_bytes = srv->cap;
  if (peak_running) *peak_running = srv->peak_running;
  if (reset) {
    srv->peak_bytes = srv->in_use;
    srv->peak_running = srv->running;
  }
  return QDWHP_OK;
}

extern "C" int qdwhp_serve_destroy(qdwhp_server* srv) {
  if (!srv) return -1;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
    srv->cv_work.notify_all();
  }
  for (auto& t : srv->lanes) t.join();
  for (auto x : srv->streams) (void)hipStreamDestroy(x);
  const hipError_t e = hipFree(srv->arena);
  delete srv;
  return e == hipSuccess ? QDWHP_OK : QDWHP_ERR_HIP;
}
