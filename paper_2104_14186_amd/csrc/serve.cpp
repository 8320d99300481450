// Continuous-batching request server for EIG / SVD solves.
//
// Requests enter a FIFO.  A request is admitted when a lane is free and its
// workspace (the library's own size query, i.e. its HBM footprint) fits in
// a free range of the server's arena; lanes are host threads, each with its
// own HIP stream.  An admitted request goes through the three phases of a
// solve, each taken by whichever lane is free: its setup (estimator,
// threshold, schedule, X0); its DWH iterations, together with every other
// request of the same shape waiting at that point (grouped Gram, lockstep
// Cholesky-inversion and grouped triangular products: one persistent launch
// per phase for the whole group); then projector, subspace and Rayleigh-Ritz.
// Requests that arrive while others run are admitted as lanes and memory free
// up and join the next group of their shape; the head of the queue is never
// overtaken, so a large request cannot starve.  Iteration state lives in the
// request's arena range on the device for the whole solve.  "serve.grouped" =
// 0 runs every phase of a request on one lane instead.
//
// Every grouped launch performs each member's operations exactly as its
// standalone call would (same kernels and tile arithmetic, no order-dependent
// atomics), so a request's results do not depend on the mix it was served
// in: alone, in any mix, or as a standalone call, they are bitwise the same.

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

// An admitted request between its phases.
struct Active {
  int64_t id = 0;
  size_t off = 0, bytes = 0;
  SolveState* S = nullptr;
  qdwhp_info info{};
  hipEvent_t ready = nullptr;    // end of its last phase, on the stream that ran it
};

constexpr int kMaxGroup = 64;    // requests per grouped iteration launch sequence

}  // namespace

struct qdwhp_server {
  int dev = 0;
  char* arena = nullptr;
  size_t cap = 0;                // bytes of the arena open to requests
  char* tables = nullptr;        // one grouped-GEMM descriptor table per lane (end of the arena)
  RangeAlloc alloc{0};
  qdwhp_opts opts;
  bool grouped = true;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> queue;                 // submitted, not admitted
  std::deque<Active*> iter_q, fin_q;         // set up / iterated, waiting for the next phase
  std::map<int64_t, Request> reqs;
  int64_t next_id = 1;
  bool stop = false;
  int running = 0;               // admitted, not finished
  int peak_running = 0;
  size_t in_use = 0, peak_bytes = 0;
  int64_t groups = 0, grouped_reqs = 0;   // iteration groups run and their members
  int nlanes = 0;
  std::vector<std::thread> lanes;
  std::vector<hipStream_t> streams;

  // Each lane runs whatever phase is ready, finishing work first: the
  // subspace and Rayleigh-Ritz phase of an iterated request; else, while
  // fewer requests than lanes wait for their iterations, admission and setup
  // of the next queued request; else the iterations of every waiting request
  // with the shape of the oldest one, as one group.
  void lane_loop(int l) {
    if (hipSetDevice(dev) != hipSuccess) return;
    hipStream_t s = streams[l];
    void* table = tables + (size_t)l * grouped_table_bytes(kMaxGroup);
    std::unique_lock<std::mutex> lk(mu);
    std::vector<Active*> grp;
    std::vector<SolveState*> sv;
    for (;;) {
      if (!fin_q.empty()) {
        Active* a = fin_q.front();
        fin_q.pop_front();
        lk.unlock();
        int st = QDWHP_OK;
        if (hipStreamWaitEvent(s, a->ready, 0) != hipSuccess) st = QDWHP_ERR_HIP;
        solve_set_stream(a->S, s);
        if (st == QDWHP_OK) st = solve_finish(a->S);
        if (hipStreamSynchronize(s) != hipSuccess && st == QDWHP_OK) st = QDWHP_ERR_HIP;
        lk.lock();
        complete(a, st);
        continue;
      }
      size_t off = 0;
      // admission runs ahead of the iterations while fewer requests than
      // lanes wait for them, so that same-shape requests can meet in a group
      const bool admit_first = (int)iter_q.size() < nlanes;
      if ((admit_first || iter_q.empty()) && !queue.empty() && alloc.take(reqs[queue.front()].bytes, &off)) {
        const int64_t id = queue.front();
        queue.pop_front();
        Request& r = reqs[id];
        r.t_start = Clock::now();
        ++running;
        in_use += r.bytes;
        peak_bytes = std::max(peak_bytes, in_use);
        peak_running = std::max(peak_running, running);
        Active* a = new Active();
        a->id = id; a->off = off; a->bytes = r.bytes;
        const qdwhp_problem p = r.p;
        lk.unlock();
        int st = QDWHP_OK;
        a->S = solve_create(p, arena + off, a->bytes, &opts, s, &a->info, nullptr);
        if (hipEventCreateWithFlags(&a->ready, hipEventDisableTiming) != hipSuccess) { a->ready = nullptr; st = QDWHP_ERR_HIP; }
        if (st == QDWHP_OK) st = solve_setup(a->S);
        if (st == QDWHP_OK && !grouped) {
          st = solve_iterate(a->S);
          if (st == QDWHP_OK) st = solve_finish(a->S);
          if (hipStreamSynchronize(s) != hipSuccess && st == QDWHP_OK) st = QDWHP_ERR_HIP;
        } else if (st == QDWHP_OK && hipEventRecord(a->ready, s) != hipSuccess) {
          st = QDWHP_ERR_HIP;
        }
        if (st != QDWHP_OK) (void)hipStreamSynchronize(s);
        lk.lock();
        if (st == QDWHP_OK && grouped) {
          iter_q.push_back(a);
          cv_work.notify_all();
        } else {
          complete(a, st);
        }
        continue;
      }
      if (!iter_q.empty()) {
        const int64_t shape = solve_shape(iter_q.front()->S);
        grp.clear();
        for (auto it = iter_q.begin(); it != iter_q.end() && (int)grp.size() < kMaxGroup;) {
          if (solve_shape((*it)->S) == shape) { grp.push_back(*it); it = iter_q.erase(it); }
          else ++it;
        }
        ++groups;
        grouped_reqs += (int64_t)grp.size();
        lk.unlock();
        bool ok = true;
        sv.clear();
        for (Active* a : grp) {
          ok = ok && hipStreamWaitEvent(s, a->ready, 0) == hipSuccess;
          sv.push_back(a->S);
        }
        try {
          if (ok) iterations_grouped(sv.data(), (int)sv.size(), table, s);
        } catch (const HipError&) {
          ok = false;
        }
        for (Active* a : grp) ok = ok && hipEventRecord(a->ready, s) == hipSuccess;
        if (!ok) (void)hipStreamSynchronize(s);   // nothing may still run in a range that is given back
        lk.lock();
        for (Active* a : grp) {
          if (ok) fin_q.push_back(a);
          else complete(a, QDWHP_ERR_HIP);
        }
        cv_work.notify_all();
        continue;
      }
      if (stop && queue.empty() && running == 0) return;
      cv_work.wait(lk);
    }
  }

  // called with mu held
  void complete(Active* a, int st) {
    Request& q = reqs[a->id];
    q.t_done = Clock::now();
    q.status = st;
    q.info = a->info;
    --running;
    in_use -= a->bytes;
    alloc.give(a->off, a->bytes);
    if (a->S) solve_destroy(a->S);
    if (a->ready) (void)hipEventDestroy(a->ready);
    delete a;
    cv_done.notify_all();
    cv_work.notify_all();
  }
};

extern "C" int qdwhp_serve_create(size_t arena_bytes, int lanes, const qdwhp_opts* opts,
                                  qdwhp_server** out) {
  if (!out) return -4;
  *out = nullptr;
  if (lanes < 0) return -2;
  const int L = lanes > 0 ? lanes : (int)std::max<int64_t>(1, qdwhp_tune_get("serve.lanes", 3));
  const size_t tbytes = ((size_t)L * grouped_table_bytes(kMaxGroup) + 255) / 256 * 256;
  if (arena_bytes <= tbytes) return -1;
  auto* srv = new qdwhp_server();
  if (opts) srv->opts = *opts; else qdwhp_opts_default(&srv->opts);
  srv->grouped = qdwhp_tune_get("serve.grouped", 1) != 0;
  if (hipGetDevice(&srv->dev) != hipSuccess ||
      hipMalloc((void**)&srv->arena, arena_bytes) != hipSuccess) {
    delete srv;
    return QDWHP_ERR_HIP;
  }
  srv->cap = (arena_bytes - tbytes) / 256 * 256;
  srv->tables = srv->arena + srv->cap;
  srv->alloc = RangeAlloc(srv->cap);
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
  srv->nlanes = L;
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
                                 int64_t* groups, int64_t* grouped_requests, int reset) {
  if (!srv) return -1;
  std::lock_guard<std::mutex> g(srv->mu);
  if (peak_bytes) *peak_bytes = srv->peak_bytes;
  if (arena_bytes) *arena_bytes = srv->cap;
  if (peak_running) *peak_running = srv->peak_running;
  if (groups) *groups = srv->groups;
  if (grouped_requests) *grouped_requests = srv->grouped_reqs;
  if (reset) {
    srv->peak_bytes = srv->in_use;
    srv->peak_running = srv->running;
    srv->groups = srv->grouped_reqs = 0;
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
