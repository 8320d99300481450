// Ragged batches of independent EIG / SVD problems, in three phases.
//
//  1. setup (estimator, threshold, schedule, X0) on `lanes` concurrent HIP
//     streams, each fed by a host thread that takes the next instance
//     (largest first), with the instance's own slice of the workspace;
//  2. the DWH iterations, instances of one shape (type, rows, columns)
//     together: step i of every member whose step i is Cholesky-based runs as
//     one grouped Gram, one lockstep Cholesky-inversion (each leaf one launch
//     for all members, each product one grouped GEMM) and two grouped
//     triangular products, each a persistent launch over the members'
//     tiles; the shape groups are spread over the lanes ("batch.grouped" = 0
//     runs each instance's own steps on its lane instead);
//  3. projector QR, subspace and Rayleigh-Ritz on the lanes again; the last
//     product of every instance (V = Q2 W_k, or V = Q2 V~_k for SVD) runs in
//     one persistent ragged GEMM launch, followed by the sign steps.
//
// Every grouped launch performs each member's operations exactly as its
// standalone call would (same recursion, same tile arithmetic, no atomics),
// so each instance computes bitwise what a standalone qdwhp_eig / qdwhp_svd
// call computes, whatever else is in the batch.
#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"
#include "elem.h"

namespace qdwhp {

namespace {
std::mutex pool_mu;
std::map<int, std::vector<hipStream_t>> pool;
}  // namespace

hipStream_t lane_stream(int dev, int i) {
  std::lock_guard<std::mutex> g(pool_mu);
  auto& v = pool[dev];
  while ((int)v.size() <= i) {
    hipStream_t s;
    QDWHP_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    v.push_back(s);
  }
  return v[i];
}

size_t problem_workspace(const qdwhp_problem& p, const qdwhp_opts* o) {
  if (p.type == QDWHP_PROBLEM_EIG) return qdwhp_eig_workspace(p.n, p.fraction, o);
  return qdwhp_svd_workspace(p.m, p.n, p.k, o);
}

int run_problem(const qdwhp_problem& p, void* work, size_t lwork, const qdwhp_opts* o,
                hipStream_t s, qdwhp_info* info, Deferred* df) {
  if (p.type == QDWHP_PROBLEM_EIG)
    return eig_impl(p.A, p.n, p.lda, p.fraction, p.which, p.w, p.V, p.ldv, work, lwork, o, s, info, df);
  return svd_impl(p.A, p.m, p.n, p.lda, p.k, p.U, p.ldu, p.w, p.V, p.ldv, work, lwork, o, s, info, df);
}

double problem_cost(const qdwhp_problem& p) {
  const double n = (double)p.n, m = (p.type == QDWHP_PROBLEM_EIG) ? n : (double)p.m;
  return m * n * n;
}

}  // namespace qdwhp

using namespace qdwhp;

namespace {
size_t align256(size_t b) { return (b + 255) / 256 * 256; }

int default_lanes(int count, bool mixed) {
  const int64_t base = qdwhp_tune_get("batch.lanes", 8);
  const int64_t t = mixed ? qdwhp_tune_get("batch.lanes.mixed", base) : base;
  return (int)std::max<int64_t>(1, std::min<int64_t>(t, count));
}
}  // namespace

extern "C" size_t qdwhp_problem_workspace(const qdwhp_problem* p, const qdwhp_opts* opts) {
  if (!p) return 0;
  if (p->type != QDWHP_PROBLEM_EIG && p->type != QDWHP_PROBLEM_SVD) return 0;
  return problem_workspace(*p, opts);
}

extern "C" size_t qdwhp_batched_workspace(int count, const qdwhp_problem* probs, const qdwhp_opts* opts) {
  if (count <= 0 || !probs) return 0;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    const size_t b = qdwhp_problem_workspace(&probs[i], opts);
    if (b == 0) return 0;
    total += align256(b);
  }
  // the final grouped product's table, then one table slice per instance
  // for the shape groups of phase 2
  return total + align256(grouped_table_bytes(count)) + (size_t)count * grouped_table_bytes(1);
}

extern "C" int qdwhp_batched(int count, const qdwhp_problem* probs, void* work, size_t lwork,
                             const qdwhp_opts* opts, int lanes, void* stream, qdwhp_info* infos,
                             int* status) {
  if (count < 0) return -1;
  if (count == 0) return QDWHP_OK;
  if (!probs) return -2;
  if (!work) return -3;
  if (lanes < 0) return -6;
  const size_t need = qdwhp_batched_workspace(count, probs, opts);
  if (need == 0) return -2;
  if (lwork < need) return QDWHP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  std::vector<size_t> off(count);
  size_t o = 0;
  for (int i = 0; i < count; ++i) { off[i] = o; o += align256(problem_workspace(probs[i], opts)); }
  void* table = (char*)work + o;
  std::vector<qdwhp_info> inf(count);
  std::vector<int> st(count, QDWHP_OK);
  std::vector<Deferred> df(count);
  std::vector<SolveState*> S(count, nullptr);
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return problem_cost(probs[a]) > problem_cost(probs[b]); });
  const bool mixed = opts && opts->precision == QDWHP_MIXED_FP32;
  const int L = std::min(lanes > 0 ? lanes : default_lanes(count, mixed), count);
  const bool grouped = qdwhp_tune_get("batch.grouped", 1) != 0;
  int dev = 0;
  int rc = QDWHP_OK;
  std::vector<hipEvent_t> evs;
  auto event = [&]() {
    hipEvent_t e;
    QDWHP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    evs.push_back(e);
    return e;
  };
  try {
    QDWHP_HIP(hipGetDevice(&dev));
    hipEvent_t start = event();
    QDWHP_HIP(hipEventRecord(start, s));
    std::vector<hipStream_t> ls(L);
    for (int l = 0; l < L; ++l) {
      ls[l] = lane_stream(dev, l);
      QDWHP_HIP(hipStreamWaitEvent(ls[l], start, 0));
    }
    std::vector<int> lane_err(L, QDWHP_OK);
    // Runs phase(i, lane stream) for every instance on the lanes (host
    // threads take the next instance, largest first).
    auto on_lanes = [&](auto phase) {
      std::atomic<int> next(0);
      auto lane = [&](int l) {
        if (hipSetDevice(dev) != hipSuccess) { lane_err[l] = QDWHP_ERR_HIP; return; }
        for (int j; (j = next.fetch_add(1)) < count;) phase(order[j], ls[l]);
      };
      std::vector<std::thread> th;
      for (int l = 1; l < L; ++l) th.emplace_back(lane, l);
      lane(0);
      for (auto& t : th) t.join();
      for (int l = 0; l < L; ++l)
        if (lane_err[l] != QDWHP_OK) throw HipError{hipErrorUnknown};
    };
    auto join_into = [&](hipStream_t to) {
      for (int l = 0; l < L; ++l) {
        hipEvent_t e = event();
        QDWHP_HIP(hipEventRecord(e, ls[l]));
        QDWHP_HIP(hipStreamWaitEvent(to, e, 0));
      }
    };
    // phase 1: setup (estimator, threshold, schedule, X0)
    on_lanes([&](int i, hipStream_t ls_) {
      S[i] = solve_create(probs[i], (char*)work + off[i], align256(problem_workspace(probs[i], opts)), opts,
                          ls_, &inf[i], &df[i]);
      st[i] = solve_setup(S[i]);
    });
    // every lane waits for every other lane's setups
    auto cross_join = [&]() {
      std::vector<hipEvent_t> e(L);
      for (int l = 0; l < L; ++l) { e[l] = event(); QDWHP_HIP(hipEventRecord(e[l], ls[l])); }
      for (int l = 0; l < L; ++l)
        for (int j = 0; j < L; ++j)
          if (j != l) QDWHP_HIP(hipStreamWaitEvent(ls[l], e[j], 0));
    };
    // phase 2: the DWH iterations, one grouped run per shape (instances of
    // equal type and size share every launch), the groups spread over the lanes
    if (grouped) {
      cross_join();
      std::map<int64_t, std::vector<int>> by_shape;
      for (int j = 0; j < count; ++j)
        if (st[order[j]] == QDWHP_OK) by_shape[solve_shape(S[order[j]])].push_back(order[j]);
      std::vector<std::vector<int>> groups;
      for (auto& kv : by_shape) groups.push_back(kv.second);
      std::stable_sort(groups.begin(), groups.end(), [&](const std::vector<int>& a, const std::vector<int>& b) {
        return problem_cost(probs[a[0]]) * a.size() > problem_cost(probs[b[0]]) * b.size();
      });
      std::vector<size_t> toff(groups.size());
      size_t t = 0;
      for (size_t gi = 0; gi < groups.size(); ++gi) { toff[gi] = t; t += grouped_table_bytes((int)groups[gi].size()); }
      char* tables = (char*)table + align256(grouped_table_bytes(count));
      std::atomic<int> next(0);
      auto lane = [&](int l) {
        if (hipSetDevice(dev) != hipSuccess) { lane_err[l] = QDWHP_ERR_HIP; return; }
        try {
          for (int gi; (gi = next.fetch_add(1)) < (int)groups.size();) {
            std::vector<SolveState*> v;
            for (int i : groups[gi]) v.push_back(S[i]);
            iterations_grouped(v.data(), (int)v.size(), tables + toff[gi], ls[l]);
          }
        } catch (const HipError&) {
          lane_err[l] = QDWHP_ERR_HIP;
        }
      };
      std::vector<std::thread> th;
      for (int l = 1; l < L; ++l) th.emplace_back(lane, l);
      lane(0);
      for (auto& x : th) x.join();
      for (int l = 0; l < L; ++l)
        if (lane_err[l] != QDWHP_OK) throw HipError{hipErrorUnknown};
      cross_join();
    }
    // phase 3: projector, subspace, Rayleigh-Ritz (and phase 2 per lane when not grouped)
    on_lanes([&](int i, hipStream_t ls_) {
      if (st[i] != QDWHP_OK) return;
      solve_set_stream(S[i], ls_);
      if (!grouped) st[i] = solve_iterate(S[i]);
      if (st[i] == QDWHP_OK) st[i] = solve_finish(S[i]);
    });
    join_into(s);
    // deferred products of every successful instance: one ragged launch
    std::vector<GroupedDesc> gd;
    std::vector<int> who;
    for (int i = 0; i < count; ++i) {
      if (st[i] != QDWHP_OK) continue;
      const Gemm& g = df[i].g;
      gd.push_back(GroupedDesc{g.M, g.N, g.K, g.alpha, g.beta, g.A, g.lda, g.B, g.ldb, g.C, g.ldc});
      who.push_back(i);
    }
    dgemm_grouped(gd.data(), (int)gd.size(), false, false, table, s);
    for (int i : who) {
      const Deferred& d = df[i];
      sign_normalize(d.V, d.ldv, d.n, d.k, d.U, d.ldu, d.m, s);
    }
  } catch (const HipError&) {
    rc = QDWHP_ERR_HIP;
  }
  // the states are released once their work has drained
  (void)hipStreamSynchronize(s);
  for (auto* p : S) if (p) solve_destroy(p);
  for (auto e : evs) (void)hipEventDestroy(e);
  for (int i = 0; i < count; ++i) {
    if (infos) infos[i] = inf[i];
    if (status) status[i] = st[i];
    if (rc == QDWHP_OK && st[i] != QDWHP_OK) rc = st[i];
  }
  return rc;
}

extern "C" size_t qdwhp_dgemm_grouped_workspace(int count) {
  return count > 0 ? grouped_table_bytes(count) : 0;
}

extern "C" int qdwhp_dgemm_grouped(int count, int transa, int transb, const int64_t* m, const int64_t* n,
                                   const int64_t* k, const double* alpha, const double* const* A,
                                   const int64_t* lda, const double* const* B, const int64_t* ldb,
                                   const double* beta, double* const* C, const int64_t* ldc,
                                   void* work, size_t lwork, void* stream) {
  if (count < 0) return -1;
  if (count == 0) return QDWHP_OK;
  if (!m || !n || !k || !alpha || !A || !lda || !B || !ldb || !beta || !C || !ldc) return -4;
  if (!work) return -16;
  if (lwork < grouped_table_bytes(count)) return QDWHP_ERR_WORKSPACE;
  std::vector<GroupedDesc> d(count);
  for (int i = 0; i < count; ++i) {
    const int64_t ar = transa ? k[i] : m[i], br = transb ? n[i] : k[i];
    if (m[i] < 0 || n[i] < 0 || k[i] < 0) return -4;
    if (lda[i] < std::max<int64_t>(1, ar) || ldb[i] < std::max<int64_t>(1, br) ||
        ldc[i] < std::max<int64_t>(1, m[i]))
      return -9;
    if ((m[i] > 0 && n[i] > 0) && (!C[i] || (k[i] > 0 && (!A[i] || !B[i])))) return -8;
    d[i] = GroupedDesc{m[i], n[i], k[i], alpha[i], beta[i], A[i], lda[i], B[i], ldb[i], C[i], ldc[i]};
  }
  try {
    dgemm_grouped(d.data(), count, transa != 0, transb != 0, work, (hipStream_t)stream);
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}
