// Ragged batches of independent EIG / SVD problems.
//
// A batch of uneven sizes runs on `lanes` concurrent HIP streams, each fed
// by a host thread that takes the next instance (largest first) and drives
// its solve on the lane's stream with the instance's own slice of the
// workspace.  The solves of small instances are latency-bound (many short
// launches and a few host round trips), so instances on different lanes
// overlap on the device.  The last matrix product of every instance
// (V = Q2 W_k, or V = Q2 V~_k for SVD) is deferred and all of them run in
// one persistent ragged GEMM launch on the caller's stream, followed by the
// sign steps.
//
// Each instance computes exactly what a standalone qdwhp_eig / qdwhp_svd call
// computes: the same kernels with the same launch shapes (no choice depends
// on the batch composition) and no atomics whose order could vary, so the
// results are bitwise identical.
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

int default_lanes(int count) {
  const int64_t t = qdwhp_tune_get("batch.lanes", 8);
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
  return total + align256(grouped_table_bytes(count));
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
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return problem_cost(probs[a]) > problem_cost(probs[b]); });
  const int L = std::min(lanes > 0 ? lanes : default_lanes(count), count);
  int dev = 0;
  int rc = QDWHP_OK;
  std::vector<hipEvent_t> evs;
  try {
    QDWHP_HIP(hipGetDevice(&dev));
    hipEvent_t start;
    QDWHP_HIP(hipEventCreateWithFlags(&start, hipEventDisableTiming));
    evs.push_back(start);
    QDWHP_HIP(hipEventRecord(start, s));
    std::vector<hipStream_t> ls(L);
    for (int l = 0; l < L; ++l) {
      ls[l] = lane_stream(dev, l);
      QDWHP_HIP(hipStreamWaitEvent(ls[l], start, 0));
    }
    std::atomic<int> next(0);
    std::vector<int> lane_err(L, QDWHP_OK);
    auto lane = [&](int l) {
      if (hipSetDevice(dev) != hipSuccess) { lane_err[l] = QDWHP_ERR_HIP; return; }
      for (int j; (j = next.fetch_add(1)) < count;) {
        const int i = order[j];
        st[i] = run_problem(probs[i], (char*)work + off[i], align256(problem_workspace(probs[i], opts)),
                            opts, ls[l], &inf[i], &df[i]);
      }
    };
    std::vector<std::thread> th;
    for (int l = 1; l < L; ++l) th.emplace_back(lane, l);
    lane(0);
    for (auto& t : th) t.join();
    for (int l = 0; l < L; ++l) {
      if (lane_err[l] != QDWHP_OK) throw HipError{hipErrorUnknown};
      hipEvent_t e;
      QDWHP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
      evs.push_back(e);
      QDWHP_HIP(hipEventRecord(e, ls[l]));
      QDWHP_HIP(hipStreamWaitEvent(s, e, 0));
    }
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
