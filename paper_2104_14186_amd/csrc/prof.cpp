// Live per-launch timing of the GEMM kernel (hipEvents on the launch stream)
// with the algorithmic flop count of each launch, for roofline reporting.
#include <mutex>
#include <vector>

#include "qdwhp.h"
#include "common.h"

namespace qdwhp {
namespace {

struct Pending { hipEvent_t a, b; double flops; };
std::mutex mu;
bool active = false;
std::vector<Pending> pending;
std::vector<hipEvent_t> pool;

hipEvent_t get_event() {
  if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
  hipEvent_t e;
  QDWHP_HIP(hipEventCreate(&e));
  return e;
}

}  // namespace

bool prof_active() { return active; }

void prof_begin_launch(hipStream_t s, void** tok) {
  std::lock_guard<std::mutex> g(mu);
  Pending p{get_event(), get_event(), 0.0};
  QDWHP_HIP(hipEventRecord(p.a, s));
  pending.push_back(p);
  *tok = (void*)(pending.size());
}

void prof_end_launch(hipStream_t s, void* tok, double flops) {
  std::lock_guard<std::mutex> g(mu);
  Pending& p = pending[(size_t)tok - 1];
  QDWHP_HIP(hipEventRecord(p.b, s));
  p.flops = flops;
}

}  // namespace qdwhp

using namespace qdwhp;

extern "C" void qdwhp_profile_begin(void) {
  std::lock_guard<std::mutex> g(mu);
  active = true;
}

extern "C" int qdwhp_profile_end(double* flops, double* ms, int64_t* launches) {
  std::lock_guard<std::mutex> g(mu);
  active = false;
  double f = 0.0, t = 0.0;
  try {
    for (auto& p : pending) {
      QDWHP_HIP(hipEventSynchronize(p.b));
      float e = 0.f;
      QDWHP_HIP(hipEventElapsedTime(&e, p.a, p.b));
      t += e;
      f += p.flops;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
  } catch (const HipError&) {
    pending.clear();
    return QDWHP_ERR_HIP;
  }
  if (flops) *flops = f;
  if (ms) *ms = t;
  if (launches) *launches = (int64_t)pending.size();
  pending.clear();
  return QDWHP_OK;
}
