// Pool of helper streams with event rings (see common.h): a leased set is
// returned when its lease ends and reused by the next lease on that device.
#include <map>
#include <mutex>
#include <vector>

#include "common.h"

namespace qdwhp {
namespace {
std::mutex aux_mu;
std::map<int, std::vector<AuxSet*>> aux_free;   // per device; sets live until the process ends
}  // namespace

AuxLease::AuxLease(int dev) : dev_(dev) {
  {
    std::lock_guard<std::mutex> g(aux_mu);
    auto& v = aux_free[dev];
    if (!v.empty()) { set_ = v.back(); v.pop_back(); }
  }
  if (!set_) {
    AuxSet* a = new AuxSet;
    QDWHP_HIP(hipStreamCreateWithFlags(&a->s, hipStreamNonBlocking));
    for (int i = 0; i < kAuxRing; ++i) {
      QDWHP_HIP(hipEventCreateWithFlags(&a->ready[i], hipEventDisableTiming));
      QDWHP_HIP(hipEventCreateWithFlags(&a->done[i], hipEventDisableTiming));
    }
    set_ = a;
  }
}

AuxLease::~AuxLease() {
  // work still queued (an error path) finishes before the set is reused
  (void)hipStreamSynchronize(set_->s);
  std::lock_guard<std::mutex> g(aux_mu);
  aux_free[dev_].push_back(set_);
}

}  // namespace qdwhp
