// Captured launch sequences (hipGraphs) of the static part of a solve.
//
// Once the threshold and the step kinds are fixed, the DWH iterations are a
// fixed sequence of launches on fixed workspace buffers; only the weights
// change from solve to solve, and the steps read those from a device
// parameter block.  The first solve with a given key (workspace buffers,
// sizes, step kinds, precision plan) records the sequence into a graph;
// later solves with the same key replay it with one launch.  Entries live
// until qdwhp_graphs_clear (which waits for the device first) or the end of
// the process; beyond kMaxGraphs keys, sequences run uncaptured.
#include <map>
#include <mutex>
#include <vector>

#include "qdwhp.h"
#include "common.h"
#include "graphs.h"

namespace qdwhp {
namespace {
constexpr size_t kMaxGraphs = 256;
std::mutex mu;
std::map<std::vector<int64_t>, hipGraphExec_t>& cache() {
  static std::map<std::vector<int64_t>, hipGraphExec_t> c;
  return c;
}
}  // namespace

bool graph_replay(const std::vector<int64_t>& key, hipStream_t s, const std::function<void()>& body) {
  if (s == nullptr) return false;   // the legacy default stream cannot be captured
  {
    std::lock_guard<std::mutex> g(mu);
    auto it = cache().find(key);
    if (it != cache().end()) {
      QDWHP_HIP(hipGraphLaunch(it->second, s));
      return true;
    }
    if (cache().size() >= kMaxGraphs) return false;
  }
  QDWHP_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  hipGraph_t graph = nullptr;
  try {
    body();
  } catch (...) {
    (void)hipStreamEndCapture(s, &graph);
    if (graph) (void)hipGraphDestroy(graph);
    throw;
  }
  QDWHP_HIP(hipStreamEndCapture(s, &graph));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  QDWHP_HIP(e);
  {
    std::lock_guard<std::mutex> g(mu);
    auto ins = cache().emplace(key, exec);
    if (!ins.second) {   // another thread captured the same key meanwhile
      (void)hipGraphExecDestroy(exec);
      exec = ins.first->second;
    }
  }
  QDWHP_HIP(hipGraphLaunch(exec, s));
  return true;
}

size_t graph_count() {
  std::lock_guard<std::mutex> g(mu);
  return cache().size();
}

}  // namespace qdwhp

extern "C" int qdwhp_graphs_clear(void) {
  std::lock_guard<std::mutex> g(qdwhp::mu);
  if (qdwhp::cache().empty()) return QDWHP_OK;
  // no replay may still be running when its executable goes
  if (hipDeviceSynchronize() != hipSuccess) return QDWHP_ERR_HIP;
  for (auto& e : qdwhp::cache()) (void)hipGraphExecDestroy(e.second);
  qdwhp::cache().clear();
  return QDWHP_OK;
}

extern "C" int64_t qdwhp_graphs_count(void) { return (int64_t)qdwhp::graph_count(); }
