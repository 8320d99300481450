// Capture-once / replay-many launch sequences (graphs.cpp).
#pragma once
#include <cstdint>
#include <functional>
#include <vector>

#include "common.h"

namespace qdwhp {
// Replays the graph stored under `key` on s, or captures body() (which must
// only enqueue work on s: no host synchronisation, no memset nodes) into a
// new graph, stores and launches it.  Returns false (nothing enqueued) when
// capture is not possible; the caller then runs body() directly.
bool graph_replay(const std::vector<int64_t>& key, hipStream_t s, const std::function<void()>& body);
size_t graph_count();
}  // namespace qdwhp
