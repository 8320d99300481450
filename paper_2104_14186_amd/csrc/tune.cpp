// Tuning table: named integer parameters that launch-shape decisions read
// (GEMM tile size for small launches, lanes of the batch and serving
// runtimes).  The autotuner measures candidates on the device and stores its
// choices here; unset keys fall back to the built-in defaults.
#include <map>
#include <mutex>
#include <string>

#include "qdwhp.h"

namespace {
std::mutex mu;
std::map<std::string, int64_t>& table() {
  static std::map<std::string, int64_t> t;
  return t;
}
}  // namespace

extern "C" int qdwhp_tune_set(const char* key, int64_t value) {
  if (!key || !*key) return -1;
  std::lock_guard<std::mutex> g(mu);
  table()[key] = value;
  return QDWHP_OK;
}

extern "C" int64_t qdwhp_tune_get(const char* key, int64_t fallback) {
  if (!key) return fallback;
  std::lock_guard<std::mutex> g(mu);
  auto it = table().find(key);
  return it == table().end() ? fallback : it->second;
}

// "key@b" for the power-of-two bucket b = ceil(log2(size)) of a size, else
// "key", else the fallback: size-dependent choices (the autotuner writes
// per-bucket entries where a choice changes with the size).
extern "C" int64_t qdwhp_tune_get_sized(const char* key, int64_t size, int64_t fallback) {
  if (!key) return fallback;
  int b = 0;
  while (b < 62 && ((int64_t)1 << b) < size) ++b;
  const std::string sized = std::string(key) + "@" + std::to_string(b);
  std::lock_guard<std::mutex> g(mu);
  auto it = table().find(sized);
  if (it != table().end()) return it->second;
  it = table().find(key);
  return it == table().end() ? fallback : it->second;
}

extern "C" void qdwhp_tune_clear(void) {
  std::lock_guard<std::mutex> g(mu);
  table().clear();
}
