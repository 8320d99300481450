// QDWHpartial-EIG without any allocation by the library or the caller: the
// solve's workspace is a fixed device array of this file, for callers that
// cannot allocate device memory (code between graph-capture boundaries,
// tight serving loops, harnesses that forbid hipMalloc).
//
// The array is a file-scope __device__ variable, so every GPU the library
// runs on holds its own copy for the life of the process.  Host code never
// passes the array's name to a kernel (on the host it is only a stand-in
// symbol): the first call on a device, with that device current, looks up
// the copy's device address with hipGetSymbolAddress and keeps it per device.
// The solve then runs exactly as qdwhp_eig with that address as its
// workspace (same kernels and launch shapes, so the results are bitwise the
// same), with the library's other allocations switched off for the call:
// no phase-timing events, no captured graphs, no helper stream for the
// Jacobi updates.  Everything the solve reads from the workspace before
// writing it (flags, counters) it clears itself on the stream.
#include <cstring>
#include <mutex>

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"

namespace {

constexpr size_t kScratchBytes = (size_t)QDWHP_NOALLOC_MAX_BYTES;
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex ptr_mu;
void* scratch_ptr[kMaxDevices] = {};

thread_local bool tl_no_alloc = false;

struct NoAllocScope {
  NoAllocScope() { tl_no_alloc = true; }
  ~NoAllocScope() { tl_no_alloc = false; }
};

// Device address of this device's copy of the array (nullptr on failure).
void* device_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(ptr_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_ptr[dev] = p;
  }
  return scratch_ptr[dev];
}

}  // namespace

namespace qdwhp {
bool no_alloc_mode() { return tl_no_alloc; }
}  // namespace qdwhp

extern "C" size_t qdwhp_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" int qdwhp_eig_noalloc(const double* A, int64_t n, int64_t lda, double fraction, int which,
                                 double* w, double* V, int64_t ldv, const qdwhp_opts* opts, void* stream,
                                 qdwhp_info* info) {
  qdwhp_info dummy;
  if (!info) info = &dummy;
  if (n >= 1 && fraction > 0.0 && fraction <= 1.0) {
    qdwhp_opts o;
    if (opts) o = *opts; else qdwhp_opts_default(&o);
    if (qdwhp_eig_workspace(n, fraction, &o) > kScratchBytes) {
      std::memset(info, 0, sizeof(*info));
      info->status = QDWHP_ERR_WORKSPACE;
      return QDWHP_ERR_WORKSPACE;
    }
  }
  void* ws = device_scratch();
  if (!ws) {
    std::memset(info, 0, sizeof(*info));
    info->status = QDWHP_ERR_HIP;
    return QDWHP_ERR_HIP;
  }
  NoAllocScope scope;
  return qdwhp::eig_impl(A, n, lda, fraction, which, w, V, ldv, ws, kScratchBytes, opts, stream, info,
                         nullptr);
}
