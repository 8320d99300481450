// Shared definitions for the QDWHpartial HIP kernels (gfx950 / CDNA4).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace qdwhp {

typedef double v4d __attribute__((ext_vector_type(4)));

// Status codes mirrored from the public header.
enum {
  ST_OK = 0, ST_NONFINITE = 1, ST_NO_SUBSPACE = 2, ST_CHOL_BREAKDOWN = 3,
  ST_WORKSPACE = 4, ST_HIP = 5, ST_NOCONV = 6
};

struct HipError {
  hipError_t err;
};

#define QDWHP_HIP(call)                                                       \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) throw ::qdwhp::HipError{e_};                        \
  } while (0)

#define QDWHP_LAUNCH_CHECK() QDWHP_HIP(hipGetLastError())

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// ---------------------------------------------------------------- GEMM ----
// C = alpha * op(A) op(B) + beta * C (+ diag on the diagonal), column-major.
// Tile filter and per-tile K ranges let triangular operands and symmetric
// outputs skip work.
enum TileFilter { TILES_ALL = 0, TILES_UPPER = 1 };
enum KLo { KLO_ZERO = 0, KLO_ROW = 1, KLO_COL = 2 };
enum KHi { KHI_K = 0, KHI_ROW = 1, KHI_COL = 2 };

struct Gemm {
  int64_t M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  const double* A = nullptr; int64_t lda = 0; bool ta = false; int64_t sA = 0;
  const double* B = nullptr; int64_t ldb = 0; bool tb = false; int64_t sB = 0;
  double* C = nullptr; int64_t ldc = 0; int64_t sC = 0;
  int batch = 1;
  int tiles = TILES_ALL;
  int klo = KLO_ZERO, khi = KHI_K;
  int64_t koff = 0;      // offset subtracted from row0/col0 when forming K ranges
  double diag = 0.0;     // added to C(i,i) after the update (0: none)
  const double* Cin = nullptr;  // beta term read from Cin (ld ldcin) instead of C
  int64_t ldcin = 0, sCin = 0;
  // Read the stored A (or B) as unit lower trapezoidal (Householder vectors
  // kept below the diagonal of a geqrf result): entries above the diagonal
  // are 0 and the diagonal is 1.
  bool a_unit_lower = false, b_unit_lower = false;
  // Optional scratch for a deterministic split-K (partials summed in order).
  double* ws = nullptr; int64_t ws_doubles = 0;
  int splitk = 1;        // set by dgemm(); callers leave it at 1
  bool f32 = false;      // FP32 matrix cores (operands rounded to FP32, FP64 epilogue)
  // with f32: A and B are stored as FP32 (the pointers hold floats, leading
  // dimensions in floats), read at half the bytes; C stays FP64
  bool in32 = false;
  // alpha = dscal[ia] and beta = dscal[ib] (device memory) when set, so a
  // captured launch sequence can be replayed with new scalars
  const double* dscal = nullptr; int ia = -1, ib = -1;
};
void dgemm(const Gemm& g, hipStream_t s);
// Algorithmic flops of one GEMM call: 2 x (number of products the operation
// needs), honouring the upper-output and triangular K-range structure.
double gemm_flops(const Gemm& g);

// No-allocation mode of the calling thread (noalloc.hip): while set, the
// solve path creates no events, streams or graphs (phase timing off, the
// iterations run uncaptured, Jacobi updates H and V in one launch per round).
bool no_alloc_mode();

// ------------------------------------------------ helper streams ----
// A helper stream with a ring of event pairs, leased from a per-device pool
// (aux_stream.cpp): the sets live until the process ends, so a solve that
// overlaps work on a second stream creates no stream or event per call.
constexpr int kAuxRing = 4;
struct AuxSet {
  hipStream_t s;
  hipEvent_t ready[kAuxRing], done[kAuxRing];
};
class AuxLease {
 public:
  explicit AuxLease(int dev);
  ~AuxLease();     // waits for the helper stream, then returns the set to the pool
  AuxSet* operator->() const { return set_; }
  AuxLease(const AuxLease&) = delete;
  AuxLease& operator=(const AuxLease&) = delete;

 private:
  int dev_;
  AuxSet* set_ = nullptr;
};

// Live kernel timing (prof.cpp).
bool prof_active();
void prof_begin_launch(hipStream_t s, void** tok);
void prof_end_launch(hipStream_t s, void* tok, double flops);

// ------------------------------------------------------- small kernels ----
void fill(double* X, int64_t m, int64_t n, int64_t ld, double v, double diag, hipStream_t s);
void copy(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t s);
void mirror_upper(double* X, int64_t n, int64_t ld, hipStream_t s);
// dst[0..count) = vals (count <= 128) through kernel arguments: no host
// buffer outlives the call and the copy can sit in a captured graph.
void write_params(double* dst, const double* vals, int count, hipStream_t s);

// ------------------------------------------------- Cholesky / inverse ----
// Z (n x n SPD, upper triangle read) -> Z^{-1} (both triangles).  work holds
// spd_inverse_doubles(n) doubles; flag is a device int set to 1 on a
// non-positive or non-finite pivot (never cleared here).
int64_t spd_inverse_doubles(int64_t n);
// Z (upper triangle read) -> W^{-1} (n x n upper, zeros below, ld n) at the
// start of work (same size as spd_inverse); Z's upper triangle gets W.
void chol_inverse_factor(double* Z, int64_t n, int64_t ldz, double* work, int* flag, hipStream_t s);
void spd_inverse(double* Z, int64_t n, int64_t ldz, double* work, int* flag, hipStream_t s);

}  // namespace qdwhp
