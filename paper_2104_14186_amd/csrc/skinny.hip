// Products with few right-hand columns, C (m x nv) = alpha A (m x k) B
// (k x nv) and C (n x nv) = alpha A^T B, for the Krylov blocks of the estimator (a few Lanczos steps open
// Algorithms 1 and 2).  With nv = 8 such a product is bound by reading A
// once from HBM; a 64-wide matrix-core tile would spend 8x its work on
// padding and leave most of the chip idle.  One thread per row of A: for
// each k it reads A[i][k] (consecutive rows on consecutive lanes) and
// updates nv sums with B[k][:] from LDS.  k is split over workgroups;
// partial sums are added in split order by a second kernel, so results
// are reproducible bit for bit.
#include "common.h"
#include "skinny.h"

namespace qdwhp {
namespace {

constexpr int ST = 256;   // threads (rows) per workgroup
constexpr int KC = 128;   // k values staged per pass
constexpr int KMIN = 32;  // fewest k values of one split

template <int NVC>
__global__ __launch_bounds__(ST) void skinny_kernel(const double* A, int64_t lda, int64_t m, int64_t k,
                                                    const double* B, int64_t ldb, int nv, int64_t kchunk,
                                                    double* part) {
  __shared__ double Bs[KC][NVC];
  const int64_t i = (int64_t)blockIdx.x * ST + threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.y * kchunk;
  const int64_t k1 = (k0 + kchunk < k) ? k0 + kchunk : k;
  double acc[NVC];
#pragma unroll
  for (int j = 0; j < NVC; ++j) acc[j] = 0.0;
  for (int64_t kb = k0; kb < k1; kb += KC) {
    const int kn = (int)((k1 - kb) < KC ? (k1 - kb) : KC);
    __syncthreads();
    for (int e = threadIdx.x; e < KC * NVC; e += ST) {
      const int kk = e % KC, j = e / KC;
      Bs[kk][j] = (kk < kn && j < nv) ? B[(kb + kk) + (int64_t)j * ldb] : 0.0;
    }
    __syncthreads();
    if (i < m) {
      const double* Ai = A + i + kb * lda;
      int kk = 0;
      for (; kk + 8 <= kn; kk += 8) {   // eight independent loads in flight
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = Ai[(int64_t)(kk + u) * lda];
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
          for (int j = 0; j < NVC; ++j) acc[j] += a[u] * Bs[kk + u][j];
      }
      for (; kk < kn; ++kk) {
        const double a = Ai[(int64_t)kk * lda];
#pragma unroll
        for (int j = 0; j < NVC; ++j) acc[j] += a * Bs[kk][j];
      }
    }
  }
  if (i < m) {
    double* p = part + (int64_t)blockIdx.y * m * NVC;
#pragma unroll
    for (int j = 0; j < NVC; ++j)
      if (j < nv) p[i + (int64_t)j * m] = acc[j];
  }
}

__global__ void skinny_reduce(const double* part, int64_t m, int nvc, int nv, int splits, double alpha,
                              double* C, int64_t ldc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= m || j >= nv) return;
  double s = 0.0;
  for (int z = 0; z < splits; ++z) s += part[(int64_t)z * m * nvc + i + (int64_t)j * m];
  C[i + (int64_t)j * ldc] = alpha * s;
}

template <int NVC>
void launch(const double* A, int64_t lda, int64_t m, int64_t k, const double* B, int64_t ldb, int nv,
            double alpha, double* C, int64_t ldc, double* ws, int64_t ws_doubles, hipStream_t s) {
  // Small m has few row blocks, so k is split finely (down to KMIN values
  // per split) to keep enough workgroups reading A at once; large m splits
  // k coarsely and reads A in long runs.
  const int64_t rb = cdiv(m, ST);
  int64_t S = cdiv(1024, rb);                       // about 1024 workgroups
  const int64_t smax_k = cdiv(k, KMIN);
  if (S > smax_k) S = smax_k;
  const int64_t smax_ws = ws_doubles / (m * NVC);
  if (S > smax_ws) S = smax_ws;
  if (S > 64) S = 64;
  if (S < 1) throw HipError{hipErrorInvalidValue};   // workspace below one split
  const int64_t kchunk = cdiv(cdiv(k, S), KMIN) * KMIN;
  S = cdiv(k, kchunk);
  skinny_kernel<NVC><<<dim3((unsigned)rb, (unsigned)S), ST, 0, s>>>(A, lda, m, k, B, ldb, nv, kchunk, ws);
  QDWHP_LAUNCH_CHECK();
  skinny_reduce<<<dim3((unsigned)cdiv(m, 256), (unsigned)nv), 256, 0, s>>>(ws, m, NVC, nv, (int)S, alpha, C, ldc);
  QDWHP_LAUNCH_CHECK();
}

// C (n x nv) = alpha A^T B for A m x n (lda), B m x nv: CT columns of A per
// workgroup; a thread runs over rows t, t + ST, ... of its columns and keeps
// CT x NVC sums, which the workgroup then adds (butterflies inside each
// wave, then the four waves in order), so results are reproducible.
constexpr int CT = 8;   // columns of A per workgroup

template <int NVC>
__global__ __launch_bounds__(ST) void skinny_t_kernel(const double* A, int64_t lda, int64_t m, int64_t n,
                                                      const double* B, int64_t ldb, int nv, double alpha,
                                                      double* C, int64_t ldc) {
  __shared__ double red[ST / 64][CT * NVC];
  const int64_t c0 = (int64_t)blockIdx.x * CT;
  double acc[CT][NVC];
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int j = 0; j < NVC; ++j) acc[c][j] = 0.0;
  for (int64_t r = threadIdx.x; r < m; r += ST) {
    double b[NVC], a[CT];
#pragma unroll
    for (int j = 0; j < NVC; ++j) b[j] = (j < nv) ? B[r + (int64_t)j * ldb] : 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c) a[c] = (c0 + c < n) ? A[r + (c0 + c) * lda] : 0.0;
#pragma unroll
    for (int c = 0; c < CT; ++c)
#pragma unroll
      for (int j = 0; j < NVC; ++j) acc[c][j] += a[c] * b[j];
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CT; ++c)
#pragma unroll
    for (int j = 0; j < NVC; ++j) {
      double v = acc[c][j];
      for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
      if (lane == 0) red[wv][c * NVC + j] = v;
    }
  __syncthreads();
  for (int e = threadIdx.x; e < CT * NVC; e += ST) {
    const int c = e / NVC, j = e % NVC;
    if (c0 + c < n && j < nv) {
      double v = red[0][e];
      for (int w = 1; w < ST / 64; ++w) v += red[w][e];
      C[(c0 + c) + (int64_t)j * ldc] = alpha * v;
    }
  }
}

}  // namespace

void skinny_gemm_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* B, int64_t ldb, int nv,
                   double alpha, double* C, int64_t ldc, hipStream_t s) {
  if (n <= 0 || nv <= 0) return;
  if (nv > 8) throw HipError{hipErrorInvalidValue};
  if (m <= 0) {
    fill(C, n, nv, ldc, 0.0, 0.0, s);
    return;
  }
  skinny_t_kernel<8><<<(unsigned)cdiv(n, CT), ST, 0, s>>>(A, lda, m, n, B, ldb, nv, alpha, C, ldc);
  QDWHP_LAUNCH_CHECK();
}

// Room for 16 splits of k (fewer when a caller passes less).
int64_t skinny_ws_doubles(int64_t m, int nv) { return 16 * m * (nv <= 8 ? 8 : nv <= 16 ? 16 : 32); }

void skinny_gemm(const double* A, int64_t lda, int64_t m, int64_t k, const double* B, int64_t ldb, int nv,
                 double alpha, double* C, int64_t ldc, double* ws, int64_t ws_doubles, hipStream_t s) {
  if (m <= 0 || nv <= 0) return;
  if (nv > 32) throw HipError{hipErrorInvalidValue};
  if (k <= 0) {
    fill(C, m, nv, ldc, 0.0, 0.0, s);
    return;
  }
  if (nv <= 8) launch<8>(A, lda, m, k, B, ldb, nv, alpha, C, ldc, ws, ws_doubles, s);
  else if (nv <= 16) launch<16>(A, lda, m, k, B, ldb, nv, alpha, C, ldc, ws, ws_doubles, s);
  else launch<32>(A, lda, m, k, B, ldb, nv, alpha, C, ldc, ws, ws_doubles, s);
}

}  // namespace qdwhp
