// Elementwise and reduction kernels of the solve drivers.
#include "common.h"
#include "elem.h"

namespace qdwhp {
namespace {

constexpr int TT = 64;   // tile edge of the transposing kernels

// X = f (tau I - sgn A) - s I        (scaled and shifted matrix, Sec. 4.1)
__global__ void eig_x0_kernel(const double* A, int64_t lda, double* X, int64_t ldx, int64_t n,
                              double f, double tau, double sgn, double s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    if (i >= n) continue;
    double v = -f * sgn * A[i + j * lda];
    if (i == j) v += f * tau - s;
    X[i + j * ldx] = v;
  }
}

// X (rows x cols) = op(A) / alpha, op = transpose when trans (A is cols x rows).
__global__ __launch_bounds__(256) void scale_t_kernel(const double* A, int64_t lda, double* X, int64_t ldx,
                                                      int64_t rows, int64_t cols, double inv, int trans) {
  __shared__ double T[TT][TT + 1];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * TT, c0 = (int64_t)blockIdx.y * TT;
  if (!trans) {
    for (int yy = ty; yy < TT; yy += 4) {
      const int64_t r = r0 + tx, c = c0 + yy;
      if (r < rows && c < cols) X[r + c * ldx] = A[r + c * lda] * inv;
    }
    return;
  }
  // X[r][c] = A[c][r]: read A tile rows c0.., cols r0..
  for (int yy = ty; yy < TT; yy += 4) {
    const int64_t ar = c0 + tx, ac = r0 + yy;
    T[yy][tx] = (ar < cols && ac < rows) ? A[ar + ac * lda] : 0.0;   // T[r - r0][c - c0]
  }
  __syncthreads();
  for (int yy = ty; yy < TT; yy += 4) {
    const int64_t r = r0 + tx, c = c0 + yy;
    if (r < rows && c < cols) X[r + c * ldx] = T[tx][yy] * inv;
  }
}

// W = [sqrt(c) X; I]   ((m + n) x n)
__global__ void stacked_kernel(const double* X, int64_t ldx, double* W, int64_t ldw, int64_t m, int64_t n,
                               double sc, const double* dsc) {
  if (dsc) sc = *dsc;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    if (i < m) W[i + j * ldw] = sc * X[i + j * ldx];
    else if (i < m + n) W[i + j * ldw] = (i - m == j) ? 1.0 : 0.0;
  }
}

// X <- (X + X^T)/2 on TT x TT tile pairs (bi >= bj).
__global__ __launch_bounds__(256) void symmetrize_kernel(double* X, int64_t n, int64_t ld) {
  __shared__ double U[TT][TT + 1];
  __shared__ double L[TT][TT + 1];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = bi * TT, c0 = bj * TT;   // lower tile rows r0.., cols c0..
  for (int yy = ty; yy < TT; yy += 4) {
    const int64_t r = r0 + tx, c = c0 + yy;
    L[tx][yy] = (r < n && c < n) ? X[r + c * ld] : 0.0;            // L[r-r0][c-c0]
    const int64_t ur = c0 + tx, uc = r0 + yy;                      // upper tile
    U[tx][yy] = (ur < n && uc < n) ? X[ur + uc * ld] : 0.0;        // U[ur-c0][uc-r0]
  }
  __syncthreads();
  for (int yy = ty; yy < TT; yy += 4) {
    // lower element (r0+tx, c0+yy) pairs with upper (c0+yy, r0+tx) = U[yy][tx]
    const int64_t r = r0 + tx, c = c0 + yy;
    const double avg = 0.5 * (L[tx][yy] + U[yy][tx]);
    if (r < n && c < n) X[r + c * ld] = avg;
    const int64_t ur = c0 + tx, uc = r0 + yy;
    const double avg2 = 0.5 * (U[tx][yy] + L[yy][tx]);
    if (ur < n && uc < n) X[ur + uc * ld] = avg2;
  }
}

// B = (X + I)/2 (Algorithm 1 projector).
__global__ void half_plus_i_kernel(const double* X, int64_t ldx, double* B, int64_t ldb, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    if (i < n) B[i + j * ldb] = 0.5 * (X[i + j * ldx] + (i == j ? 1.0 : 0.0));
}

__global__ void to_f32_kernel(const double* X, int64_t ldx, float* Y, int64_t ldy, int64_t m, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    if (i < m) Y[i + j * ldy] = (float)X[i + j * ldx];
}

__global__ void diag_kernel(const double* A, int64_t lda, int64_t n, double* d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = A[i + i * lda];
}

// R (n x n) = upper triangle of A (zeros below).
__global__ void upper_copy_kernel(const double* A, int64_t lda, double* R, int64_t ldr, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    if (i < n) R[i + j * ldr] = (i <= j) ? A[i + j * lda] : 0.0;
}

// Column j of V: largest |entry| (lowest index on ties) made positive; the
// same flip applied to column j of U (if any).
__global__ __launch_bounds__(256) void sign_kernel(double* V, int64_t ldv, int64_t rows, double* U,
                                                   int64_t ldu, int64_t urows) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int64_t j = blockIdx.x;
  double best = -1.0;
  int64_t idx = 0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) {
    const double a = fabs(V[r + j * ldv]);
    if (a > best) { best = a; idx = r; }
  }
  bv[threadIdx.x] = best; bi[threadIdx.x] = idx;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double ob = bv[threadIdx.x + s];
      const int64_t oi = bi[threadIdx.x + s];
      if (ob > bv[threadIdx.x] || (ob == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = ob; bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool flip = V[bi[0] + j * ldv] < 0.0;
  if (!flip) return;
  for (int64_t r = threadIdx.x; r < rows; r += 256) V[r + j * ldv] = -V[r + j * ldv];
  if (U)
    for (int64_t r = threadIdx.x; r < urows; r += 256) U[r + j * ldu] = -U[r + j * ldu];
}

__global__ void scale_vec_kernel(const double* x, double* y, int64_t n, double a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// flag = 1 if any entry of the m x n matrix is not finite.
__global__ void nonfinite_kernel(const double* A, int64_t lda, int64_t m, int64_t n, int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    if (i < m && !isfinite(A[i + j * lda])) *flag = 1;
}

inline dim3 grid2(int64_t m, int64_t n) {
  return dim3((unsigned)cdiv(m, 256), (unsigned)(n < 65535 ? n : 65535));
}

}  // namespace

void eig_x0(const double* A, int64_t lda, double* X, int64_t ldx, int64_t n, double f, double tau,
            double sgn, double s, hipStream_t st) {
  eig_x0_kernel<<<grid2(n, n), 256, 0, st>>>(A, lda, X, ldx, n, f, tau, sgn, s);
  QDWHP_LAUNCH_CHECK();
}
void scale_copy(const double* A, int64_t lda, double* X, int64_t ldx, int64_t rows, int64_t cols,
                double inv, bool trans, hipStream_t st) {
  scale_t_kernel<<<dim3((unsigned)cdiv(rows, TT), (unsigned)cdiv(cols, TT)), 256, 0, st>>>(
      A, lda, X, ldx, rows, cols, inv, trans ? 1 : 0);
  QDWHP_LAUNCH_CHECK();
}
void stacked(const double* X, int64_t ldx, double* W, int64_t ldw, int64_t m, int64_t n, double sc,
             hipStream_t st, const double* dsc) {
  stacked_kernel<<<grid2(m + n, n), 256, 0, st>>>(X, ldx, W, ldw, m, n, sc, dsc);
  QDWHP_LAUNCH_CHECK();
}
void symmetrize(double* X, int64_t n, int64_t ld, hipStream_t st) {
  const unsigned t = (unsigned)cdiv(n, TT);
  symmetrize_kernel<<<dim3(t, t), 256, 0, st>>>(X, n, ld);
  QDWHP_LAUNCH_CHECK();
}
void to_f32(const double* X, int64_t ldx, float* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st) {
  if (m <= 0 || n <= 0) return;
  to_f32_kernel<<<grid2(m, n), 256, 0, st>>>(X, ldx, Y, ldy, m, n);
  QDWHP_LAUNCH_CHECK();
}
void half_plus_identity(const double* X, int64_t ldx, double* B, int64_t ldb, int64_t n, hipStream_t st) {
  half_plus_i_kernel<<<grid2(n, n), 256, 0, st>>>(X, ldx, B, ldb, n);
  QDWHP_LAUNCH_CHECK();
}
void diagonal(const double* A, int64_t lda, int64_t n, double* d, hipStream_t st) {
  diag_kernel<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(A, lda, n, d);
  QDWHP_LAUNCH_CHECK();
}
void upper_copy(const double* A, int64_t lda, double* R, int64_t ldr, int64_t n, hipStream_t st) {
  upper_copy_kernel<<<grid2(n, n), 256, 0, st>>>(A, lda, R, ldr, n);
  QDWHP_LAUNCH_CHECK();
}
void sign_normalize(double* V, int64_t ldv, int64_t rows, int64_t k, double* U, int64_t ldu,
                    int64_t urows, hipStream_t st) {
  if (k <= 0) return;
  sign_kernel<<<(unsigned)k, 256, 0, st>>>(V, ldv, rows, U, ldu, urows);
  QDWHP_LAUNCH_CHECK();
}
void scale_vec(const double* x, double* y, int64_t n, double a, hipStream_t st) {
  scale_vec_kernel<<<(unsigned)cdiv(n, 256), 256, 0, st>>>(x, y, n, a);
  QDWHP_LAUNCH_CHECK();
}
void nonfinite(const double* A, int64_t lda, int64_t m, int64_t n, int* flag, hipStream_t st) {
  nonfinite_kernel<<<grid2(m, n), 256, 0, st>>>(A, lda, m, n, flag);
  QDWHP_LAUNCH_CHECK();
}

}  // namespace qdwhp
