// Memory-bound helpers: fill, strided copy, mirror of the upper triangle.
#include "common.h"

namespace qdwhp {
namespace {

__global__ void fill_kernel(double* X, int64_t m, int64_t n, int64_t ld, double v, double dg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  for (int64_t jj = j; jj < n; jj += gridDim.y)
    if (i < m) X[i + jj * ld] = (i == jj) ? dg : v;
}

__global__ void copy_kernel(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y)
    if (i < m) Y[i + j * ldy] = X[i + j * ldx];
}

// 64x64 tiles, 256 threads: tile (bi, bj) with bi > bj copies the transpose of
// tile (bj, bi); diagonal tiles copy their upper part into their lower part.
__global__ __launch_bounds__(256) void mirror_kernel(double* X, int64_t n, int64_t ld) {
  __shared__ double T[64][65];
  const int64_t bi = blockIdx.x, bj = blockIdx.y;
  if (bi < bj) return;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t r0 = bj * 64, c0 = bi * 64;  // source tile rows r0.., cols c0..
  for (int yy = ty; yy < 64; yy += 4) {
    const int64_t r = r0 + tx, c = c0 + yy;
    T[yy][tx] = (r < n && c < n) ? X[r + c * ld] : 0.0;   // T[c-c0][r-r0]
  }
  __syncthreads();
  // destination: rows c0.., cols r0..   X[c][r] = X[r][c]
  for (int yy = ty; yy < 64; yy += 4) {
    const int64_t dr = c0 + tx, dc = r0 + yy;   // dest row, dest col
    if (dr < n && dc < n && dr > dc) X[dr + dc * ld] = T[tx][yy];
  }
}

}  // namespace

void fill(double* X, int64_t m, int64_t n, int64_t ld, double v, double dg, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((unsigned)cdiv(m, 256), (unsigned)(n < 65535 ? n : 65535));
  fill_kernel<<<grid, 256, 0, s>>>(X, m, n, ld, v, dg);
  QDWHP_LAUNCH_CHECK();
}

void copy(const double* X, int64_t ldx, double* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  dim3 grid((unsigned)cdiv(m, 256), (unsigned)(n < 65535 ? n : 65535));
  copy_kernel<<<grid, 256, 0, s>>>(X, ldx, Y, ldy, m, n);
  QDWHP_LAUNCH_CHECK();
}

void mirror_upper(double* X, int64_t n, int64_t ld, hipStream_t s) {
  if (n <= 1) return;
  const unsigned t = (unsigned)cdiv(n, 64);
  mirror_kernel<<<dim3(t, t), 256, 0, s>>>(X, n, ld);
  QDWHP_LAUNCH_CHECK();
}

namespace {
struct Params { double v[128]; int count; };
__global__ void write_params_kernel(double* dst, Params p) {
  const int i = threadIdx.x;
  if (i < p.count) dst[i] = p.v[i];
}
}  // namespace

void write_params(double* dst, const double* vals, int count, hipStream_t s) {
  if (count <= 0) return;
  if (count > 128) throw HipError{hipErrorInvalidValue};
  Params p;
  for (int i = 0; i < count; ++i) p.v[i] = vals[i];
  p.count = count;
  write_params_kernel<<<1, 128, 0, s>>>(dst, p);
  QDWHP_LAUNCH_CHECK();
}

}  // namespace qdwhp
