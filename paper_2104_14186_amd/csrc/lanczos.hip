// Lanczos runs for the spectrum bounds and the wanted threshold.
//
// Algorithm 1 bounds the spectrum with a few Lanczos steps and Algorithm 2
// scales by a norm estimate.  Here nv independent runs of m steps are carried
// together (the operator is applied to all current vectors with one GEMM);
// each step re-orthogonalises against the run's whole basis twice
// (classical Gram-Schmidt, deterministic two-pass reductions).  The run's
// start vector is the Philox4x32-10 Gaussian stream (Salmon et al., SC'11)
// with the layout documented in lanczos.h; the same stream, drawn at another
// counter, restarts a run whose residual vanishes.
#include "common.h"
#include "lanczos.h"

namespace qdwhp {
namespace {

constexpr int LZ_T = 256;
constexpr int LZ_ROWS = 2048;      // up to this n, one workgroup per run does a whole step
constexpr int LZ_CHUNK = 512;      // rows per workgroup of the partial dot products

__device__ inline void philox_round(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
  c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
}

__device__ inline void philox10(uint32_t c[4], uint64_t seed) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k0, k1);
    if (r < 9) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
  }
}

// out[i] for i < n: Gaussian entry i of stream `stream`.
__global__ void gaussian_kernel(double* out, int64_t n, uint64_t seed, uint64_t stream) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * p >= n) return;
  uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), (uint32_t)stream, 0u};
  philox10(c, seed);
  const double sc = 1.1102230246251565e-16;   // 2^-53
  const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * sc;
  const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) * sc;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  out[2 * p] = rad * cs;
  if (2 * p + 1 < n) out[2 * p + 1] = rad * sn;
}

__device__ inline double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < LZ_T / 64; ++i) s += red[i];
  return s;
}

// out[c] = sum over rows r0 <= r < r1 of Qr[r + c ldq] * w[r] for c < ncol,
// 32 columns per pass: each thread keeps its partial sums in registers, one
// wave reduction per column and one barrier per pass.  The arithmetic order
// equals block_sum applied column by column.  red holds LZ_T/64 x 32 values.
__device__ inline void block_dots(const double* Qr, int64_t ldq, int64_t r0, int64_t r1, const double* w,
                                  int ncol, double* red, double* out) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c0 = 0; c0 < ncol; c0 += 32) {
    double part[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) part[k] = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += LZ_T) {
      const double x = w[r];
#pragma unroll
      for (int k = 0; k < 32; ++k)
        if (c0 + k < ncol) part[k] += Qr[r + (int64_t)(c0 + k) * ldq] * x;
    }
#pragma unroll
    for (int k = 0; k < 32; ++k)
      for (int o = 32; o > 0; o >>= 1) part[k] += __shfl_xor(part[k], o);
    __syncthreads();
    if (lane == 0)
#pragma unroll
      for (int k = 0; k < 32; ++k) red[wv * 32 + k] = part[k];
    __syncthreads();
    if (threadIdx.x < 32 && c0 + (int)threadIdx.x < ncol) {
      double sm = 0.0;
      for (int i = 0; i < LZ_T / 64; ++i) sm += red[i * 32 + threadIdx.x];
      out[c0 + threadIdx.x] = sm;
    }
  }
  __syncthreads();
}

// part[run][chunk][c] = sum over the chunk's rows of Q_run[r][c] * w_run[r], c < ncol.
__global__ __launch_bounds__(LZ_T) void dots_kernel(const double* Q, int64_t n, int64_t qstride,
                                                    const double* W, int64_t wstride, int ncol,
                                                    double* part, int nchunk, const int* active) {
  __shared__ double red[LZ_T / 64 * 32];
  const int run = blockIdx.y, ch = blockIdx.x;
  if (active && !active[run]) return;
  const double* Qr = Q + run * qstride;
  const double* w = W + run * wstride;
  const int64_t r0 = (int64_t)ch * LZ_CHUNK;
  const int64_t r1 = (r0 + LZ_CHUNK < n) ? r0 + LZ_CHUNK : n;
  block_dots(Qr, n, r0, r1, w, ncol, red, part + ((int64_t)run * nchunk + ch) * 128);
}

// w_run <- w_run - Q_run d, with d = sum over chunks of part (fixed order).
// Also stores d[c] (c < ncol) to dout[run][c] when dout != nullptr.
__global__ __launch_bounds__(LZ_T) void sub_kernel(const double* Q, int64_t n, int64_t qstride,
                                                   double* W, int64_t wstride, int ncol,
                                                   const double* part, int nchunk, double* dout,
                                                   const int* active) {
  __shared__ double d[128];
  const int run = blockIdx.y;
  if (active && !active[run]) return;
  for (int c = threadIdx.x; c < ncol; c += LZ_T) {
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[((int64_t)run * nchunk + ch) * 128 + c];
    d[c] = s;
    if (dout && blockIdx.x == 0) dout[run * 128 + c] = s;
  }
  __syncthreads();
  const double* Qr = Q + run * qstride;
  double* w = W + run * wstride;
  const int64_t r = (int64_t)blockIdx.x * LZ_T + threadIdx.x;
  if (r < n) {
    double acc = w[r];
    for (int c = 0; c < ncol; ++c) acc -= Qr[r + c * n] * d[c];
    w[r] = acc;
  }
}

// q_next_run = w_run / ||w_run|| using the squared-norm partials; stores ||w||.
__global__ __launch_bounds__(LZ_T) void normalize_kernel(const double* W, int64_t wstride, double* Qn,
                                                         int64_t qstride, int64_t n, const double* part,
                                                         int nchunk, double* nrm_out, const int* active) {
  const int run = blockIdx.y;
  if (active && !active[run]) return;
  __shared__ double nrm;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int ch = 0; ch < nchunk; ++ch) s += part[((int64_t)run * nchunk + ch) * 128];
    nrm = sqrt(s);
    if (blockIdx.x == 0 && nrm_out) nrm_out[run] = nrm;
  }
  __syncthreads();
  const int64_t r = (int64_t)blockIdx.x * LZ_T + threadIdx.x;
  if (r < n) Qn[r + run * qstride] = (nrm > 0.0) ? W[r + run * wstride] / nrm : 0.0;
}

// Step bookkeeping on the device (no host round trip per step): alpha_j =
// q_j^T w (from the first CGS pass), beta_j = ||w||.  A run whose beta_j falls
// below 1e-10 times its running |T| bound has found an invariant subspace:
// beta_j is set to 0 (the tridiagonal decouples) and the run is flagged for a
// restart with a fresh random vector.  The last step never restarts.
__global__ void step_kernel(const double* dvec, const double* nrm, int nv, int m, int j,
                            double* alpha, double* beta, double* amax, int* active) {
  const int i = threadIdx.x;
  if (i >= nv) return;
  const double a = dvec[i * 128 + j];
  alpha[i * m + j] = a;
  const double am = fmax(amax[i], fabs(a) + (j > 0 ? beta[i * m + j - 1] : 0.0));
  amax[i] = am;
  const double b = nrm[i];
  int act = 0;
  if (j == m - 1) beta[i * m + j] = b;
  else if (b <= 1e-10 * am) { beta[i * m + j] = 0.0; act = 1; }
  else beta[i * m + j] = b;
  active[i] = act;
}

// Gaussian stream for each flagged run (grid.y = run): W_run <- stream nv + run*m + j.
__global__ void restart_gaussian_kernel(double* W, int64_t n, uint64_t seed, int nv, int m, int j,
                                        const int* active) {
  const int run = blockIdx.y;
  if (!active[run]) return;
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * p >= n) return;
  const uint64_t stream = (uint64_t)nv + (uint64_t)run * m + j;
  uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), (uint32_t)stream, 0u};
  philox10(c, seed);
  const double sc = 1.1102230246251565e-16;
  const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * sc;
  const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) * sc;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  double* w = W + run * n;
  w[2 * p] = rad * cs;
  if (2 * p + 1 < n) w[2 * p + 1] = rad * sn;
}

// Gaussian entry r of stream `stream` (the layout of gaussian_kernel).
__device__ inline double gaussian_entry(int64_t r, uint64_t seed, uint64_t stream) {
  const int64_t p = r >> 1;
  uint32_t c[4] = {(uint32_t)p, (uint32_t)((uint64_t)p >> 32), (uint32_t)stream, 0u};
  philox10(c, seed);
  const double sc = 1.1102230246251565e-16;
  const double u1 = ((double)(c[0] >> 5) * 67108864.0 + (double)(c[1] >> 6) + 0.5) * sc;
  const double u2 = ((double)(c[2] >> 5) * 67108864.0 + (double)(c[3] >> 6) + 0.5) * sc;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(6.283185307179586 * u2, &sn, &cs);
  return (r & 1) ? rad * sn : rad * cs;
}

// Two passes of classical Gram-Schmidt of w against q_0..q_j by one
// workgroup (rows r = t + LZ_T i of each thread), the arithmetic of
// dots_kernel / sub_kernel over a single row chunk; d0 (optional) receives
// the first pass's coefficients.
__device__ inline void cgs2_block(const double* Qr, int64_t n, double* w, int ncol, double* d,
                                  double* red, double* d0) {
  for (int pass = 0; pass < 2; ++pass) {
    block_dots(Qr, n, 0, n, w, ncol, red, d);
    if (pass == 0 && d0)
      for (int c = threadIdx.x; c < ncol; c += LZ_T) d0[c] = d[c];
    for (int64_t r = threadIdx.x; r < n; r += LZ_T) {
      double acc = w[r];
      for (int c = 0; c < ncol; ++c) acc -= Qr[r + c * n] * d[c];
      w[r] = acc;
    }
    __syncthreads();
  }
}

// Everything of Lanczos step j after the operator product, for n <= LZ_ROWS,
// in one launch (one workgroup per run): re-orthogonalisation, norm, the
// step bookkeeping of step_kernel, the restart of a run that broke down, and
// q_{j+1}.  The multi-launch sequence, taken above LZ_ROWS, sums its dot
// products over row chunks of LZ_CHUNK; here they come from one chunk.
__global__ __launch_bounds__(LZ_T) void step_fused_kernel(double* Q, int64_t n, int64_t qstride, double* W,
                                                          int nv, int m, int j, uint64_t seed, double* dvec,
                                                          double* alpha, double* beta, double* amax,
                                                          int* active) {
  __shared__ double red[LZ_T / 64 * 32];
  __shared__ double d[128];
  __shared__ double d0[128];
  __shared__ double nrm_s;
  __shared__ int restart_s;
  const int run = blockIdx.x;
  double* Qr = Q + run * qstride;
  double* w = W + run * n;
  (void)dvec;
  cgs2_block(Qr, n, w, j + 1, d, red, d0);
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += LZ_T) acc += w[r] * w[r];
  const double ss = block_sum(acc, red);
  if (threadIdx.x == 0) {
    const double b = sqrt(ss);
    const double a = d0[j];   // first-pass coefficient of q_j
    alpha[run * m + j] = a;
    const double am = fmax(amax[run], fabs(a) + (j > 0 ? beta[run * m + j - 1] : 0.0));
    amax[run] = am;
    int act = 0;
    if (j == m - 1) beta[run * m + j] = b;
    else if (b <= 1e-10 * am) { beta[run * m + j] = 0.0; act = 1; }
    else beta[run * m + j] = b;
    active[run] = act;
    nrm_s = b;
    restart_s = act;
  }
  __syncthreads();
  double nr = nrm_s;
  if (restart_s) {   // fresh random direction, orthogonalised against the basis
    const uint64_t stream = (uint64_t)nv + (uint64_t)run * m + j;
    for (int64_t r = threadIdx.x; r < n; r += LZ_T) w[r] = gaussian_entry(r, seed, stream);
    __syncthreads();
    cgs2_block(Qr, n, w, j + 1, d, red, nullptr);
    double a2 = 0.0;
    for (int64_t r = threadIdx.x; r < n; r += LZ_T) a2 += w[r] * w[r];
    nr = sqrt(block_sum(a2, red));
  }
  double* qn = Qr + (int64_t)(j + 1) * n;
  for (int64_t r = threadIdx.x; r < n; r += LZ_T) qn[r] = (nr > 0.0) ? w[r] / nr : 0.0;
}

// Eigenvalues of each run's m x m tridiagonal (diagonal alpha, off-diagonal
// beta) by the implicit symmetric QR iteration with Wilkinson shift (Golub &
// Van Loan, Matrix Computations, Sec. 8.3), one thread per run.  Only the
// first and last rows of the eigenvector matrix are carried along: the
// Gauss-quadrature weight of node i is (first component)^2 (Golub & Welsch)
// and its Ritz residual is |beta_m| |last component|.
// The serial QR iteration of one run is a chain of dependent reads and
// writes of d, e, z0, zl: with lds set they live in LDS (one padded slice
// per thread), else in the global scratch; the arithmetic is the same.
__global__ void tridiag_eig_kernel(const double* alpha, const double* beta, int nv, int m,
                                   double* scratch, double* theta, double* weight, double* resid,
                                   int* fail, int lds) {
  extern __shared__ double sl[];
  if (threadIdx.x == 0) *fail = 0;
  __syncthreads();
  const int run = blockIdx.x * blockDim.x + threadIdx.x;
  if (run >= nv) return;
  double* d = lds ? sl + (int64_t)threadIdx.x * (4 * m + 1) : scratch + (int64_t)run * 4 * m;
  double* e = d + m;
  double* z0 = e + m;
  double* zl = z0 + m;
  for (int i = 0; i < m; ++i) {
    d[i] = alpha[run * m + i];
    e[i] = (i + 1 < m) ? beta[run * m + i] : 0.0;
    z0[i] = (i == 0) ? 1.0 : 0.0;
    zl[i] = (i == m - 1) ? 1.0 : 0.0;
  }
  const double u = 1.1102230246251565e-16;
  int hi = m - 1, steps = 0;
  while (hi > 0) {
    for (int i = 0; i < hi; ++i)
      if (fabs(e[i]) <= u * (fabs(d[i]) + fabs(d[i + 1]))) e[i] = 0.0;
    if (e[hi - 1] == 0.0) { --hi; continue; }
    int lo = hi - 1;
    while (lo > 0 && e[lo - 1] != 0.0) --lo;
    if (++steps > 40 * m) { *fail = 1; break; }
    // Wilkinson shift from the trailing 2x2 of the unreduced block [lo, hi]
    const double tb = e[hi - 1];
    const double del = 0.5 * (d[hi - 1] - d[hi]);
    const double den = del + (del >= 0.0 ? 1.0 : -1.0) * hypot(del, tb);
    const double mu = d[hi] - tb * tb / den;
    double x = d[lo] - mu, z = e[lo];
    for (int k = lo; k < hi; ++k) {
      // rotation in the (k, k+1) plane that zeroes z against x
      const double r = hypot(x, z);
      double c = 1.0, s = 0.0;
      if (r > 0.0) { c = x / r; s = z / r; }
      if (k > lo) e[k - 1] = r;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk + 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk - 2.0 * c * s * ek + c * c * dk1;
      e[k] = (c * c - s * s) * ek + c * s * (dk1 - dk);
      double bulge = 0.0;
      if (k + 1 < hi) { bulge = s * e[k + 1]; e[k + 1] = c * e[k + 1]; }
      const double a0 = z0[k], a1 = z0[k + 1];
      z0[k] = c * a0 + s * a1; z0[k + 1] = -s * a0 + c * a1;
      const double b0 = zl[k], b1 = zl[k + 1];
      zl[k] = c * b0 + s * b1; zl[k + 1] = -s * b0 + c * b1;
      x = e[k]; z = bulge;
    }
  }
  const double bm = fabs(beta[run * m + m - 1]);
  for (int i = 0; i < m; ++i) {
    theta[run * m + i] = d[i];
    weight[run * m + i] = z0[i] * z0[i];
    resid[run * m + i] = bm * fabs(zl[i]);
  }
}

}  // namespace

int64_t lanczos_doubles(int64_t n, int64_t rows_op, int nv, int m) {
  const int64_t N = (int64_t)nv * m;
  const int64_t nchunk = cdiv(n > rows_op ? n : rows_op, LZ_CHUNK);
  return n * (int64_t)(m + 1) * nv       // bases
         + 2 * n * nv + rows_op * nv      // w, spare, operator temp
         + 2 * nv * 128 * nchunk          // partials
         + nv * 128 * 2 + 4 * (int64_t)nv * m  // d, alpha/beta, norms
         + 4 * N + 3 * N + 2 * nv + 256;       // tridiagonal scratch, nodes, amax/flags
}

void gaussian_fill(double* out, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s) {
  if (count <= 0) return;
  gaussian_kernel<<<(unsigned)cdiv(cdiv(count, 2), 256), 256, 0, s>>>(out, count, seed, stream);
  QDWHP_LAUNCH_CHECK();
}

// Runs the Lanczos processes; `op` applies the operator to nv columns.
LanczosResult lanczos(const LanczosOp& op, int64_t n, int nv, int m, uint64_t seed, double* ws,
                      hipStream_t s) {
  const int64_t N = (int64_t)nv * m;
  const int nchunk = (int)cdiv(n, LZ_CHUNK);
  const bool fused = n <= LZ_ROWS;
  double* Q = ws;                 ws += n * (int64_t)(m + 1) * nv;   // run i: Q + i*n*(m+1)
  double* Wv = ws;                ws += n * nv;
  double* G = ws;                 ws += n * nv;
  double* tmp = ws;               ws += op.rows_tmp * nv;
  double* part = ws;              ws += 2 * (int64_t)nv * 128 * cdiv(n > op.rows_tmp ? n : op.rows_tmp, LZ_CHUNK);
  double* dvec = ws;              ws += nv * 128 * 2;
  double* alpha = ws;             ws += (int64_t)nv * m;
  double* beta = ws;              ws += (int64_t)nv * m;
  double* nrm = ws;               ws += 2 * (int64_t)nv * m;
  double* tscr = ws;              ws += 4 * N;
  double* theta = ws;             ws += N;
  double* weight = ws;            ws += N;
  double* resid = ws;             ws += N;
  double* amax = ws;              ws += nv;
  int* d_active = (int*)ws;       ws += nv;   // nv ints, then the failure flag
  const int64_t qs = n * (m + 1);
  const dim3 gdots((unsigned)nchunk, (unsigned)nv);
  const dim3 grow((unsigned)cdiv(n, LZ_T), (unsigned)nv);
  const dim3 ggauss((unsigned)cdiv(cdiv(n, 2), 256), (unsigned)nv);

  // start vectors
  for (int i = 0; i < nv; ++i) {
    gaussian_kernel<<<(unsigned)cdiv(cdiv(n, 2), 256), 256, 0, s>>>(G + i * n, n, seed, (uint64_t)i);
    QDWHP_LAUNCH_CHECK();
  }
  fill(amax, nv, 1, nv, 0.0, 0.0, s);
  fill(beta, nv, m, nv, 0.0, 0.0, s);
  dots_kernel<<<gdots, LZ_T, 0, s>>>(G, n, n, G, n, 1, part, nchunk, nullptr);
  QDWHP_LAUNCH_CHECK();
  normalize_kernel<<<grow, LZ_T, 0, s>>>(G, n, Q, qs, n, part, nchunk, nullptr, nullptr);
  QDWHP_LAUNCH_CHECK();

  for (int j = 0; j < m; ++j) {
    // w = Op q_j for all runs (columns at stride qs)
    op.apply(Q + (int64_t)j * n, qs, Wv, n, tmp, s);
    if (fused) {   // one workgroup per run covers the vector: one launch for the rest
      step_fused_kernel<<<nv, LZ_T, 0, s>>>(Q, n, qs, Wv, nv, m, j, seed, dvec, alpha, beta, amax, d_active);
      QDWHP_LAUNCH_CHECK();
      continue;
    }
    // two passes of classical Gram-Schmidt against q_0..q_j
    for (int pass = 0; pass < 2; ++pass) {
      dots_kernel<<<gdots, LZ_T, 0, s>>>(Q, n, qs, Wv, n, j + 1, part, nchunk, nullptr);
      QDWHP_LAUNCH_CHECK();
      sub_kernel<<<grow, LZ_T, 0, s>>>(Q, n, qs, Wv, n, j + 1, part, nchunk,
                                       pass == 0 ? dvec : nullptr, nullptr);
      QDWHP_LAUNCH_CHECK();
    }
    dots_kernel<<<gdots, LZ_T, 0, s>>>(Wv, n, n, Wv, n, 1, part, nchunk, nullptr);
    QDWHP_LAUNCH_CHECK();
    normalize_kernel<<<grow, LZ_T, 0, s>>>(Wv, n, Q + (int64_t)(j + 1) * n, qs, n, part, nchunk, nrm, nullptr);
    QDWHP_LAUNCH_CHECK();
    step_kernel<<<1, 64, 0, s>>>(dvec, nrm, nv, m, j, alpha, beta, amax, d_active);
    QDWHP_LAUNCH_CHECK();
    if (j == m - 1) break;
    // restart of the flagged runs (the kernels return at once for the others)
    restart_gaussian_kernel<<<ggauss, 256, 0, s>>>(Wv, n, seed, nv, m, j, d_active);
    QDWHP_LAUNCH_CHECK();
    for (int pass = 0; pass < 2; ++pass) {
      dots_kernel<<<gdots, LZ_T, 0, s>>>(Q, n, qs, Wv, n, j + 1, part, nchunk, d_active);
      QDWHP_LAUNCH_CHECK();
      sub_kernel<<<grow, LZ_T, 0, s>>>(Q, n, qs, Wv, n, j + 1, part, nchunk, nullptr, d_active);
      QDWHP_LAUNCH_CHECK();
    }
    dots_kernel<<<gdots, LZ_T, 0, s>>>(Wv, n, n, Wv, n, 1, part, nchunk, d_active);
    QDWHP_LAUNCH_CHECK();
    normalize_kernel<<<grow, LZ_T, 0, s>>>(Wv, n, Q + (int64_t)(j + 1) * n, qs, n, part, nchunk,
                                           nullptr, d_active);
    QDWHP_LAUNCH_CHECK();
  }
  int* d_fail = d_active + nv;
  // nv <= 64 runs, one thread each; LDS while their slices fit in 64 KiB
  const size_t tlds = (size_t)nv * (4 * (size_t)m + 1) * sizeof(double);
  const int use_lds = tlds <= 65536 ? 1 : 0;
  tridiag_eig_kernel<<<1, 64, use_lds ? tlds : 0, s>>>(alpha, beta, nv, m, tscr, theta, weight, resid, d_fail,
                                                       use_lds);
  QDWHP_LAUNCH_CHECK();
  std::vector<double> h_a((size_t)N), h_b((size_t)N), th(N), wt(N), rs(N);
  int h_fail = 0;
  QDWHP_HIP(hipMemcpyAsync(h_a.data(), alpha, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(h_b.data(), beta, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(th.data(), theta, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(wt.data(), weight, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(rs.data(), resid, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(&h_fail, d_fail, sizeof(int), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  // nodes in descending order (ties by run-major index)
  std::vector<int64_t> idx(N);
  for (int64_t i = 0; i < N; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int64_t x, int64_t y) { return th[x] > th[y]; });
  LanczosResult res;
  res.sweeps = h_fail ? -1 : 0;
  res.nodes.resize(N); res.weights.resize(N); res.resid.resize(N);
  for (int64_t i = 0; i < N; ++i) {
    res.nodes[i] = th[idx[i]]; res.weights[i] = wt[idx[i]]; res.resid[i] = rs[idx[i]];
  }
  res.alpha = h_a; res.beta = h_b; res.nv = nv; res.m = m; res.n = n;
  return res;
}

}  // namespace qdwhp
