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
constexpr int LZ_ROWS = 2048;      // rows per workgroup in the dot/update kernels

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

// part[run][chunk][c] = sum over the chunk's rows of Q_run[r][c] * w_run[r], c < ncol.
__global__ __launch_bounds__(LZ_T) void dots_kernel(const double* Q, int64_t n, int64_t qstride,
                                                    const double* W, int64_t wstride, int ncol,
                                                    double* part, int nchunk, const int* active) {
  __shared__ double red[LZ_T / 64];
  const int run = blockIdx.y, ch = blockIdx.x;
  if (active && !active[run]) return;
  const double* Qr = Q + run * qstride;
  const double* w = W + run * wstride;
  const int64_t r0 = (int64_t)ch * LZ_ROWS;
  const int64_t r1 = (r0 + LZ_ROWS < n) ? r0 + LZ_ROWS : n;
  for (int c = 0; c < ncol; ++c) {
    double acc = 0.0;
    for (int64_t r = r0 + threadIdx.x; r < r1; r += LZ_T) acc += Qr[r + c * n] * w[r];
    const double s = block_sum(acc, red);
    if (threadIdx.x == 0) part[((int64_t)run * nchunk + ch) * 128 + c] = s;
  }
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

// Block-diagonal matrix of the runs' tridiagonals: T (nv*m square).
__global__ void tridiag_kernel(const double* alpha, const double* beta, int nv, int m, double* T) {
  const int N = nv * m;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  const int i = (int)(e % N), j = (int)(e / N);
  double v = 0.0;
  if (i / m == j / m) {
    const int run = i / m, a = i % m, b = j % m;
    if (a == b) v = alpha[run * m + a];
    else if (a == b + 1) v = beta[run * m + b];
    else if (b == a + 1) v = beta[run * m + a];
  }
  T[i + (int64_t)j * N] = v;
}

// For each eigenpair (column c of W) of the block-diagonal T: the run holding
// it, its quadrature weight (first component in that run)^2 and residual
// bound |beta_m y_m|.
__global__ void nodes_kernel(const double* W, int nv, int m, const double* beta, double* weight,
                             double* resid) {
  const int N = nv * m;
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= N) return;
  int best = 0;
  double bm = -1.0;
  for (int run = 0; run < nv; ++run) {
    double s = 0.0;
    for (int a = 0; a < m; ++a) { const double v = W[run * m + a + (int64_t)c * N]; s += v * v; }
    if (s > bm) { bm = s; best = run; }
  }
  const double y0 = W[best * m + (int64_t)c * N];
  const double ym = W[best * m + m - 1 + (int64_t)c * N];
  weight[c] = y0 * y0;
  resid[c] = fabs(beta[best * m + m - 1] * ym);
}

}  // namespace

int64_t lanczos_doubles(int64_t n, int64_t rows_op, int nv, int m) {
  const int64_t N = (int64_t)nv * m;
  const int64_t nchunk = cdiv(n > rows_op ? n : rows_op, LZ_ROWS);
  return n * (int64_t)(m + 1) * nv       // bases
         + 2 * n * nv + rows_op * nv      // w, spare, operator temp
         + 2 * nv * 128 * nchunk          // partials
         + nv * 128 * 2 + 4 * (int64_t)nv * m  // d, alpha/beta
         + N * N * 2 + syev_scratch_doubles(N) + 4 * N + 256;
}

// Runs the Lanczos processes; `op` applies the operator to nv columns.
LanczosResult lanczos(const LanczosOp& op, int64_t n, int nv, int m, uint64_t seed, double* ws,
                      hipStream_t s) {
  const int64_t N = (int64_t)nv * m;
  const int nchunk = (int)cdiv(n, LZ_ROWS);
  double* Q = ws;                 ws += n * (int64_t)(m + 1) * nv;   // run i: Q + i*n*(m+1)
  double* Wv = ws;                ws += n * nv;
  double* G = ws;                 ws += n * nv;
  double* tmp = ws;               ws += op.rows_tmp * nv;
  double* part = ws;              ws += 2 * (int64_t)nv * 128 * cdiv(n > op.rows_tmp ? n : op.rows_tmp, LZ_ROWS);
  double* dvec = ws;              ws += nv * 128 * 2;
  double* alpha = ws;             ws += (int64_t)nv * m;
  double* beta = ws;              ws += (int64_t)nv * m;
  double* nrm = ws;               ws += 2 * (int64_t)nv * m;
  double* T = ws;                 ws += N * N;
  double* Wt = ws;                ws += N * N;
  double* js = ws;                ws += syev_scratch_doubles(N);
  double* theta = ws;             ws += N;
  double* weight = ws;            ws += N;
  double* resid = ws;             ws += N;
  const int64_t qs = n * (m + 1);
  const dim3 gdots((unsigned)nchunk, (unsigned)nv);
  const dim3 grow((unsigned)cdiv(n, LZ_T), (unsigned)nv);

  // start vectors
  for (int i = 0; i < nv; ++i) {
    gaussian_kernel<<<(unsigned)cdiv(cdiv(n, 2), 256), 256, 0, s>>>(G + i * n, n, seed, (uint64_t)i);
    QDWHP_LAUNCH_CHECK();
  }
  dots_kernel<<<gdots, LZ_T, 0, s>>>(G, n, n, G, n, 1, part, nchunk, nullptr);
  QDWHP_LAUNCH_CHECK();
  normalize_kernel<<<grow, LZ_T, 0, s>>>(G, n, Q, qs, n, part, nchunk, nullptr, nullptr);
  QDWHP_LAUNCH_CHECK();

  std::vector<double> h_a((size_t)nv * m), h_b((size_t)nv * m, 0.0), h_nrm(nv);
  std::vector<double> amax(nv, 0.0);
  std::vector<int> h_active(nv);
  int* d_active = (int*)(nrm + nv * (int64_t)m);   // spare room after nrm (nv ints)
  for (int j = 0; j < m; ++j) {
    // w = Op q_j for all runs (columns at stride qs)
    op.apply(Q + (int64_t)j * n, qs, Wv, n, tmp, s);
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
    std::vector<double> h_d((size_t)nv * 128);
    QDWHP_HIP(hipMemcpyAsync(h_d.data(), dvec, sizeof(double) * nv * 128, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipMemcpyAsync(h_nrm.data(), nrm, sizeof(double) * nv, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    bool restart = false;
    for (int i = 0; i < nv; ++i) {
      const double a = h_d[(size_t)i * 128 + j];
      h_a[(size_t)i * m + j] = a;
      amax[i] = std::max(amax[i], std::fabs(a) + (j > 0 ? h_b[(size_t)i * m + j - 1] : 0.0));
      const double b = h_nrm[i];
      h_active[i] = 0;
      if (j == m - 1) { h_b[(size_t)i * m + j] = b; continue; }
      if (b <= 1e-10 * amax[i]) { h_active[i] = 1; restart = true; h_b[(size_t)i * m + j] = 0.0; }
      else h_b[(size_t)i * m + j] = b;
    }
    if (restart && j < m - 1) {
      QDWHP_HIP(hipMemcpyAsync(d_active, h_active.data(), sizeof(int) * nv, hipMemcpyHostToDevice, s));
      for (int i = 0; i < nv; ++i)
        if (h_active[i]) {
          gaussian_kernel<<<(unsigned)cdiv(cdiv(n, 2), 256), 256, 0, s>>>(
              Wv + i * n, n, seed, (uint64_t)(nv + (int64_t)i * m + j));
          QDWHP_LAUNCH_CHECK();
        }
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
  }
  QDWHP_HIP(hipMemcpyAsync(alpha, h_a.data(), sizeof(double) * nv * m, hipMemcpyHostToDevice, s));
  QDWHP_HIP(hipMemcpyAsync(beta, h_b.data(), sizeof(double) * nv * m, hipMemcpyHostToDevice, s));
  tridiag_kernel<<<(unsigned)cdiv(N * N, 256), 256, 0, s>>>(alpha, beta, nv, m, T);
  QDWHP_LAUNCH_CHECK();
  LanczosResult res;
  res.sweeps = syev(T, N, N, theta, Wt, N, js, s);
  nodes_kernel<<<(unsigned)cdiv(N, 256), 256, 0, s>>>(Wt, nv, m, beta, weight, resid);
  QDWHP_LAUNCH_CHECK();
  res.nodes.resize(N); res.weights.resize(N); res.resid.resize(N);
  QDWHP_HIP(hipMemcpyAsync(res.nodes.data(), theta, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(res.weights.data(), weight, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(res.resid.data(), resid, sizeof(double) * N, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  res.alpha = h_a; res.beta = h_b; res.nv = nv; res.m = m; res.n = n;
  return res;
}

}  // namespace qdwhp
