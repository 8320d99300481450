// QDWHpartial-EIG for complex Hermitian matrices (Sec. 4 treats real
// symmetric matrices; the Hermitian case carries over with conjugate
// transposes).
//
// The solve runs on the real symmetric embedding
//     M = [ Re A  -Im A ]
//         [ Im A   Re A ]   (2n x 2n),
// whose spectrum is that of A with every eigenvalue twice: A (x + i y) =
// lambda (x + i y) exactly when M [x; y] = lambda [x; y], and then also
// M [-y; x] = lambda [-y; x].  The map [x; y] -> x + i y takes M's products,
// Cholesky-based and QR-based steps to those of A, so every iteration, the
// projector QR and the Rayleigh-Ritz step are the real path's kernels on M
// (twice the flops of the same steps in complex arithmetic; the products
// themselves cost the same, the factorizations twice).  The k wanted complex
// pairs are the 2k wanted real pairs of M taken back: the real Ritz vectors
// of one complex eigenvalue span {u, J u}, both of which map to multiples of
// the same complex vector, so each cluster of 2p real Ritz values within
// 1e-12 ||A|| of each other gives p complex vectors by Gram-Schmidt in
// complex arithmetic (twice, modified) over its real Ritz vectors in order,
// keeping those with more than half their norm left.  A real Ritz vector's
// residual carries over unchanged to its complex image.  Images of real
// Ritz vectors of different but close eigenvalues are orthogonal only up to
// the real solver's mixing of those eigenvectors (about u ||A|| / gap), so
// the k vectors then take two symmetric (Loewdin) orthonormalization steps
// V <- V (I - E/2 + 3 E^2/8), E = V^H V - I, in complex arithmetic on
// planar real and imaginary parts (real GEMMs); E couples only vectors of
// close eigenvalues, so the residuals move by about |E_ij| |lambda_i -
// lambda_j| ~ u ||A||.  Every returned vector is scaled by a unit complex
// number that makes its largest-magnitude entry real and positive (lowest
// index on ties).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"

namespace qdwhp {
namespace {

// M (2n x 2n, ld 2n) from the interleaved complex A (n x n, ld lda complex).
__global__ void embed_kernel(const double* __restrict__ A, int64_t lda, int64_t n, double* __restrict__ M) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t n2 = 2 * n;
  for (int64_t j = blockIdx.y; j < n; j += gridDim.y) {
    if (i >= n) continue;
    const double re = A[2 * (i + j * lda)], im = A[2 * (i + j * lda) + 1];
    M[i + j * n2] = re;
    M[(n + i) + (n + j) * n2] = re;
    M[(n + i) + j * n2] = im;
    M[i + (n + j) * n2] = -im;
  }
}

struct Cluster { int start, size, out, p; };

constexpr int PT = 256;

// Block sums of two values (all threads get the totals).
__device__ void block_sum2(double& a, double& b, double* sh) {
  const int t = threadIdx.x;
  sh[t] = a;
  sh[PT + t] = b;
  __syncthreads();
  for (int s = PT / 2; s > 0; s >>= 1) {
    if (t < s) { sh[t] += sh[t + s]; sh[PT + t] += sh[PT + t + s]; }
    __syncthreads();
  }
  a = sh[0];
  b = sh[PT];
  __syncthreads();
}

// One workgroup per cluster: complex Gram-Schmidt over the cluster's real
// Ritz vectors (columns of V2, 2n x ., ld 2n), writing the kept ones to V
// (interleaved complex, ld ldv) and their Ritz values to w.
__global__ __launch_bounds__(PT) void pair_select_kernel(const double* __restrict__ V2, int64_t n,
                                                         const double* __restrict__ w2, const Cluster* cl,
                                                         double* __restrict__ V, int64_t ldv, double* __restrict__ w,
                                                         int* flag) {
  // V: interleaved complex columns (used here as scratch for the selection)
  __shared__ double sh[2 * PT];
  const Cluster c = cl[blockIdx.x];
  const int t = threadIdx.x;
  int kept = 0;
  for (int jj = 0; jj < c.size && kept < c.p; ++jj) {
    const int64_t j = c.start + jj;
    double* v = V + 2 * (int64_t)(c.out + kept) * ldv;
    for (int64_t r = t; r < n; r += PT) {
      v[2 * r] = V2[r + j * 2 * n];
      v[2 * r + 1] = V2[n + r + j * 2 * n];
    }
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < kept; ++q) {
        const double* s = V + 2 * (int64_t)(c.out + q) * ldv;
        // <s, v> = sum conj(s) v
        double dr = 0.0, di = 0.0;
        for (int64_t r = t; r < n; r += PT) {
          const double sr = s[2 * r], si = s[2 * r + 1], vr = v[2 * r], vi = v[2 * r + 1];
          dr += sr * vr + si * vi;
          di += sr * vi - si * vr;
        }
        block_sum2(dr, di, sh);
        for (int64_t r = t; r < n; r += PT) {
          const double sr = s[2 * r], si = s[2 * r + 1];
          v[2 * r] -= dr * sr - di * si;
          v[2 * r + 1] -= dr * si + di * sr;
        }
        __syncthreads();
      }
    }
    double nr = 0.0, dummy = 0.0;
    for (int64_t r = t; r < n; r += PT) nr += v[2 * r] * v[2 * r] + v[2 * r + 1] * v[2 * r + 1];
    block_sum2(nr, dummy, sh);
    const double nrm = sqrt(nr);
    if (nrm > 0.5) {
      const double inv = 1.0 / nrm;
      for (int64_t r = t; r < n; r += PT) { v[2 * r] *= inv; v[2 * r + 1] *= inv; }
      if (t == 0) w[c.out + kept] = w2[j];
      ++kept;
    }
    __syncthreads();
  }
  if (t == 0 && kept < c.p) *flag = 1;
}

// Planar (Pr, Pi: n x k, ld n) <-> interleaved complex (V: n x k, ld ldv).
__global__ void to_planar_kernel(const double* __restrict__ V, int64_t ldv, int64_t n, int64_t k,
                                 double* __restrict__ Pr, double* __restrict__ Pi) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    if (i >= n) continue;
    Pr[i + j * n] = V[2 * (i + j * ldv)];
    Pi[i + j * n] = V[2 * (i + j * ldv) + 1];
  }
}
__global__ void to_interleaved_kernel(const double* __restrict__ Pr, const double* __restrict__ Pi, int64_t n,
                                      int64_t k, double* __restrict__ V, int64_t ldv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < k; j += gridDim.y) {
    if (i >= n) continue;
    V[2 * (i + j * ldv)] = Pr[i + j * n];
    V[2 * (i + j * ldv) + 1] = Pi[i + j * n];
  }
}

// One symmetric orthonormalization step on planar V = Vr + i Vi (n x k):
// E = V^H V - I = Gr + i Gi, T = I - E/2 + 3 E^2 / 8 = Tr + i Ti,
// V <- V T into (Wr, Wi).
void loewdin_step(const double* Vr, const double* Vi, int64_t n, int64_t k, double* Gr, double* Gi,
                  double* Tr, double* Ti, double* Wr, double* Wi, hipStream_t s) {
  auto gemm = [&](bool ta, const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                  int64_t M, int64_t N, int64_t K, double alpha, double beta, const double* Cin, double diag) {
    Gemm g;
    g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.beta = beta; g.ta = ta;
    g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.diag = diag;
    if (Cin) { g.Cin = Cin; g.ldcin = ldc; }
    dgemm(g, s);
  };
  gemm(true, Vr, n, Vr, n, Gr, k, k, k, n, 1.0, 0.0, nullptr, -1.0);      // Gr = Vr^T Vr - I
  gemm(true, Vi, n, Vi, n, Gr, k, k, k, n, 1.0, 1.0, Gr, 0.0);          //    + Vi^T Vi
  gemm(true, Vr, n, Vi, n, Gi, k, k, k, n, 1.0, 0.0, nullptr, 0.0);     // Gi = Vr^T Vi
  gemm(true, Vi, n, Vr, n, Gi, k, k, k, n, -1.0, 1.0, Gi, 0.0);         //    - Vi^T Vr
  gemm(false, Gr, k, Gr, k, Tr, k, k, k, k, 0.375, -0.5, Gr, 1.0);      // Tr = I - Gr/2 + 3/8 Gr Gr
  gemm(false, Gi, k, Gi, k, Tr, k, k, k, k, -0.375, 1.0, Tr, 0.0);      //      - 3/8 Gi Gi
  gemm(false, Gr, k, Gi, k, Ti, k, k, k, k, 0.375, -0.5, Gi, 0.0);      // Ti = -Gi/2 + 3/8 Gr Gi
  gemm(false, Gi, k, Gr, k, Ti, k, k, k, k, 0.375, 1.0, Ti, 0.0);       //      + 3/8 Gi Gr
  gemm(false, Vr, n, Tr, k, Wr, n, n, k, k, 1.0, 0.0, nullptr, 0.0);    // Wr = Vr Tr - Vi Ti
  gemm(false, Vi, n, Ti, k, Wr, n, n, k, k, -1.0, 1.0, Wr, 0.0);
  gemm(false, Vr, n, Ti, k, Wi, n, n, k, k, 1.0, 0.0, nullptr, 0.0);    // Wi = Vr Ti + Vi Tr
  gemm(false, Vi, n, Tr, k, Wi, n, n, k, k, 1.0, 1.0, Wi, 0.0);
}

// Column j of V scaled by conj(v_m) / |v_m|, v_m its largest-magnitude entry
// (lowest index on ties).
__global__ __launch_bounds__(PT) void phase_kernel(double* __restrict__ V, int64_t n, int64_t ldv) {
  __shared__ double sm[PT];
  __shared__ int64_t si[PT];
  const int t = threadIdx.x;
  double* v = V + 2 * (int64_t)blockIdx.x * ldv;
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t r = t; r < n; r += PT) {
    const double a = v[2 * r] * v[2 * r] + v[2 * r + 1] * v[2 * r + 1];
    if (a > best) { best = a; bi = r; }
  }
  sm[t] = best;
  si[t] = bi;
  __syncthreads();
  for (int s = PT / 2; s > 0; s >>= 1) {
    if (t < s && (sm[t + s] > sm[t] || (sm[t + s] == sm[t] && si[t + s] < si[t]))) {
      sm[t] = sm[t + s];
      si[t] = si[t + s];
    }
    __syncthreads();
  }
  const int64_t m = si[0];
  const double pr = v[2 * m], pi = v[2 * m + 1];
  const double a = sqrt(pr * pr + pi * pi);
  __syncthreads();
  if (!(a > 0.0)) return;
  const double cr = pr / a, ci = -pi / a;   // conj(v_m) / |v_m|
  for (int64_t r = t; r < n; r += PT) {
    const double xr = v[2 * r], xi = v[2 * r + 1];
    v[2 * r] = xr * cr - xi * ci;
    v[2 * r + 1] = xr * ci + xi * cr;
  }
}

int64_t wanted(int64_t n, double fraction) { return qdwhp_eig_count(n, fraction); }

// Workspace: M, w2, V2, the cluster table and a flag, then the real solve's.
struct HLayout {
  size_t m_off, w2_off, v2_off, cl_off, flag_off, pl_off, g_off, real_off, total;
};
HLayout layout(int64_t n, double fraction, const qdwhp_opts* opts) {
  const int64_t k = wanted(n, fraction);
  HLayout L;
  size_t off = 0;
  auto take = [&](size_t bytes) { const size_t o = off; off += (bytes + 255) / 256 * 256; return o; };
  L.m_off = take(sizeof(double) * 4 * n * n);
  L.w2_off = take(sizeof(double) * 2 * k);
  L.v2_off = take(sizeof(double) * 4 * n * k);
  L.cl_off = take(sizeof(Cluster) * 2 * k);
  L.flag_off = take(sizeof(int) * 64);
  L.pl_off = take(sizeof(double) * 4 * n * k);     // Vr, Vi, Wr, Wi (n x k each)
  L.g_off = take(sizeof(double) * 4 * k * k);      // Gr, Gi, Tr, Ti (k x k each)
  L.real_off = off;
  L.total = off + qdwhp_eig_workspace(2 * n, (double)k / (double)n, opts);
  return L;
}

}  // namespace
}  // namespace qdwhp

using namespace qdwhp;

extern "C" size_t qdwhp_heig_workspace(int64_t n, double fraction, const qdwhp_opts* opts) {
  if (n < 1 || !(fraction > 0.0) || fraction > 1.0) return 0;
  return layout(n, fraction, opts).total;
}

extern "C" int qdwhp_heig(const double* A, int64_t n, int64_t lda, double fraction, int which, double* w,
                          double* V, int64_t ldv, void* work, size_t lwork, const qdwhp_opts* opts,
                          void* stream, qdwhp_info* info) {
  qdwhp_info dummy;
  if (!info) info = &dummy;
  std::memset(info, 0, sizeof(*info));
  int bad = 0;
  if (!A) bad = -1;
  else if (n < 1) bad = -2;
  else if (lda < n) bad = -3;
  else if (!(fraction > 0.0) || fraction > 1.0) bad = -4;
  else if (which != QDWHP_LARGEST && which != QDWHP_SMALLEST) bad = -5;
  else if (!w) bad = -6;
  else if (!V) bad = -7;
  else if (ldv < n) bad = -8;
  else if (!work) bad = -9;
  if (bad) { info->status = bad; return bad; }
  const HLayout L = layout(n, fraction, opts);
  if (lwork < L.total) { info->status = QDWHP_ERR_WORKSPACE; return QDWHP_ERR_WORKSPACE; }
  const int64_t k = wanted(n, fraction);
  hipStream_t s = (hipStream_t)stream;
  char* base = (char*)work;
  double* M = (double*)(base + L.m_off);
  double* w2 = (double*)(base + L.w2_off);
  double* V2 = (double*)(base + L.v2_off);
  Cluster* cl = (Cluster*)(base + L.cl_off);
  int* flag = (int*)(base + L.flag_off);
  try {
    const int64_t n2 = 2 * n;
    embed_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)std::min<int64_t>(n, 65535)), 256, 0, s>>>(A, lda, n, M);
    QDWHP_LAUNCH_CHECK();
    const int st = eig_impl(M, n2, n2, (double)k / (double)n, which, w2, V2, n2, base + L.real_off,
                            L.total - L.real_off, opts, stream, info, nullptr);
    info->k = k;
    if (st != QDWHP_OK) return st;
    // clusters of the 2k real Ritz values (in the returned order)
    std::vector<double> h(2 * k);
    QDWHP_HIP(hipMemcpyAsync(h.data(), w2, sizeof(double) * 2 * k, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    const double scale = std::max({std::fabs(info->lmax), std::fabs(info->lmin), std::fabs(h[0]),
                                   std::fabs(h[2 * k - 1]), 1e-300});
    std::vector<Cluster> cs;
    int64_t j = 0;
    while (j < 2 * k) {
      int64_t e = j + 1;
      while (e < 2 * k && std::fabs(h[e] - h[e - 1]) <= 1e-12 * scale) ++e;
      cs.push_back(Cluster{(int)j, (int)(e - j), 0, (int)((e - j) / 2)});
      j = e;
    }
    int64_t total = 0;
    for (const auto& c : cs) total += c.p;
    for (auto& c : cs)                      // odd clusters (a cut through a pair) take the remainder
      if (total < k && (c.size & 1)) { ++c.p; ++total; }
    if (total != k) { info->status = QDWHP_ERR_NO_SUBSPACE; return QDWHP_ERR_NO_SUBSPACE; }
    int64_t out = 0;
    for (auto& c : cs) { c.out = (int)out; out += c.p; }
    QDWHP_HIP(hipMemcpyAsync(cl, cs.data(), sizeof(Cluster) * cs.size(), hipMemcpyHostToDevice, s));
    QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    pair_select_kernel<<<(unsigned)cs.size(), PT, 0, s>>>(V2, n, w2, cl, V, ldv, w, flag);
    QDWHP_LAUNCH_CHECK();
    // two symmetric orthonormalization steps on planar copies, then back
    double* P = (double*)(base + L.pl_off);
    double *Vr = P, *Vi = P + n * k, *Wr = P + 2 * n * k, *Wi = P + 3 * n * k;
    double* G = (double*)(base + L.g_off);
    const dim3 g2((unsigned)cdiv(n, 256), (unsigned)std::min<int64_t>(k, 65535));
    to_planar_kernel<<<g2, 256, 0, s>>>(V, ldv, n, k, Vr, Vi);
    QDWHP_LAUNCH_CHECK();
    for (int it = 0; it < 2; ++it) {
      loewdin_step(Vr, Vi, n, k, G, G + k * k, G + 2 * k * k, G + 3 * k * k, Wr, Wi, s);
      std::swap(Vr, Wr);
      std::swap(Vi, Wi);
    }
    to_interleaved_kernel<<<g2, 256, 0, s>>>(Vr, Vi, n, k, V, ldv);
    QDWHP_LAUNCH_CHECK();
    phase_kernel<<<(unsigned)k, PT, 0, s>>>(V, n, ldv);
    QDWHP_LAUNCH_CHECK();
    int hf = 0;
    QDWHP_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (hf) { info->status = QDWHP_ERR_NO_SUBSPACE; return QDWHP_ERR_NO_SUBSPACE; }
  } catch (const HipError&) {
    info->status = QDWHP_ERR_HIP;
    return QDWHP_ERR_HIP;
  }
  info->status = QDWHP_OK;
  return QDWHP_OK;
}
