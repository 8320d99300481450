// Inverse of a symmetric positive definite matrix through its Cholesky factor.
//
// Used by the Cholesky-based DWH step (Eq. (3)): with Z = I + c X^T X = W^T W,
// the update (X W^{-1}) W^{-T} equals X Z^{-1}, and Z is well conditioned
// (cond(Z) <= 1 + c x_max^2, which the step-kind rule keeps <= kappa_max), so
// the explicit inverse is as accurate as the two triangular solves while
// turning the solve into one GEMM with no serial chain.
//
// The Cholesky-based step uses the inverse factor W^{-1} directly (two
// triangular products, (X W^{-1}) W^{-T}, as written in Eq. (3)); the full
// inverse Z^{-1} = W^{-1} W^{-T} is also available and formed in three passes:
//   1. recursive Cholesky with simultaneous inversion: splitting Z into
//      [Z11 Z12; . Z22] gives W11 = chol(Z11), W12 = W11^{-T} Z12,
//      Z22 <- Z22 - W12^T W12, W22 = chol(Z22) and
//      W^{-1}_{12} = -W11^{-1} W12 W22^{-1}; 64x64 leaves are factored and
//      inverted in LDS by one workgroup;
//   2. Z^{-1} = W^{-1} W^{-T}, upper tiles only, K starting at the tile column;
//   3. mirror the upper triangle.
#include "common.h"

namespace qdwhp {
namespace {

constexpr int NB = 64;

// Factor the bs x bs leaf (bs <= 64) at Z (upper triangle read) and write its
// inverse factor W^{-1} (upper, zeros below) to Wi.  The factor W itself is
// written back to Z's upper triangle.
__global__ __launch_bounds__(256) void chol_inv_leaf(double* Z, int64_t ldz, double* Wi, int64_t ldw,
                                                     int bs, int* flag) {
  __shared__ double S[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double rpiv;
  __shared__ double rd[NB];
  const int t = threadIdx.x;
  for (int e = t; e < NB * NB; e += 256) {
    const int r = e % NB, c = e / NB;
    double v = 0.0;
    if (r < bs && c < bs) v = (r <= c) ? Z[r + (int64_t)c * ldz] : 0.0;
    S[r][c] = v;
    X[r][c] = 0.0;
  }
  __syncthreads();
  for (int j = 0; j < bs; ++j) {
    if (t == 0) {
      double d = S[j][j];
      if (!(d > 0.0) || !isfinite(d)) { *flag = 1; d = 1.0; }
      const double p = sqrt(d);
      S[j][j] = p;
      rpiv = 1.0 / p;
    }
    __syncthreads();
    if (t > j && t < bs) S[j][t] *= rpiv;
    __syncthreads();
    // trailing update without branches, so the 16 independent read-modify-
    // writes of a thread issue together
#pragma unroll
    for (int u = 0; u < NB * NB / 256; ++u) {
      const int e = t + 256 * u, r = e % NB, c = e / NB;
      const double f = (r > j && r <= c && c < bs) ? S[j][r] : 0.0;
      S[r][c] -= f * S[j][c];
    }
    __syncthreads();
  }
  // back substitution W X = I, one column of X per thread (X upper
  // triangular); the diagonal reciprocals are formed once, so the dependent
  // chain of each column has no division
  if (t < bs) rd[t] = 1.0 / S[t][t];
  __syncthreads();
  if (t < bs) {
    const int c = t;
    X[c][c] = rd[c];
    for (int i = c - 1; i >= 0; --i) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;   // independent chains
      int k = i + 1;
      for (; k + 3 <= c; k += 4) {
        a0 += S[i][k] * X[k][c];
        a1 += S[i][k + 1] * X[k + 1][c];
        a2 += S[i][k + 2] * X[k + 2][c];
        a3 += S[i][k + 3] * X[k + 3][c];
      }
      for (; k <= c; ++k) a0 += S[i][k] * X[k][c];
      X[i][c] = -((a0 + a1) + (a2 + a3)) * rd[i];
    }
  }
  __syncthreads();
  for (int e = t; e < bs * bs; e += 256) {
    const int r = e % bs, c = e / bs;
    if (r <= c) Z[r + (int64_t)c * ldz] = S[r][c];
    Wi[r + (int64_t)c * ldw] = (r <= c) ? X[r][c] : 0.0;
  }
}

struct Rec {
  double* Z; int64_t ldz; double* Wi; int64_t ldw; double* T; int* flag; hipStream_t s;

  void run(int64_t o, int64_t m) {
    double* Zo = Z + o + o * ldz;
    double* Wo = Wi + o + o * ldw;
    if (m <= NB) {
      chol_inv_leaf<<<1, 256, 0, s>>>(Zo, ldz, Wo, ldw, (int)m, flag);
      QDWHP_LAUNCH_CHECK();
      return;
    }
    const int64_t nblk = cdiv(m, NB);
    const int64_t n1 = NB * cdiv(nblk, 2), n2 = m - n1;
    run(o, n1);
    double* Z12 = Zo + n1 * ldz;
    double* Z22 = Zo + n1 + n1 * ldz;
    double* W11i = Wo;
    double* W22i = Wo + n1 + n1 * ldw;
    double* W12i = Wo + n1 * ldw;
    // T = W11^{-T} Z12  (A = W11^{-1} upper, transposed: k <= row)
    Gemm g;
    g.M = n1; g.N = n2; g.K = n1; g.alpha = 1.0; g.beta = 0.0;
    g.A = W11i; g.lda = ldw; g.ta = true; g.B = Z12; g.ldb = ldz; g.C = T; g.ldc = n1;
    g.khi = KHI_ROW;
    dgemm(g, s);
    copy(T, n1, Z12, ldz, n1, n2, s);          // Z12 <- W12
    // Z22 <- Z22 - W12^T W12 (upper tiles)
    Gemm h;
    h.M = n2; h.N = n2; h.K = n1; h.alpha = -1.0; h.beta = 1.0;
    h.A = Z12; h.lda = ldz; h.ta = true; h.B = Z12; h.ldb = ldz; h.C = Z22; h.ldc = ldz;
    h.tiles = TILES_UPPER;
    dgemm(h, s);
    run(o + n1, n2);
    // T = W12 W22^{-1}  (B upper: k <= col)
    Gemm u;
    u.M = n1; u.N = n2; u.K = n2; u.A = Z12; u.lda = ldz; u.B = W22i; u.ldb = ldw;
    u.C = T; u.ldc = n1; u.khi = KHI_COL;
    dgemm(u, s);
    // W^{-1}_{12} = -W11^{-1} T  (A upper: k >= row)
    Gemm v;
    v.M = n1; v.N = n2; v.K = n1; v.alpha = -1.0; v.A = W11i; v.lda = ldw; v.B = T; v.ldb = n1;
    v.C = W12i; v.ldc = ldw; v.klo = KLO_ROW;
    dgemm(v, s);
  }
};

}  // namespace

int64_t spd_inverse_doubles(int64_t n) {
  const int64_t n1 = NB * cdiv(cdiv(n, NB), 2);
  return n * n + n1 * (n - n1 > 0 ? n - n1 : 1) + 64;
}

void chol_inverse_factor(double* Z, int64_t n, int64_t ldz, double* work, int* flag, hipStream_t s) {
  if (n <= 0) return;
  double* Wi = work;
  double* T = work + n * n;
  fill(Wi, n, n, n, 0.0, 0.0, s);
  Rec r{Z, ldz, Wi, n, T, flag, s};
  r.run(0, n);
}

void spd_inverse(double* Z, int64_t n, int64_t ldz, double* work, int* flag, hipStream_t s) {
  if (n <= 0) return;
  double* Wi = work;
  chol_inverse_factor(Z, n, ldz, work, flag, s);
  // Z^{-1} = W^{-1} W^{-T}: upper tiles, k >= tile column.
  Gemm g;
  g.M = n; g.N = n; g.K = n; g.A = Wi; g.lda = n; g.B = Wi; g.ldb = n; g.tb = true;
  g.C = Z; g.ldc = ldz; g.tiles = TILES_UPPER; g.klo = KLO_COL;
  dgemm(g, s);
  mirror_upper(Z, n, ldz, s);
}

}  // namespace qdwhp
