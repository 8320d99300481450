// Householder QR without pivoting (geqrf layout) and explicit Q columns.
//
// Used for the stacked matrix [sqrt(c) X; I] of the QR-based step (Eq. (2))
// and for the spectral projector whose R diagonal reveals the subspace size
// (Sec. 4.1, Theorem 1 and "Choosing the subspace size").
//
// Blocked right-looking factorization with panels of QB = 128 columns:
//  * panel: factored in sub-panels of QI = 32 columns, each finished
//    sub-panel applied to the rest of the panel as a blocked update (the
//    same T / three-GEMM form as the trailing update), so the per-column
//    launches sweep at most 32 columns;
//  * sub-panel by Cholesky QR with Householder reconstruction (default when
//    the stream is not being captured): the sub-panel P (h x 32) is
//    orthonormalised by two Cholesky-QR passes (P = Q R, R = R2 R1), and the
//    Householder form of the same factorization is rebuilt from Q: an LU
//    factorization without pivoting of S - Q1 (Q1 the top 32 x 32 block of
//    Q, S = diag(+-1) chosen at each elimination step so that the pivot has
//    magnitude 1 + |.|) gives the unit-lower reflector block Y1 = L and U;
//    then Y2 = -Q2 U^{-1}, T = U S Y1^{-T}, tau = diag(T) and R_H = S R,
//    which is exactly the LAPACK-convention Householder QR of P (Ballard,
//    Demmel, Grigori, Jacquelin, Knight, Nguyen, "Reconstructing Householder
//    vectors from tall-skinny QR", 2015).  Five launches per sub-panel
//    instead of one per column.  A sub-panel whose first-pass pivots show a
//    column within 1e-5 of the span of the earlier ones (relative), or whose
//    first pass leaves Q^T Q more than 0.1 from I, sets a flag; the host
//    checks it after each panel, restores the panel from a copy taken
//    before it and factors it by the column steps below (the panel holding
//    the first tiny |R_ii| of the projector QR takes this path).  The
//    second pass and the reconstruction start from the first pass's Q as
//    stored (Q = Q_1 R2^{-1}, Y2 = -Q2 U^{-1} with Q_1 = P R1^{-1} rounded
//    once): folding R1^{-1} into a single product with P would carry
//    rounding of order u cond(P) into Q;
//  * column step: one launch per column over the whole grid.  Launch j forms
//    reflector j from column statistics reduced from the previous launch
//    (norm of the column below the pivot, its dot products with the other
//    panel columns, and the pivot row), applies it to this workgroup's rows,
//    and accumulates the statistics of column j+1 -- so a column costs one
//    pass over the panel and one launch, with no atomics (partials are
//    summed in a fixed order, results are bitwise reproducible);
//  * T factor of the compact WY form I - V T V^T from G = V^T V
//    (split-K GEMM) and the forward recurrence T(0:j,j) = -tau_j T(0:j,0:j) G(0:j,j);
//  * trailing update C <- (I - V T^T V^T) C as three GEMMs with V read in
//    place from below the diagonal (unit-lower operand mask).
#include <algorithm>
#include <memory>

#include "common.h"
#include "qdwhp.h"
#include "qr.h"

namespace qdwhp {
namespace {

constexpr int CH = 32;          // columns per register chunk
constexpr int RPT_MAX = 8;      // rows per thread
constexpr int QT = 256;         // threads per workgroup
constexpr int NWG_MAX = 64;     // workgroups per column launch
constexpr int QI = 32;          // sub-panel width of the column launches

struct Panel {
  double* P; int64_t ld; int64_t h; int w;
  double* tau;
  double* part;     // [2][NWG_MAX][QB] partial statistics (double-buffered by launch parity)
  double* piv;      // [2][QB] pivot-row values
  int nwg; int rpt;
};

// Launch j (j = -1 gathers the statistics of column 0 only):
//  1. sums the previous launch's partials (fixed order) into the statistics of
//     column j: t_c = sum_{r > j} P[r][j] P[r][c], c >= j, and reads the pivot
//     row P[j][c] saved by the previous launch;
//  2. forms reflector j (LAPACK convention: beta = -sign(x0) ||x||,
//     tau = (beta - x0)/beta, v = x/(x0 - beta) below the pivot, v_j = 1);
//  3. applies H_j to this workgroup's rows of columns j+1.. and stores v;
//  4. accumulates the statistics of column j+1 from the updated values and
//     saves the new pivot row.
// All loads of a reduction are issued before they are consumed (independent
// chains), since every column pays these latencies on the critical path.
__global__ __launch_bounds__(QT) void qr_col_kernel(Panel a, int j) {
  __shared__ double sh_s[QB];
  __shared__ double sh_w[QB];
  __shared__ double sh_half[2][QB];
  __shared__ double sh_acc[QT][CH + 1];
  __shared__ double sh_seg[QT / CH][CH];
  const int t = threadIdx.x, g = blockIdx.x;
  const int w = a.w;
  const int64_t ld = a.ld;
  double* P = a.P;
  const double* part_in = a.part + (int64_t)((j + 2) & 1) * NWG_MAX * QB;
  double* part_out = a.part + (int64_t)((j + 1) & 1) * NWG_MAX * QB;
  const double* piv_in = a.piv + ((j + 2) & 1) * QB;
  double* piv_out = a.piv + ((j + 1) & 1) * QB;

  // One row per thread (panels up to QT * NWG_MAX rows): the row's values in
  // columns j and j+1 .. j+CH are loaded first, so their latency overlaps the
  // reduction of the statistics that define reflector j.
  const bool one_row = (a.rpt == 1);
  const int64_t r1 = (int64_t)g * QT + t;
  const bool have1 = one_row && r1 < a.h;
  const int jn1 = j + 1;
  double pj = 0.0, pre[CH];
  if (have1) {
    if (j >= 0) pj = P[r1 + j * ld];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) pre[cc] = (jn1 + cc < w) ? P[r1 + (int64_t)(jn1 + cc) * ld] : 0.0;
  }

  double tau = 0.0, scale = 0.0, beta = 0.0;
  if (j >= 0) {
    {  // column c summed by two threads over alternate partials, 8 chains each
      const int c = t & (QB - 1), half = t >> 7;
      double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      if (c >= j && c < w) {
#pragma unroll
        for (int u = 0; u < NWG_MAX / 2; ++u) {
          const int q = 2 * u + half;
          if (q < a.nwg) s8[u & 7] += part_in[(int64_t)q * QB + c];
        }
      }
      sh_half[half][c] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    }
    __syncthreads();
    if (t < QB) sh_s[t] = sh_half[0][t] + sh_half[1][t];
    __syncthreads();
    const double x0 = piv_in[j];
    const double tail2 = sh_s[j];
    if (tail2 == 0.0) {
      tau = 0.0; beta = x0; scale = 0.0;
    } else {
      const double nrm = hypot(x0, sqrt(tail2));
      beta = (x0 >= 0.0) ? -nrm : nrm;
      tau = (beta - x0) / beta;
      scale = 1.0 / (x0 - beta);
    }
    if (t < w && t > j) sh_w[t] = piv_in[t] + scale * sh_s[t];
    if (g == 0 && t == 0) a.tau[j] = tau;
    __syncthreads();
  } else {
    // the statistics-only launch applies no reflector (f = 0); LDS left by
    // an earlier kernel must not reach 0 * sh_w as a NaN
    if (t < QB) sh_w[t] = 0.0;
    __syncthreads();
  }

  if (one_row) {
    const int jn = jn1;
    const int64_t r = have1 ? r1 : -1;
    double v = 0.0;
    if (r >= 0 && j >= 0) {
      if (r > j) { v = pj * scale; P[r + j * ld] = v; }
      else if (r == j) P[j + j * ld] = beta;
    }
    const bool below = (r >= 0 && j >= 0 && r > j), pivrow = (r >= 0 && j >= 0 && r == j);
    const double f = below ? tau * v : (pivrow ? tau : 0.0);
    double x = 0.0;
    if (r >= 0 && jn < w) x = pre[0] - f * sh_w[jn];
    const bool active = (r >= 0) && (r >= jn || pivrow);   // rows above the next pivot stay put
    double cur[CH];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) cur[cc] = pre[cc];
    for (int cb = jn; cb < w; cb += CH) {
      double nxt[CH];
      const int cbn = cb + CH;
#pragma unroll
      for (int cc = 0; cc < CH; ++cc)
        nxt[cc] = (have1 && active && cbn + cc < w) ? P[r + (int64_t)(cbn + cc) * ld] : 0.0;
      double acc[CH];
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) acc[cc] = 0.0;
      if (active) {
#pragma unroll
        for (int cc = 0; cc < CH; ++cc) {
          if (cb + cc < w) {
            cur[cc] -= f * sh_w[cb + cc];
            if (r > jn) acc[cc] += x * cur[cc];
          }
        }
        if (below || pivrow) {
#pragma unroll
          for (int cc = 0; cc < CH; ++cc)
            if (cb + cc < w) P[r + (int64_t)(cb + cc) * ld] = cur[cc];
        }
        if (r == jn) {
#pragma unroll
          for (int cc = 0; cc < CH; ++cc)
            if (cb + cc < w) piv_out[cb + cc] = cur[cc];
        }
      }
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) sh_acc[t][cc] = acc[cc];
      __syncthreads();
      {
        const int cc = t & (CH - 1), seg = t / CH;
        double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < CH; ++i) s4[i & 3] += sh_acc[seg * CH + i][cc];
        sh_seg[seg][cc] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
      }
      __syncthreads();
      if (t < CH && cb + t < w) {
        double sm = 0.0;
#pragma unroll
        for (int seg = 0; seg < QT / CH; ++seg) sm += sh_seg[seg][t];
        part_out[(int64_t)g * QB + cb + t] = sm;
      }
      __syncthreads();
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) cur[cc] = nxt[cc];
    }
    return;
  }

  const int64_t rbase = (int64_t)g * QT * a.rpt;
  double vr[RPT_MAX], xn[RPT_MAX];
  int64_t rr[RPT_MAX];
#pragma unroll
  for (int q = 0; q < RPT_MAX; ++q) {
    rr[q] = rbase + (int64_t)q * QT + t;
    vr[q] = 0.0; xn[q] = 0.0;
    if (q >= a.rpt || rr[q] >= a.h) { rr[q] = -1; continue; }
    const int64_t r = rr[q];
    if (j >= 0) {
      if (r > j) {
        vr[q] = P[r + j * ld] * scale;
        P[r + j * ld] = vr[q];
      } else if (r == j) {
        P[j + j * ld] = beta;
      }
    }
  }

  const int jn = j + 1;      // column whose statistics this launch gathers
  if (jn < w) {
#pragma unroll
    for (int q = 0; q < RPT_MAX; ++q) {
      const int64_t r = rr[q];
      if (r < 0) continue;
      double x = P[r + (int64_t)jn * ld];
      if (j >= 0 && r > j) x -= tau * vr[q] * sh_w[jn];
      else if (j >= 0 && r == j) x -= tau * sh_w[jn];
      xn[q] = x;
    }
  }
  for (int cb = jn; cb < w; cb += CH) {
    double acc[CH];
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) acc[cc] = 0.0;
#pragma unroll
    for (int q = 0; q < RPT_MAX; ++q) {
      const int64_t r = rr[q];
      if (r < 0) continue;
      const bool below = (j >= 0 && r > j), pivrow = (j >= 0 && r == j);
      if (r < jn && !pivrow) continue;          // rows above the next pivot: untouched
      const double x = xn[q];
      // all loads of the chunk first: a store to P between two loads would
      // order them (the compiler cannot rule out aliasing), serialising the
      // chunk into dependent round trips
      double pv[CH];
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) pv[cc] = (cb + cc < w) ? P[r + (int64_t)(cb + cc) * ld] : 0.0;
      const double f = below ? tau * vr[q] : (pivrow ? tau : 0.0);
#pragma unroll
      for (int cc = 0; cc < CH; ++cc) {
        if (cb + cc < w) {
          pv[cc] -= f * sh_w[cb + cc];
          if (r > jn) acc[cc] += x * pv[cc];
        }
      }
      if (below || pivrow) {
#pragma unroll
        for (int cc = 0; cc < CH; ++cc)
          if (cb + cc < w) P[r + (int64_t)(cb + cc) * ld] = pv[cc];
      }
      if (r == jn) {
#pragma unroll
        for (int cc = 0; cc < CH; ++cc)
          if (cb + cc < w) piv_out[cb + cc] = pv[cc];
      }
    }
    // workgroup sums of the CH column statistics: transpose through LDS,
    // 8 segments of 32 threads, then the 8 segment sums.
#pragma unroll
    for (int cc = 0; cc < CH; ++cc) sh_acc[t][cc] = acc[cc];
    __syncthreads();
    {
      const int cc = t & (CH - 1), seg = t / CH;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 0; i < CH; ++i) s4[i & 3] += sh_acc[seg * CH + i][cc];
      sh_seg[seg][cc] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
    __syncthreads();
    if (t < CH && cb + t < w) {
      double s = 0.0;
#pragma unroll
      for (int seg = 0; seg < QT / CH; ++seg) s += sh_seg[seg][t];
      part_out[(int64_t)g * QB + cb + t] = s;
    }
    __syncthreads();
  }
}

// ---- sub-panel by Cholesky QR + Householder reconstruction -------------
constexpr int RB = 32;          // reconstruction block (= QI)
constexpr int GCH = 64;         // rows staged per chunk of the Gram kernels
constexpr int NG_MAX = 64;      // workgroups of the row-parallel kernels (partial Grams)
constexpr int ST = 1024;        // threads of the small (one-workgroup) kernels

// Partial Gram matrices of a sub-panel: workgroup g sums, over its rows
// [g rows_per, (g+1) rows_per) of P (h x w, w <= 32), the outer products
// q_r^T q_r with q_r = p_r (APPLY: p_r Rinv, Rinv 32 x 32 upper, ld 32,
// and q_r is written back over p_r), into part[g] (32 x 32, column-major;
// entries beyond w are zero).
template <bool APPLY>
__global__ __launch_bounds__(256) void tsg_kernel(double* __restrict__ P, int64_t ld, int64_t h, int w,
                                                  const double* __restrict__ Rinv, double* __restrict__ part,
                                                  int64_t rows_per) {
  __shared__ double S[GCH][RB + 1];
  __shared__ double Ri[APPLY ? RB : 1][RB + 1];
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * rows_per;
  const int64_t r1 = (r0 + rows_per < h) ? r0 + rows_per : h;
  if constexpr (APPLY) {
    for (int e = t; e < RB * RB; e += 256) {
      const int i = e % RB, j = e / RB;
      Ri[i][j] = (i <= j && j < w) ? Rinv[i + j * RB] : 0.0;
    }
  }
  const int bi = t % 16, bj = t / 16;            // this thread's 2 x 2 block of the Gram
  double a00 = 0.0, a01 = 0.0, a10 = 0.0, a11 = 0.0;
  for (int64_t rb = r0; rb < r1; rb += GCH) {
#pragma unroll
    for (int q = 0; q < GCH * RB / 256; ++q) {
      const int e = t + 256 * q, row = e % GCH, col = e / GCH;
      const int64_t r = rb + row;
      S[row][col] = (r < r1 && col < w) ? P[r + (int64_t)col * ld] : 0.0;
    }
    __syncthreads();
    if constexpr (APPLY) {
      const int row = t >> 2, c0 = (t & 3) * 8;
      double y[8];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        double s0 = 0.0, s1 = 0.0;
        const int cc = c0 + c;
        int k = 0;
        for (; k + 1 <= cc; k += 2) { s0 += S[row][k] * Ri[k][cc]; s1 += S[row][k + 1] * Ri[k + 1][cc]; }
        if (k <= cc) s0 += S[row][k] * Ri[k][cc];
        y[c] = s0 + s1;
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 8; ++c) S[row][c0 + c] = y[c];
      __syncthreads();
      // the first pass's Q replaces P: the second pass and the
      // reconstruction work from these rounded values (recomputing them
      // from P, or folding R1^{-1} into a later product, would carry the
      // rounding of P R1^{-1}, of order u cond(P), into Q)
#pragma unroll
      for (int q = 0; q < GCH * RB / 256; ++q) {
        const int e = t + 256 * q, row2 = e % GCH, col = e / GCH;
        const int64_t r = rb + row2;
        if (r < r1 && col < w) P[r + (int64_t)col * ld] = S[row2][col];
      }
    }
    for (int row = 0; row < GCH; ++row) {
      const double x0 = S[row][2 * bi], x1 = S[row][2 * bi + 1];
      const double y0 = S[row][2 * bj], y1 = S[row][2 * bj + 1];
      a00 += x0 * y0; a01 += x0 * y1; a10 += x1 * y0; a11 += x1 * y1;
    }
    __syncthreads();
  }
  double* o = part + (int64_t)blockIdx.x * RB * RB;
  o[2 * bi + (2 * bj) * RB] = a00;
  o[2 * bi + (2 * bj + 1) * RB] = a01;
  o[2 * bi + 1 + (2 * bj) * RB] = a10;
  o[2 * bi + 1 + (2 * bj + 1) * RB] = a11;
}

// Sum of ng (<= NG_MAX) partial Grams into G (LDS), ST threads: each entry
// by one thread over the partials in a fixed order, 16 loads in flight.
__device__ void sum_partials(const double* part, int ng, double (*G)[RB + 1]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < RB * RB / ST; ++q) {
    const int e = t + ST * q;
    double a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) a[u] = 0.0;
    for (int g0 = 0; g0 < ng; g0 += 16) {
#pragma unroll
      for (int u = 0; u < 16; ++u)
        if (g0 + u < ng) a[u] += part[(int64_t)(g0 + u) * RB * RB + e];
    }
#pragma unroll
    for (int h = 8; h > 0; h >>= 1)
#pragma unroll
      for (int u = 0; u < h; ++u) a[u] += a[u + h];
    G[e % RB][e / RB] = a[0];
  }
  __syncthreads();
}

// Upper Cholesky factor R (G = R^T R, G's upper triangle) of the leading
// w x w block, G overwritten (LDS).  A pivot at or below rel * G(k,k), or
// not finite, counts as a failure and is replaced by G(k,k) (or 1) so that
// everything stays finite.  One barrier per step: step k reads row k of the
// working matrix, updates the rows below it and writes row k of R (a
// separate array), so no entry is read and written in the same step.
// Returns the failure on every thread.  ST threads.
__device__ bool small_chol(double (*G)[RB + 1], double (*R)[RB + 1], int w, double rel) {
  const int t = threadIdx.x;
  __shared__ double d0[RB];
  __shared__ int bad;
  if (t == 0) bad = 0;
  if (t < RB) d0[t] = (t < w) ? G[t][t] : 1.0;
  for (int e = t; e < RB * RB; e += ST) R[e % RB][e / RB] = 0.0;
  __syncthreads();
  for (int k = 0; k < w; ++k) {
    double piv = G[k][k];
    const double ref = d0[k];
    const bool fail = !(piv > rel * ref) || !(ref > 0.0) || !isfinite(piv);
    if (fail) piv = (ref > 0.0 && isfinite(ref)) ? ref : 1.0;
    const double rk = sqrt(piv), rinv = 1.0 / rk, pinv = 1.0 / piv;
    if (t == 0 && fail) bad = 1;
    for (int e = t; e < RB * RB; e += ST) {
      const int i = e % RB, j = e / RB;
      if (j < w && i <= j && i >= k) {
        if (i == k) R[k][j] = (j == k) ? rk : G[k][j] * rinv;
        else G[i][j] -= G[k][i] * G[k][j] * pinv;
      }
    }
    __syncthreads();
  }
  return bad != 0;
}

// Inverse of the upper triangular w x w block of R into Ri (zeros
// elsewhere): thread j back-substitutes column j.
__device__ void small_upper_inv(double (*R)[RB + 1], double (*Ri)[RB + 1], int w) {
  const int t = threadIdx.x;
  for (int e = t; e < RB * RB; e += ST) Ri[e % RB][e / RB] = 0.0;
  __syncthreads();
  if (t < w) {
    const int j = t;
    Ri[j][j] = 1.0 / R[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int p = i + 1; p <= j; ++p) s += R[i][p] * Ri[p][j];
      Ri[i][j] = -s / R[i][i];
    }
  }
  __syncthreads();
}

// Pass-one factor: R1 and R1^{-1} (32 x 32, ld 32) from the partial Grams.
// first: this is the panel's first sub-panel (the flag is reset, else only set).
__global__ __launch_bounds__(ST) void cq_chol_kernel(const double* __restrict__ part, int ng, int w,
                                                      double* __restrict__ R1, double* __restrict__ R1inv,
                                                      int* flag, int first) {
  __shared__ double G[RB][RB + 1];
  __shared__ double R[RB][RB + 1];
  __shared__ double Ri[RB][RB + 1];
  const int t = threadIdx.x;
  sum_partials(part, ng, G);
  const bool bad = small_chol(G, R, w, 1e-10);
  small_upper_inv(R, Ri, w);
  for (int e = t; e < RB * RB; e += ST) {
    R1[e] = R[e % RB][e / RB];
    R1inv[e] = Ri[e % RB][e / RB];
  }
  if (t == 0) {
    if (first) *flag = bad ? 1 : 0;
    else if (bad) *flag = 1;
  }
}

// Pass two and the reconstruction (one workgroup; see the file comment).
// P: the sub-panel's top-left corner, holding the first pass's Q (its first
// w rows are the top block).  With R2 the factor of the second Gram:
// Q = P R2^{-1}, W = S - Q1 = L U (signs chosen during the elimination).
// Outputs: Nm = -R2^{-1} U^{-1} (32 x 32, ld 32, upper; Y2 = P2 Nm), RL
// (32 x 32: R_H = S R2 R1 on and above the diagonal, L below), T (w x w
// upper in the panel's T slot, ld QB) and tau (w).
__global__ __launch_bounds__(ST) void cq_recon_kernel(const double* __restrict__ part, int ng, int w,
                                                       const double* __restrict__ R1g,
                                                       const double* __restrict__ P, int64_t ld,
                                                       double* __restrict__ Nm, double* __restrict__ RL,
                                                       double* __restrict__ T, double* __restrict__ tau,
                                                       int* flag) {
  __shared__ double A[RB][RB + 1];      // G2, then U^{-1}
  __shared__ double B[RB][RB + 1];      // R2, then U
  __shared__ double C[RB][RB + 1];      // R2^{-1}
  __shared__ double D[RB][RB + 1];      // R1, then L^{-1}
  __shared__ double Rm[RB][RB + 1];     // R = R2 R1
  __shared__ double W[RB][RB + 1];      // -Q1 -> L (below) / U (on and above)
  __shared__ double Pt[RB][RB + 1];     // the top block of the first pass's Q, then L
  __shared__ double sg[RB], ud[RB];
  __shared__ double red[ST];
  const int t = threadIdx.x;
  sum_partials(part, ng, A);
  // distance of pass one's Q from orthonormal
  double dev = 0.0;
  for (int e = t; e < w * w; e += ST) {
    const int i = e % w, j = e / w;
    dev = fmax(dev, fabs(A[i][j] - (i == j ? 1.0 : 0.0)));
  }
  red[t] = dev;
  __syncthreads();
  for (int sft = ST / 2; sft > 0; sft >>= 1) {
    if (t < sft) red[t] = fmax(red[t], red[t + sft]);
    __syncthreads();
  }
  bool bad = !(red[0] <= 0.1);
  __syncthreads();
  bad = small_chol(A, B, w, 0.5) || bad;
  small_upper_inv(B, C, w);
  for (int e = t; e < RB * RB; e += ST) {
    const int i = e % RB, j = e / RB;
    D[i][j] = R1g[e];
    Pt[i][j] = (i < w && j < w) ? P[i + (int64_t)j * ld] : 0.0;
  }
  __syncthreads();
  // R = R2 R1; W = -Q1 = -P1 R2^{-1}
  for (int e = t; e < RB * RB; e += ST) {
    const int i = e % RB, j = e / RB;
    double r = 0.0, q = 0.0;
    if (i < w && j < w) {
      if (i <= j)
        for (int k = i; k <= j; ++k) r += B[i][k] * D[k][j];
      for (int k = 0; k <= j; ++k) q += Pt[i][k] * C[k][j];
    }
    Rm[i][j] = r;
    W[i][j] = -q;
  }
  __syncthreads();
  double (*Lo)[RB + 1] = Pt;            // Pt is no longer needed
  // LU of S - Q1 without pivoting, S(i) chosen at step i: U(i,i) = S(i) + c
  // with S(i) = sign(c), c the updated (i,i) entry of -Q1.  One barrier per
  // step: U(k,k) goes to ud, column k of L to Lo (separate arrays), so the
  // entries read in step k are not written in it.
  for (int k = 0; k < w; ++k) {
    const double c = W[k][k];
    const double sk = (c >= 0.0) ? 1.0 : -1.0;
    const double ukk = sk + c, uinv = 1.0 / ukk;
    if (t == 0) { sg[k] = sk; ud[k] = ukk; }
    for (int e = t; e < RB * RB; e += ST) {
      const int i = e % RB, j = e / RB;
      if (i > k && i < w && j >= k && j < w) {
        if (j == k) Lo[i][k] = W[i][k] * uinv;
        else W[i][j] -= W[i][k] * W[k][j] * uinv;
      }
    }
    __syncthreads();
  }
  for (int e = t; e < RB * RB; e += ST) {
    const int i = e % RB, j = e / RB;
    if (i < w && j < w) {
      if (i == j) W[i][i] = ud[i];
      else if (i > j) W[i][j] = Lo[i][j];
    }
  }
  __syncthreads();
  // U^{-1} into A (the upper part of W is U)
  for (int e = t; e < RB * RB; e += ST) {
    const int i = e % RB, j = e / RB;
    B[i][j] = (i <= j && j < w) ? W[i][j] : 0.0;
  }
  __syncthreads();
  small_upper_inv(B, A, w);
  // L^{-1} (unit lower) into D: thread j forward-substitutes column j
  for (int e = t; e < RB * RB; e += ST) D[e % RB][e / RB] = 0.0;
  __syncthreads();
  if (t < w) {
    const int j = t;
    D[j][j] = 1.0;
    for (int i = j + 1; i < w; ++i) {
      double s = 0.0;
      for (int p = j; p < i; ++p) s += W[i][p] * D[p][j];
      D[i][j] = -s;
    }
  }
  __syncthreads();
  // outputs
  for (int e = t; e < RB * RB; e += ST) {
    const int i = e % RB, j = e / RB;
    double nm = 0.0, tv = 0.0, rl = 0.0;
    if (i < w && j < w) {
      if (i <= j) {
        for (int k = i; k <= j; ++k) nm -= C[i][k] * A[k][j];
        // T(i,j) = sum_k U(i,k) S(k) Linv(j,k), k in [i, j]
        for (int k = i; k <= j; ++k) tv += W[i][k] * sg[k] * D[j][k];
        rl = sg[i] * Rm[i][j];
      } else {
        rl = W[i][j];
      }
    }
    Nm[e] = nm;
    RL[e] = rl;
    if (i < w && j < w) T[i + (int64_t)j * QB] = tv;
    if (i == j && i < w) tau[i] = tv;
  }
  if (t == 0 && bad) *flag = 1;
}

// Writes the reconstructed sub-panel unless the flag is set: rows below the
// first w (the first pass's Q) become Y2 = Q2 Nm, the first w rows R_H
// (upper) and L (below).  Four threads per row, each loading and writing 8
// columns; workgroup g takes rows [64 g, 64 g + 64).  Registers are capped
// at 128 per lane (four waves per SIMD) so that its waves find room beside
// the trailing update's GEMM, which runs next to the panel.
__global__ __launch_bounds__(256, 4) void cq_write_kernel(double* __restrict__ P, int64_t ld, int64_t h, int w,
                                                       const double* __restrict__ Nm,
                                                       const double* __restrict__ RL, const int* flag) {
  if (*flag) return;
  __shared__ double Ns[RB][RB + 1];
  __shared__ double Xs[64][RB + 1];      // the workgroup's 64 rows of the first pass's Q
  const int t = threadIdx.x;
  for (int e = t; e < RB * RB; e += 256) Ns[e % RB][e / RB] = Nm[e];
  const int lr = t >> 2, c0 = (t & 3) * 8;
  const int64_t r = (int64_t)blockIdx.x * 64 + lr;
  const bool body = r < h && r >= w;
  // each thread stages its own 8 columns of its row
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int c = c0 + u;
    Xs[lr][c] = (body && c < w) ? P[r + (int64_t)c * ld] : 0.0;
  }
  __syncthreads();
  if (r >= h) return;
  if (!body) {
#pragma unroll
    for (int c = c0; c < c0 + 8; ++c)
      if (c < w) P[r + (int64_t)c * ld] = RL[r + c * RB];
    return;
  }
  // Nm is upper triangular with zeros stored below: the full sums give the
  // triangular product.  Two sums per output (even and odd k), each in
  // increasing k.  The row is read from LDS, so a thread's stores (its own
  // 8 columns, read from HBM only by itself) race with nothing.
  double s0[8], s1[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s0[u] = s1[u] = 0.0;
#pragma unroll 2
  for (int k = 0; k < RB; k += 2) {
    const double xa = Xs[lr][k], xb = Xs[lr][k + 1];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      s0[u] += xa * Ns[k][c0 + u];
      s1[u] += xb * Ns[k + 1][c0 + u];
    }
  }
#pragma unroll
  for (int u = 0; u < 8; ++u)
    if (c0 + u < w) P[r + (int64_t)(c0 + u) * ld] = s0[u] + s1[u];
}

// T (w x w, upper) of the compact WY form from G = V^T V and tau:
// T(j,j) = tau_j, T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j).  One LDS array
// holds G above the diagonal and T^T on and below it.
//   1. the diagonal blocks of TL = 32 by the recurrence, thread i owning row
//      i of its block (rows are independent);
//   2. blocks merged pairwise, 32 -> 64 -> 128: for consecutive reflector
//      sets with factors T1, T2 the merged factor has the off-diagonal block
//      T12 = -T1 (V1^T V2) T2 = -T1 G12 T2, formed as Y = G12 T2 (T2 upper)
//      then -T1 Y (T1 upper), 32 columns of Y at a time in LDS.
// The recurrence alone would leave row 0 a chain of w^2/2 dependent steps.
constexpr int TL = 32;
constexpr int BTT = 1024;       // threads of build_t_kernel
__global__ __launch_bounds__(BTT) void build_t_kernel(const double* G, int64_t ldg, const double* tau,
                                                     double* T, int64_t ldt, int w) {
  __shared__ double L[QB][QB];          // row pitch QB: the diagonal walk of step 1 has odd stride
  __shared__ double Ys[2 * TL][TL + 1];
  const int t = threadIdx.x;
  for (int e = t; e < w * w; e += BTT) {   // only the w x w corner is used
    const int r = e % w, c = e / w;
    L[r][c] = (r < c) ? G[r + (int64_t)c * ldg] : 0.0;
  }
  __syncthreads();
  if (t < w) {
    const int i = t, jend = ((i / TL + 1) * TL < w) ? (i / TL + 1) * TL : w;
    L[i][i] = tau[i];                       // T(i,i), stored at L[i][i]
    for (int j = i + 1; j < jend; ++j) {
      // T(i,k) = L[k][i]; G(k,j) = L[k][j]; four independent chains
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
      int k = i;
      for (; k + 4 <= j; k += 4) {
        a0 += L[k][i] * L[k][j];
        a1 += L[k + 1][i] * L[k + 1][j];
        a2 += L[k + 2][i] * L[k + 2][j];
        a3 += L[k + 3][i] * L[k + 3][j];
      }
      for (; k < j; ++k) a0 += L[k][i] * L[k][j];
      L[j][i] = -tau[j] * ((a0 + a1) + (a2 + a3));
    }
  }
  __syncthreads();
  for (int sz = TL; sz < w; sz *= 2) {            // merge blocks of sz into 2 sz
    // combos a0 = 0, 2 sz, ...; each takes sz rows of Ys, TL columns at a time
    const int ncombo = (QB / (2 * sz)) < 1 ? 1 : QB / (2 * sz);
    for (int cb = 0; cb < sz; cb += TL) {
      // Y(r, c) = sum_{k <= c} G(a0 + r, a0 + sz + k) T(a0 + sz + k, a0 + sz + c)
      for (int e = t; e < ncombo * sz * TL; e += BTT) {
        const int cc = e % TL, r = (e / TL) % sz, q = e / (TL * sz);
        const int a0 = q * 2 * sz, c = cb + cc;
        if (a0 + sz + c >= w) continue;
        const int bj = a0 + sz;
        double a0s = 0.0, a1s = 0.0, a2s = 0.0, a3s = 0.0;   // independent chains
        int k = 0;
        for (; k + 3 <= c; k += 4) {
          a0s += L[a0 + r][bj + k] * L[bj + c][bj + k];
          a1s += L[a0 + r][bj + k + 1] * L[bj + c][bj + k + 1];
          a2s += L[a0 + r][bj + k + 2] * L[bj + c][bj + k + 2];
          a3s += L[a0 + r][bj + k + 3] * L[bj + c][bj + k + 3];
        }
        for (; k <= c; ++k) a0s += L[a0 + r][bj + k] * L[bj + c][bj + k];
        Ys[q * sz + r][cc] = (a0s + a1s) + (a2s + a3s);
      }
      __syncthreads();
      // T(a0 + r, a0 + sz + c) = -sum_{k >= r} T(a0 + r, a0 + k) Y(k, c)
      for (int e = t; e < ncombo * sz * TL; e += BTT) {
        const int cc = e % TL, r = (e / TL) % sz, q = e / (TL * sz);
        const int a0 = q * 2 * sz, c = cb + cc;
        if (a0 + sz + c >= w) continue;
        const int yb = q * sz;
        double a0s = 0.0, a1s = 0.0, a2s = 0.0, a3s = 0.0;
        int k = r;
        for (; k + 4 <= sz; k += 4) {
          a0s += L[a0 + k][a0 + r] * Ys[yb + k][cc];
          a1s += L[a0 + k + 1][a0 + r] * Ys[yb + k + 1][cc];
          a2s += L[a0 + k + 2][a0 + r] * Ys[yb + k + 2][cc];
          a3s += L[a0 + k + 3][a0 + r] * Ys[yb + k + 3][cc];
        }
        for (; k < sz; ++k) a0s += L[a0 + k][a0 + r] * Ys[yb + k][cc];
        L[a0 + sz + c][a0 + r] = -((a0s + a1s) + (a2s + a3s));
      }
      __syncthreads();
    }
  }
  for (int e = t; e < w * w; e += BTT) {
    const int r = e % w, c = e / w;
    T[r + (int64_t)c * ldt] = (r <= c) ? L[c][r] : 0.0;
  }
}

__global__ void eye_cols_kernel(double* Q, int64_t m, int64_t q, int64_t ldq, int64_t c0) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t j = blockIdx.y; j < q; j += gridDim.y)
    if (i < m) Q[i + j * ldq] = (i == c0 + j) ? 1.0 : 0.0;
}

}  // namespace

int64_t qr_scratch_doubles(int64_t m, int64_t n) {
  const int64_t nn = n > 1 ? n : 1;
  const int64_t mm = m > 1 ? m : 1;
  return 2 * 64 * QB + 2 * QB + QB * QB + 2 * QB * nn + 64 * QB * QB + 8 * QB * nn + 256 +
         (int64_t)NG_MAX * RB * RB + 4 * RB * RB + 64 + QB * mm + 2 * QB * nn + 64 * QB * QB + 8 * QB * nn;
}

QrScratch carve_qr_scratch(double* w, int64_t m, int64_t n) {
  const int64_t nn = n > 1 ? n : 1;
  const int64_t mm = m > 1 ? m : 1;
  QrScratch s;
  s.part = w; w += 2 * 64 * QB;
  s.piv = w; w += 2 * QB;
  s.G = w; w += QB * QB;
  s.W1 = w; w += QB * nn;
  s.W2 = w; w += QB * nn;
  s.ws = w; s.ws_doubles = 64 * QB * QB + 8 * QB * nn;
  w += s.ws_doubles + 256;
  s.cq_part = w; w += (int64_t)NG_MAX * RB * RB;
  s.cq_small = w; w += 4 * RB * RB;
  s.cq_flag = reinterpret_cast<int*>(w); w += 64;
  s.backup = w; s.backup_rows = mm; w += QB * mm;
  s.W1b = w; w += QB * nn;
  s.W2b = w; w += QB * nn;
  s.wsb = w; s.wsb_doubles = 64 * QB * QB + 8 * QB * nn;
  return s;
}

namespace {

// T (w x w, ld QB) of the compact WY form of the w reflectors stored below
// the diagonal of V (h x w): G = V^T V, then the T recurrence.
void build_t(const double* V, int64_t h, int w, int64_t ld, const double* tau, double* T,
             const QrScratch& sc, hipStream_t s) {
  Gemm g;
  g.M = w; g.N = w; g.K = h; g.A = V; g.lda = ld; g.ta = true; g.a_unit_lower = true;
  g.B = V; g.ldb = ld; g.b_unit_lower = true; g.C = sc.G; g.ldc = QB;
  g.ws = sc.ws; g.ws_doubles = sc.ws_doubles;
  dgemm(g, s);
  build_t_kernel<<<1, BTT, 0, s>>>(sc.G, QB, tau, T, QB, w);
  QDWHP_LAUNCH_CHECK();
}

// C (h x nc, ld) <- (I - V T^T V^T) C: W1 = V^T C, W2 = T^T W1, C -= V W2.
// Work buffers of a block-reflector update (one set per stream).
struct QtBufs {
  double* W1; double* W2; double* ws; int64_t ws_doubles;
};
QtBufs main_bufs(const QrScratch& sc) { return QtBufs{sc.W1, sc.W2, sc.ws, sc.ws_doubles}; }

void apply_qt(const double* V, int64_t h, int w, int64_t ld, const double* T, double* C, int64_t nc,
              const QtBufs& b, hipStream_t s) {
  Gemm g1;   // W1 = V^T C
  g1.M = w; g1.N = nc; g1.K = h; g1.A = V; g1.lda = ld; g1.ta = true; g1.a_unit_lower = true;
  g1.B = C; g1.ldb = ld; g1.C = b.W1; g1.ldc = QB; g1.ws = b.ws; g1.ws_doubles = b.ws_doubles;
  dgemm(g1, s);
  Gemm g2;   // W2 = T^T W1
  g2.M = w; g2.N = nc; g2.K = w; g2.A = T; g2.lda = QB; g2.ta = true;
  g2.B = b.W1; g2.ldb = QB; g2.C = b.W2; g2.ldc = QB;
  dgemm(g2, s);
  Gemm g3;   // C -= V W2
  g3.M = h; g3.N = nc; g3.K = w; g3.alpha = -1.0; g3.beta = 1.0;
  g3.A = V; g3.lda = ld; g3.a_unit_lower = true; g3.B = b.W2; g3.ldb = QB;
  g3.C = C; g3.ldc = ld;
  dgemm(g3, s);
}
void apply_qt(const double* V, int64_t h, int w, int64_t ld, const double* T, double* C, int64_t nc,
              const QrScratch& sc, hipStream_t s) {
  apply_qt(V, h, w, ld, T, C, nc, main_bufs(sc), s);
}

}  // namespace

namespace {

// Rows a panel at column c0 (w columns) touches.  For a stacked matrix
// [A; I] (stacked = rows of A, the identity below), the reflectors of
// columns before c0 fill only rows 0 .. c0-1 of the identity block, so the
// panel's columns are zero below stacked row stacked + c0 + w and its
// reflectors (and the trailing update) stop there.
int64_t panel_rows(int64_t m, int64_t c0, int w, int64_t stacked) {
  const int64_t h = m - c0;
  return stacked > 0 ? std::min<int64_t>(h, stacked + w) : h;
}

// Sub-panels of one panel by Cholesky QR with Householder reconstruction
// (V: the panel, h x w); sub-panel T factors go to the panel's T slot.
// Returns false when a sub-panel failed its checks (the panel is then
// partly overwritten and must be restored by the caller).
bool panel_recon(double* V, int64_t h, int w, int64_t lda, double* tau, double* T, const QrScratch& sc,
                 hipStream_t s) {
  double* R1 = sc.cq_small;
  double* R1inv = R1 + RB * RB;
  double* Nm = R1inv + RB * RB;
  double* RL = Nm + RB * RB;
  for (int j0 = 0; j0 < w; j0 += QI) {
    const int wi = (w - j0) < QI ? (w - j0) : QI;
    double* P = V + j0 + j0 * lda;
    const int64_t hp = h - j0;
    const int ng = (int)std::min<int64_t>(NG_MAX, cdiv(hp, GCH));
    const int64_t rows_per = cdiv(hp, ng);
    tsg_kernel<false><<<ng, 256, 0, s>>>(P, lda, hp, wi, nullptr, sc.cq_part, rows_per);
    QDWHP_LAUNCH_CHECK();
    cq_chol_kernel<<<1, ST, 0, s>>>(sc.cq_part, ng, wi, R1, R1inv, sc.cq_flag, j0 == 0 ? 1 : 0);
    QDWHP_LAUNCH_CHECK();
    tsg_kernel<true><<<ng, 256, 0, s>>>(P, lda, hp, wi, R1inv, sc.cq_part, rows_per);
    QDWHP_LAUNCH_CHECK();
    cq_recon_kernel<<<1, ST, 0, s>>>(sc.cq_part, ng, wi, R1, P, lda, Nm, RL, T, tau + j0, sc.cq_flag);
    QDWHP_LAUNCH_CHECK();
    cq_write_kernel<<<(unsigned)cdiv(hp, 64), 256, 0, s>>>(P, lda, hp, wi, Nm, RL, sc.cq_flag);
    QDWHP_LAUNCH_CHECK();
    const int rest = w - j0 - wi;
    if (rest > 0) apply_qt(P, hp, wi, lda, T, P + (int64_t)wi * lda, rest, sc, s);
  }
  int hf = 0;
  QDWHP_HIP(hipMemcpyAsync(&hf, sc.cq_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  return hf == 0;
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return true;
  return st != hipStreamCaptureStatusNone;
}

}  // namespace

int64_t geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, double* Tall,
              const QrScratch& sc, hipStream_t s, const PanelWatch* watch, bool recon, int64_t stacked) {
  const bool use_recon = recon && sc.cq_part && qdwhp_tune_get("qr.recon", 1) != 0 && !stream_capturing(s);
  // per panel height: "qr.recon@b" (b = ceil(log2 h)) where the autotuner set it
  // Overlap (only where the host already waits per panel): the update of
  // the next panel's columns stays on the main stream, the rest of the
  // trailing update goes to a helper stream and runs while the next panel
  // is factored.  A panel's columns must have every earlier update, so
  // the main stream waits for the helper's previous update before touching
  // the next panel.  Every column gets the same updates in the same order
  // as on one stream; only the K split of the narrow V^T C product (chosen
  // from its tile count) differs, a rounding-level difference.
  const bool overlap = use_recon && sc.W1b && !no_alloc_mode() && qdwhp_tune_get("qr.overlap", 1) != 0;
  std::unique_ptr<AuxLease> aux;
  if (overlap) {
    int dev = 0;
    QDWHP_HIP(hipGetDevice(&dev));
    aux.reset(new AuxLease(dev));
  }
  const QtBufs mb = main_bufs(sc);
  const QtBufs ab = overlap ? QtBufs{sc.W1b, sc.W2b, sc.wsb, sc.wsb_doubles} : mb;
  int64_t last_wide = -1;        // panel index of the helper stream's last update
  auto join = [&]() {
    if (last_wide >= 0) QDWHP_HIP(hipStreamWaitEvent(s, (*aux)->done[last_wide % kAuxRing], 0));
  };
  int64_t pi = 0;
  for (int64_t c0 = 0; c0 < n; c0 += QB, ++pi) {
    const int w = (int)((n - c0) < QB ? (n - c0) : QB);
    const int64_t h = panel_rows(m, c0, w, stacked);
    double* V = A + c0 + c0 * lda;
    double* T = Tall + (c0 / QB) * QB * QB;
    bool done = false;
    if (use_recon && h <= sc.backup_rows && qdwhp_tune_get_sized("qr.recon", h, 1) != 0) {
      QDWHP_HIP(hipMemcpy2DAsync(sc.backup, h * sizeof(double), V, lda * sizeof(double), h * sizeof(double),
                                 w, hipMemcpyDeviceToDevice, s));
      done = panel_recon(V, h, w, lda, tau + c0, T, sc, s);
      if (!done)
        QDWHP_HIP(hipMemcpy2DAsync(V, lda * sizeof(double), sc.backup, h * sizeof(double), h * sizeof(double),
                                   w, hipMemcpyDeviceToDevice, s));
    }
    // The panel by column steps, in sub-panels of QI columns: the column
    // launches only sweep their sub-panel, and each finished sub-panel's
    // reflectors reach the rest of the panel as one blocked update (its T is
    // built in the panel's T slot, which the panel's own T overwrites below).
    for (int j0 = 0; !done && j0 < w; j0 += QI) {
      const int wi = (w - j0) < QI ? (w - j0) : QI;
      Panel p;
      p.P = V + j0 + j0 * lda; p.ld = lda; p.h = h - j0; p.w = wi;
      p.tau = tau + c0 + j0; p.part = sc.part; p.piv = sc.piv;
      p.rpt = (int)cdiv(p.h, (int64_t)QT * NWG_MAX);
      if (p.rpt > RPT_MAX) throw HipError{hipErrorInvalidValue};   // h > 131072 rows
      p.nwg = (int)cdiv(p.h, (int64_t)QT * p.rpt);
      for (int j = -1; j < wi; ++j) {
        qr_col_kernel<<<p.nwg, QT, 0, s>>>(p, j);
        QDWHP_LAUNCH_CHECK();
      }
      const int rest = w - j0 - wi;
      if (rest > 0) {
        build_t(p.P, p.h, wi, lda, p.tau, T, sc, s);
        apply_qt(p.P, p.h, wi, lda, T, p.P + (int64_t)wi * lda, rest, sc, s);
      }
    }
    build_t(V, h, w, lda, tau + c0, T, sc, s);
    if (watch && (*watch)(c0, w)) { join(); return c0 + w; }   // the caller needs no further columns
    const int64_t nc = n - c0 - w;
    if (nc <= 0) continue;
    double* C = A + c0 + (c0 + w) * lda;
    if (!overlap) { apply_qt(V, h, w, lda, T, C, nc, mb, s); continue; }
    const int64_t nnext = nc < QB ? nc : QB;
    const int64_t nrest = nc - nnext;
    if (nrest > 0) {                           // the rest, on the helper stream
      hipStream_t sb = (*aux)->s;
      QDWHP_HIP(hipEventRecord((*aux)->ready[pi % kAuxRing], s));
      QDWHP_HIP(hipStreamWaitEvent(sb, (*aux)->ready[pi % kAuxRing], 0));
      apply_qt(V, h, w, lda, T, C + nnext * lda, nrest, ab, sb);
    }
    join();                                    // the next panel has the earlier updates
    apply_qt(V, h, w, lda, T, C, nnext, mb, s);
    if (nrest > 0) {
      QDWHP_HIP(hipEventRecord((*aux)->done[pi % kAuxRing], (*aux)->s));
      last_wide = pi;
    }
  }
  join();
  return n;
}

void orgqr(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
           int64_t c0, int64_t q, double* Q, int64_t ldq, const QrScratch& sc, hipStream_t s, int64_t stacked) {
  if (q <= 0) return;
  dim3 grid((unsigned)cdiv(m, 256), (unsigned)(q < 65535 ? q : 65535));
  eye_cols_kernel<<<grid, 256, 0, s>>>(Q, m, q, ldq, c0);
  QDWHP_LAUNCH_CHECK();
  apply_q(A, m, lda, Tall, upto, Q, q, ldq, sc, s, stacked);
}

void apply_q(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
             double* Q, int64_t q, int64_t ldq, const QrScratch& sc, hipStream_t s, int64_t stacked) {
  if (upto <= 0 || q <= 0) return;
  const int64_t np = cdiv(upto, QB);
  for (int64_t pi = np - 1; pi >= 0; --pi) {
    const int64_t pc0 = pi * QB;
    const int w = (int)((upto - pc0) < QB ? (upto - pc0) : QB);
    const int64_t h = panel_rows(m, pc0, w, stacked);
    const double* V = A + pc0 + pc0 * lda;
    const double* T = Tall + pi * QB * QB;
    double* Qp = Q + pc0;
    Gemm g1;   // W1 = V^T Qp
    g1.M = w; g1.N = q; g1.K = h; g1.A = V; g1.lda = lda; g1.ta = true; g1.a_unit_lower = true;
    g1.B = Qp; g1.ldb = ldq; g1.C = sc.W1; g1.ldc = QB; g1.ws = sc.ws; g1.ws_doubles = sc.ws_doubles;
    dgemm(g1, s);
    Gemm g2;   // W2 = T W1
    g2.M = w; g2.N = q; g2.K = w; g2.A = T; g2.lda = QB; g2.B = sc.W1; g2.ldb = QB;
    g2.C = sc.W2; g2.ldc = QB;
    dgemm(g2, s);
    Gemm g3;   // Qp -= V W2
    g3.M = h; g3.N = q; g3.K = w; g3.alpha = -1.0; g3.beta = 1.0;
    g3.A = V; g3.lda = lda; g3.a_unit_lower = true; g3.B = sc.W2; g3.ldb = QB; g3.C = Qp; g3.ldc = ldq;
    dgemm(g3, s);
  }
}

}  // namespace qdwhp
