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
#include "common.h"
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
__global__ __launch_bounds__(QB) void build_t_kernel(const double* G, int64_t ldg, const double* tau,
                                                     double* T, int64_t ldt, int w) {
  __shared__ double L[QB][QB];          // row pitch QB: the diagonal walk of step 1 has odd stride
  __shared__ double Ys[2 * TL][TL + 1];
  const int t = threadIdx.x;
  for (int e = t; e < w * w; e += QB) {   // only the w x w corner is used
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
      for (int e = t; e < ncombo * sz * TL; e += QB) {
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
      for (int e = t; e < ncombo * sz * TL; e += QB) {
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
  for (int e = t; e < w * w; e += QB) {
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
  (void)m;
  const int64_t nn = n > 1 ? n : 1;
  return 2 * 64 * QB + 2 * QB + QB * QB + 2 * QB * nn + 64 * QB * QB + 8 * QB * nn + 256;
}

QrScratch carve_qr_scratch(double* w, int64_t m, int64_t n) {
  (void)m;
  const int64_t nn = n > 1 ? n : 1;
  QrScratch s;
  s.part = w; w += 2 * 64 * QB;
  s.piv = w; w += 2 * QB;
  s.G = w; w += QB * QB;
  s.W1 = w; w += QB * nn;
  s.W2 = w; w += QB * nn;
  s.ws = w; s.ws_doubles = 64 * QB * QB + 8 * QB * nn;
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
  build_t_kernel<<<1, QB, 0, s>>>(sc.G, QB, tau, T, QB, w);
  QDWHP_LAUNCH_CHECK();
}

// C (h x nc, ld) <- (I - V T^T V^T) C: W1 = V^T C, W2 = T^T W1, C -= V W2.
void apply_qt(const double* V, int64_t h, int w, int64_t ld, const double* T, double* C, int64_t nc,
              const QrScratch& sc, hipStream_t s) {
  Gemm g1;   // W1 = V^T C
  g1.M = w; g1.N = nc; g1.K = h; g1.A = V; g1.lda = ld; g1.ta = true; g1.a_unit_lower = true;
  g1.B = C; g1.ldb = ld; g1.C = sc.W1; g1.ldc = QB; g1.ws = sc.ws; g1.ws_doubles = sc.ws_doubles;
  dgemm(g1, s);
  Gemm g2;   // W2 = T^T W1
  g2.M = w; g2.N = nc; g2.K = w; g2.A = T; g2.lda = QB; g2.ta = true;
  g2.B = sc.W1; g2.ldb = QB; g2.C = sc.W2; g2.ldc = QB;
  dgemm(g2, s);
  Gemm g3;   // C -= V W2
  g3.M = h; g3.N = nc; g3.K = w; g3.alpha = -1.0; g3.beta = 1.0;
  g3.A = V; g3.lda = ld; g3.a_unit_lower = true; g3.B = sc.W2; g3.ldb = QB;
  g3.C = C; g3.ldc = ld;
  dgemm(g3, s);
}

}  // namespace

int64_t geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, double* Tall,
              const QrScratch& sc, hipStream_t s, const PanelWatch* watch) {
  for (int64_t c0 = 0; c0 < n; c0 += QB) {
    const int w = (int)((n - c0) < QB ? (n - c0) : QB);
    const int64_t h = m - c0;
    double* V = A + c0 + c0 * lda;
    double* T = Tall + (c0 / QB) * QB * QB;
    // The panel itself is factored in sub-panels of QI columns: the column
    // launches only sweep their sub-panel, and each finished sub-panel's
    // reflectors reach the rest of the panel as one blocked update (its T is
    // built in the panel's T slot, which the panel's own T overwrites below).
    for (int j0 = 0; j0 < w; j0 += QI) {
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
    if (watch && (*watch)(c0, w)) return c0 + w;   // the caller needs no further columns
    const int64_t nc = n - c0 - w;
    if (nc > 0) apply_qt(V, h, w, lda, T, A + c0 + (c0 + w) * lda, nc, sc, s);
  }
  return n;
}

void orgqr(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
           int64_t c0, int64_t q, double* Q, int64_t ldq, const QrScratch& sc, hipStream_t s) {
  if (q <= 0) return;
  dim3 grid((unsigned)cdiv(m, 256), (unsigned)(q < 65535 ? q : 65535));
  eye_cols_kernel<<<grid, 256, 0, s>>>(Q, m, q, ldq, c0);
  QDWHP_LAUNCH_CHECK();
  apply_q(A, m, lda, Tall, upto, Q, q, ldq, sc, s);
}

void apply_q(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
             double* Q, int64_t q, int64_t ldq, const QrScratch& sc, hipStream_t s) {
  if (upto <= 0 || q <= 0) return;
  const int64_t np = cdiv(upto, QB);
  for (int64_t pi = np - 1; pi >= 0; --pi) {
    const int64_t pc0 = pi * QB;
    const int w = (int)((upto - pc0) < QB ? (upto - pc0) : QB);
    const int64_t h = m - pc0;
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
