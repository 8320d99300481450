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
//      inverted by one workgroup of four waves, and a node of at most 128
//      rows runs its products in two one-workgroup kernels (below);
//   2. Z^{-1} = W^{-1} W^{-T}, upper tiles only, K starting at the tile column;
//   3. mirror the upper triangle.
#include <algorithm>
#include <vector>

#include "common.h"
#include "drivers.h"

namespace qdwhp {
namespace {

constexpr int NB = 64;

// Factor the bs x bs leaf (bs <= 64) at Z (upper triangle read) and write its
// inverse factor W^{-1} (upper, zeros below) to Wi.  The factor W itself is
// written back to Z's upper triangle.  Rows and columns past bs are padded
// with the identity, so the padded block factors to the identity and leaves
// the leading block untouched.
//
// One workgroup of four waves (one per SIMD), one barrier per step.  With
// L = W^T (lower):
//   factorisation (right-looking): wave w keeps the columns j = 4c + w of
//   the matrix in registers, lane = row.  At step k every wave reads column
//   k from the LDS buffer, forms L(i, k) = A(i, k) / sqrt(A(k, k)) and
//   updates its trailing columns, A(i, j) -= L(i, k) L(j, k); the wave that
//   owns column k + 1 updates it first and publishes it into the other
//   buffer (three buffers: the rest of step k's update is applied at step
//   k + 1, while the next pivot's loads are in flight).  The pivot's
//   reciprocal square root is the hardware estimate refined by two Newton
//   steps.
//   inverse M = L^{-1} (right-looking): lane = column j, wave w keeps the
//   sums U(r, j) = sum_{k < r} L(r, k) M(k, j) for the rows r = 4q + w.
//   Row k of M, (delta - U(k, :)) / L(k, k), is published by the wave that
//   owns row k one step ahead; every wave then adds L(r, k) M(k, :) to its
//   rows past k + 1, and at the end stores its rows of M as columns of
//   W^{-1} = M^T.
// The cyclic layouts keep all four waves busy as the active part shrinks;
// each wave runs its own copy of the steps, so every register index and
// every skipped update is decided at compile time.
constexpr int LW = 256;   // threads of the leaf workgroup
constexpr int LQ = NB / 4;   // columns / rows per wave

template <int W>
__device__ __forceinline__ void leaf_wave(double* Z, int64_t ldz, double* Wi, int64_t ldw, int bs, int* flag,
                                          double (*S)[NB + 1], double (*cl)[NB], double* rpv) {
  const int i = threadIdx.x & 63;
  double a[LQ];                        // a[c] = A(i, 4c + W) (lower part; the upper part is never read)
#pragma clang loop unroll(full)
  for (int c = 0; c < LQ; ++c) a[c] = S[i][4 * c + W];
  if (W == 0) cl[0][i] = a[0];         // column 0
  __syncthreads();
  bool bad = false;
  double pli2 = 0.0;                   // step k - 1's L(i, k-1) / L(k-1, k-1), for its deferred update
#pragma clang loop unroll(full)
  for (int k = 0; k < NB; ++k) {
    const double* buf = cl[k % 3];
    const double* pbuf = cl[(k + 2) % 3];        // column k - 1 as published
    double d = buf[k];
    const double ai = buf[i];
    // step k - 1's update of this wave's columns past k (issued while the
    // pivot's loads are in flight; column k came updated from its owner)
    if (k > 0) {
#pragma clang loop unroll(full)
      for (int c = 0; c < LQ; ++c) {
        const int j = 4 * c + W;
        if (j > k) a[c] = __builtin_fma(-pli2, pbuf[j], a[c]);
      }
    }
    const bool nonpos = !(d > 0.0) || !isfinite(d);
    bad = bad || nonpos;
    d = nonpos ? 1.0 : d;
    double y = __builtin_amdgcn_rsq(d);
#pragma clang loop unroll(full)
    for (int it = 0; it < 2; ++it) y = __builtin_fma(y, __builtin_fma(-0.5 * d * y, y, 0.5), y);
    const double p = d * y;                       // L(k, k)
    const double lik = (i > k) ? ai * y : 0.0;    // L(i, k) for the rows past k
    const double li2 = lik * y;                   // times A(j, k) gives L(i, k) L(j, k)
    if ((k & 3) == W) a[k >> 2] = (i == k) ? p : ((i > k) ? lik : a[k >> 2]);   // keep L(:, k)
    if (W == 0 && i == 0) rpv[k] = y;
    if (k + 1 < NB && ((k + 1) & 3) == W) {       // column k + 1 now, then publish it
      a[(k + 1) >> 2] = __builtin_fma(-li2, buf[k + 1], a[(k + 1) >> 2]);
      cl[(k + 1) % 3][i] = a[(k + 1) >> 2];
    }
    pli2 = li2;
    __syncthreads();
  }
  if (bad && W == 0 && i == 0) *flag = 1;
  // L to LDS (row i), then W = L^T into Z's upper triangle: Z(r, c) =
  // L(c, r) for c >= r; this wave writes the columns c = 4q + W (lane = row)
#pragma clang loop unroll(full)
  for (int c = 0; c < LQ; ++c) S[i][4 * c + W] = a[c];
  __syncthreads();
  if (i < bs) {
#pragma clang loop unroll(full)
    for (int q = 0; q < LQ; ++q) {
      const int c = 4 * q + W;
      if (c < bs && c >= i) Z[i + (int64_t)c * ldz] = S[c][i];
    }
  }
  double acc[LQ], mrow[LQ];            // U(4q + W, j); M(4q + W, j) once final
#pragma clang loop unroll(full)
  for (int q = 0; q < LQ; ++q) { acc[q] = 0.0; mrow[q] = 0.0; }
  if (W == 0) {                        // row 0 of M
    const double m0 = ((i == 0) ? 1.0 : 0.0) * rpv[0];
    cl[0][i] = m0;
    mrow[0] = m0;
  }
  __syncthreads();
#pragma clang loop unroll(full)
  for (int k = 0; k < NB; ++k) {
    const double mk = cl[k & 1][i];    // M(k, j)
    if (k + 1 < NB && ((k + 1) & 3) == W) {       // row k + 1 of M, published one step ahead
      const int q1 = (k + 1) >> 2;
      acc[q1] = __builtin_fma(S[k + 1][k], mk, acc[q1]);
      const double m1 = (((i == k + 1) ? 1.0 : 0.0) - acc[q1]) * rpv[k + 1];
      cl[(k + 1) & 1][i] = m1;
      mrow[q1] = m1;
    }
#pragma clang loop unroll(full)
    for (int q = 0; q < LQ; ++q) {
      const int r = 4 * q + W;
      if (r <= k + 1) continue;                   // finished, or published above
      acc[q] = __builtin_fma(S[r][k], mk, acc[q]);
    }
    __syncthreads();
  }
  if (i < bs) {                        // W^{-1}(j, r) = M(r, j): this wave's rows of M as columns
#pragma clang loop unroll(full)
    for (int q = 0; q < LQ; ++q) {
      const int r = 4 * q + W;
      if (r < bs) Wi[i + (int64_t)r * ldw] = mrow[q];
    }
  }
}

__device__ __forceinline__ void leaf_body(double* Z, int64_t ldz, double* Wi, int64_t ldw, int bs, int* flag) {
  __shared__ double S[NB][NB + 1];     // the input (S[i][j] = A(i, j), j <= i), then L
  __shared__ double cl[3][NB];         // column k of the factorisation / row k of M
  __shared__ double rpv[NB];           // 1 / L(k, k)
  const int w = threadIdx.x >> 6, i = threadIdx.x & 63;
  {   // coalesced load of Z's upper triangle, all loads in flight: wave w
      // loads the columns c = 4q + w; S[c][r] = Z(r, c) = A(c, r), r <= c
    double v[LQ];
#pragma clang loop unroll(full)
    for (int q = 0; q < LQ; ++q) {
      const int c = 4 * q + w;
      double x = (i == c) ? 1.0 : 0.0;
      if (c < bs && i <= c) x = Z[i + (int64_t)c * ldz];
      v[q] = x;
    }
#pragma clang loop unroll(full)
    for (int q = 0; q < LQ; ++q) S[4 * q + w][i] = v[q];
  }
  __syncthreads();
  switch (w) {
    case 0: leaf_wave<0>(Z, ldz, Wi, ldw, bs, flag, S, cl, rpv); break;
    case 1: leaf_wave<1>(Z, ldz, Wi, ldw, bs, flag, S, cl, rpv); break;
    case 2: leaf_wave<2>(Z, ldz, Wi, ldw, bs, flag, S, cl, rpv); break;
    default: leaf_wave<3>(Z, ldz, Wi, ldw, bs, flag, S, cl, rpv); break;
  }
}

__global__ __launch_bounds__(LW) void chol_inv_leaf(double* Z, int64_t ldz, double* Wi, int64_t ldw,
                                                    int bs, int* flag) {
  leaf_body(Z, ldz, Wi, ldw, bs, flag);
}

// The diagonal leaves of up to LEAF_CHUNK matrices of a batch, one workgroup each.
constexpr int LEAF_CHUNK = 32;
struct LeafDesc { double* Z; int64_t ldz; double* Wi; int64_t ldw; int* flag; int bs; };
struct LeafChunk { LeafDesc d[LEAF_CHUNK]; };
__global__ __launch_bounds__(LW) void chol_inv_leaf_batched(LeafChunk c) {
  const LeafDesc d = c.d[blockIdx.x];
  leaf_body(d.Z, d.ldz, d.Wi, d.ldw, d.bs, d.flag);
}

// dst (rows x cols, ldd) = src (ld lds) for up to LEAF_CHUNK matrices.
struct CopyDesc { const double* src; int64_t lds; double* dst; int64_t ldd; int64_t rows, cols; };
struct CopyChunk { CopyDesc d[LEAF_CHUNK]; };
__global__ void copy_batched_kernel(CopyChunk c) {
  const CopyDesc d = c.d[blockIdx.y];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t q = e; q < d.rows * d.cols; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = q % d.rows, col = q / d.rows;
    d.dst[r + col * d.ldd] = d.src[r + col * d.lds];
  }
}

// The recursion's bottom node (m <= 2 NB rows: n1 = NB, n2 = m - NB <= NB)
// in two one-workgroup kernels instead of four GEMMs and a copy:
//   node_pre  (after the first leaf):  W12 = W11^{-T} Z12 (into Z12) and
//             Z22 <- Z22 - W12^T W12 (upper triangle);
//   node_post (after the second leaf): W^{-1}_{12} = -W11^{-1} (W12 W22^{-1}).
// The blocks sit in LDS, zero outside their triangles and past n2, and each
// 64 x 64 product runs on the FP64 matrix cores (wave w owns output column
// block 16 w, four 16 x 16 tiles, 16 k steps of 4).  The batched recursion
// runs the same kernels over its members, so both give the same bits.
struct NodeDesc { double* Z; int64_t ldz; double* Wi; int64_t ldw; int n2; };
struct NodeChunk { NodeDesc d[LEAF_CHUNK]; };
constexpr int NL = NB + 1;   // LDS row pitch

// All of a block's loads are issued before the first LDS store (one memory
// latency instead of one per pass).
__device__ __forceinline__ void load_block(double (*D)[NL], const double* src, int64_t ld, int rows, int cols,
                                           bool upper) {
  constexpr int PER = NB * NB / LW;
  double v[PER];
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * LW, r = e % NB, c = e / NB;
    v[p] = (r < rows && c < cols && (!upper || r <= c)) ? src[r + (int64_t)c * ld] : 0.0;
  }
#pragma unroll
  for (int p = 0; p < PER; ++p) {
    const int e = threadIdx.x + p * LW;
    D[e % NB][e / NB] = v[p];
  }
}

// acc[b] = tile (16 b, 16 w) of op(A) B for 64 x 64 LDS blocks (op = transpose
// when ta); element r of lane l is row 16 b + l / 16 + 4 r, column
// 16 w + l % 16 (the v_mfma_f64_16x16x4f64 result layout).
__device__ __forceinline__ void mm64(const double (*A)[NL], bool ta, const double (*B)[NL], v4d acc[4]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4, bj = 16 * w;
#pragma unroll
  for (int b = 0; b < 4; ++b) acc[b] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < NB; k0 += 4) {
    const int k = k0 + lk;
    const double bv = B[k][bj + li];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const double av = ta ? A[k][16 * b + li] : A[16 * b + li][k];
      acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[b], 0, 0, 0);
    }
  }
}

__global__ __launch_bounds__(LW) void node_pre_kernel(NodeChunk ch) {
  __shared__ double A[NB][NL];   // W11^{-1} (upper)
  __shared__ double B[NB][NL];   // Z12, then W12
  const NodeDesc d = ch.d[blockIdx.x];
  const int n2 = d.n2, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = 16 * w + (lane & 15), rq = lane >> 4;
  load_block(A, d.Wi, d.ldw, NB, NB, true);
  load_block(B, d.Z + (int64_t)NB * d.ldz, d.ldz, NB, n2, false);
  __syncthreads();
  v4d acc[4];
  mm64(A, true, B, acc);                    // W12 = W11^{-T} Z12
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * b + rq + 4 * r;
      B[row][col] = acc[b][r];
      if (col < n2) d.Z[row + (int64_t)(NB + col) * d.ldz] = acc[b][r];
    }
  __syncthreads();
  mm64(B, true, B, acc);                    // W12^T W12
  double* Z22 = d.Z + NB + (int64_t)NB * d.ldz;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * b + rq + 4 * r;
      if (row <= col && col < n2) Z22[row + (int64_t)col * d.ldz] -= acc[b][r];
    }
}

__global__ __launch_bounds__(LW) void node_post_kernel(NodeChunk ch) {
  __shared__ double A[NB][NL];   // W11^{-1} (upper)
  __shared__ double B[NB][NL];   // W12, then W12 W22^{-1}
  __shared__ double C[NB][NL];   // W22^{-1} (upper)
  const NodeDesc d = ch.d[blockIdx.x];
  const int n2 = d.n2, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int col = 16 * w + (lane & 15), rq = lane >> 4;
  load_block(A, d.Wi, d.ldw, NB, NB, true);
  load_block(B, d.Z + (int64_t)NB * d.ldz, d.ldz, NB, n2, false);
  load_block(C, d.Wi + NB + (int64_t)NB * d.ldw, d.ldw, n2, n2, true);
  __syncthreads();
  v4d acc[4];
  mm64(B, false, C, acc);                   // X = W12 W22^{-1}
  __syncthreads();
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r) B[16 * b + rq + 4 * r][col] = acc[b][r];
  __syncthreads();
  mm64(A, false, B, acc);                   // W11^{-1} X
  double* W12i = d.Wi + (int64_t)NB * d.ldw;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (col < n2) W12i[(16 * b + rq + 4 * r) + (int64_t)col * d.ldw] = -acc[b][r];
}

struct Rec {
  double* Z; int64_t ldz; double* Wi; int64_t ldw; double* T; int* flag; hipStream_t s;

  void run(int64_t o, int64_t m) {
    double* Zo = Z + o + o * ldz;
    double* Wo = Wi + o + o * ldw;
    if (m <= NB) {
      chol_inv_leaf<<<1, LW, 0, s>>>(Zo, ldz, Wo, ldw, (int)m, flag);
      QDWHP_LAUNCH_CHECK();
      return;
    }
    if (m <= 2 * NB) {           // bottom node: leaf, pre, leaf, post
      NodeChunk nc;
      nc.d[0] = NodeDesc{Zo, ldz, Wo, ldw, (int)(m - NB)};
      run(o, NB);
      node_pre_kernel<<<1, LW, 0, s>>>(nc);
      QDWHP_LAUNCH_CHECK();
      run(o + NB, m - NB);
      node_post_kernel<<<1, LW, 0, s>>>(nc);
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

// Largest n1 x n2 product buffer over every level of the recursion on m
// rows: a lopsided split (n2 much smaller than n1, e.g. m = 2 NB + 1) needs
// less at the top than its first half needs one level down.
static int64_t rec_t_doubles(int64_t m) {
  if (m <= 2 * NB) return 0;     // leaves and fused bottom nodes
  const int64_t n1 = NB * cdiv(cdiv(m, NB), 2), n2 = m - n1;
  return std::max(n1 * n2, std::max(rec_t_doubles(n1), rec_t_doubles(n2)));
}

int64_t spd_inverse_doubles(int64_t n) {
  return n * n + std::max<int64_t>(rec_t_doubles(n), 1) + 64;
}

void chol_inverse_factor(double* Z, int64_t n, int64_t ldz, double* work, int* flag, hipStream_t s) {
  if (n <= 0) return;
  double* Wi = work;
  double* T = work + n * n;
  fill(Wi, n, n, n, 0.0, 0.0, s);
  Rec r{Z, ldz, Wi, n, T, flag, s};
  r.run(0, n);
}

namespace {

// chol_inverse_factor's recursion (Rec::run) for several matrices of one size
// at once: the same operations in the same order, each leaf one launch over
// the matrices (chunks of LEAF_CHUNK) and each product one grouped GEMM.
struct GroupRec {
  const CholItem* it; int count; int64_t n; void* table; hipStream_t s;
  std::vector<GroupedDesc> d;

  void run(int64_t o, int64_t m) {
    if (m <= NB) {
      for (int c0 = 0; c0 < count; c0 += LEAF_CHUNK) {
        LeafChunk lc;
        const int cnt = std::min(LEAF_CHUNK, count - c0);
        for (int q = 0; q < cnt; ++q) {
          const CholItem& x = it[c0 + q];
          lc.d[q] = LeafDesc{x.Z + o + o * x.ldz, x.ldz, x.work + o + o * n, n, x.flag, (int)m};
        }
        chol_inv_leaf_batched<<<cnt, LW, 0, s>>>(lc);
        QDWHP_LAUNCH_CHECK();
      }
      return;
    }
    if (m <= 2 * NB) {           // bottom node: the standalone recursion's kernels, per member
      auto node = [&](bool pre) {
        for (int c0 = 0; c0 < count; c0 += LEAF_CHUNK) {
          NodeChunk nc;
          const int cnt = std::min(LEAF_CHUNK, count - c0);
          for (int q = 0; q < cnt; ++q) {
            const CholItem& x = it[c0 + q];
            nc.d[q] = NodeDesc{x.Z + o + o * x.ldz, x.ldz, x.work + o + o * n, n, (int)(m - NB)};
          }
          if (pre) node_pre_kernel<<<cnt, LW, 0, s>>>(nc);
          else node_post_kernel<<<cnt, LW, 0, s>>>(nc);
          QDWHP_LAUNCH_CHECK();
        }
      };
      run(o, NB);
      node(true);
      run(o + NB, m - NB);
      node(false);
      return;
    }
    const int64_t nblk = cdiv(m, NB);
    const int64_t n1 = NB * cdiv(nblk, 2), n2 = m - n1;
    run(o, n1);
    auto each = [&](auto make) {
      d.clear();
      for (int q = 0; q < count; ++q) d.push_back(make(it[q]));
    };
    // T = W11^{-T} Z12
    each([&](const CholItem& x) {
      GroupedDesc g{n1, n2, n1, 1.0, 0.0, x.work + o + o * n, n, x.Z + o + (o + n1) * x.ldz, x.ldz,
                    x.work + n * n, n1};
      g.khi = KHI_ROW;
      return g;
    });
    dgemm_grouped(d.data(), count, true, false, table, s);
    for (int c0 = 0; c0 < count; c0 += LEAF_CHUNK) {   // Z12 <- W12
      CopyChunk cc;
      const int cnt = std::min(LEAF_CHUNK, count - c0);
      for (int q = 0; q < cnt; ++q) {
        const CholItem& x = it[c0 + q];
        cc.d[q] = CopyDesc{x.work + n * n, n1, x.Z + o + (o + n1) * x.ldz, x.ldz, n1, n2};
      }
      copy_batched_kernel<<<dim3((unsigned)std::min<int64_t>(cdiv(n1 * n2, 256), 1024), cnt), 256, 0, s>>>(cc);
      QDWHP_LAUNCH_CHECK();
    }
    // Z22 <- Z22 - W12^T W12 (upper tiles)
    each([&](const CholItem& x) {
      GroupedDesc g{n2, n2, n1, -1.0, 1.0, x.Z + o + (o + n1) * x.ldz, x.ldz, x.Z + o + (o + n1) * x.ldz, x.ldz,
                    x.Z + (o + n1) + (o + n1) * x.ldz, x.ldz};
      g.tiles = TILES_UPPER;
      return g;
    });
    dgemm_grouped(d.data(), count, true, false, table, s);
    run(o + n1, n2);
    // T = W12 W22^{-1}
    each([&](const CholItem& x) {
      GroupedDesc g{n1, n2, n2, 1.0, 0.0, x.Z + o + (o + n1) * x.ldz, x.ldz, x.work + (o + n1) + (o + n1) * n, n,
                    x.work + n * n, n1};
      g.khi = KHI_COL;
      return g;
    });
    dgemm_grouped(d.data(), count, false, false, table, s);
    // W^{-1}_{12} = -W11^{-1} T
    each([&](const CholItem& x) {
      GroupedDesc g{n1, n2, n1, -1.0, 0.0, x.work + o + o * n, n, x.work + n * n, n1, x.work + o + (o + n1) * n, n};
      g.klo = KLO_ROW;
      return g;
    });
    dgemm_grouped(d.data(), count, false, false, table, s);
  }
};

}  // namespace

void chol_inverse_grouped(const CholItem* items, int count, int64_t n, void* table, hipStream_t s) {
  if (count <= 0 || n <= 0) return;
  for (int q = 0; q < count; ++q) fill(items[q].work, n, n, n, 0.0, 0.0, s);
  GroupRec r{items, count, n, table, s, {}};
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
