// FP64 MFMA GEMM for gfx950: C = alpha op(A) op(B) + beta C (+ diag I).
//
// Result layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l, element r
// holds D[l/16 + 4r][l%16]; operands A[l%16][l/16] and B[l/16][l%16].
//
// Column-major operands.  One 256-thread workgroup (4 wave64s in a 2x2
// arrangement) owns a 128x128 tile of C; each wave accumulates a 64x64
// sub-tile as 4x4 blocks of v_mfma_f64_16x16x4f64.  K is consumed in slices
// of 16, staged k-major in LDS (double-buffered, one barrier per slice) so
// that the MFMA operand of every lane is a single conflict-free 8-byte read.
//
// Tile filtering (upper tiles only) and per-tile K ranges let the same kernel
// serve symmetric outputs (Gram, SYRK updates, the inverse of Z) and
// triangular operands (inverse and Cholesky factors) without touching the
// known-zero blocks.
#include <algorithm>

#include "common.h"

namespace qdwhp {
namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PAD = 4;
constexpr int SA = BM + PAD;   // LDS row stride (doubles) of the k-major A slice
constexpr int SB = BN + PAD;

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void dgemm_kernel(Gemm g) {
  __shared__ double As[2][BK * SA];
  __shared__ double Bs[2][BK * SB];

  const int tid = threadIdx.x;
  const int64_t row0 = (int64_t)blockIdx.x * BM;
  const int64_t col0 = (int64_t)blockIdx.y * BN;
  if (g.tiles == TILES_UPPER && row0 > col0 + BN - 1) return;
  const bool split = g.splitk > 1;
  const int64_t bz = split ? 0 : blockIdx.z;
  const double* __restrict__ A = g.A + bz * g.sA;
  const double* __restrict__ B = g.B + bz * g.sB;
  double* C = g.C + bz * g.sC;
  const double* Cin = g.Cin ? g.Cin + bz * g.sCin : C;
  const int64_t ldcin = g.Cin ? g.ldcin : g.ldc;
  const int64_t M = g.M, N = g.N;
  const bool aul = g.a_unit_lower, bul = g.b_unit_lower;

  int64_t klo = 0, khi = g.K;
  if (g.klo == KLO_ROW) klo = row0 - g.koff;
  else if (g.klo == KLO_COL) klo = col0 - g.koff;
  if (g.khi == KHI_ROW) khi = row0 + BM - g.koff;
  else if (g.khi == KHI_COL) khi = col0 + BN - g.koff;
  if (klo < 0) klo = 0;
  if (khi > g.K) khi = g.K;
  if (split) {   // this workgroup's share of K, in whole BK slices
    const int64_t kc = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    const int64_t z = blockIdx.z;
    if (klo < z * kc) klo = z * kc;
    if (khi > (z + 1) * kc) khi = (z + 1) * kc;
  }

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  double ra[8], rb[8];

  auto load = [&](int64_t k0) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int64_t m, k;
      if (!TA) { m = row0 + (tid & 127); k = k0 + (tid >> 7) + 2 * r; }
      else     { k = k0 + (tid & 15);    m = row0 + (tid >> 4) + 16 * r; }
      double v = 0.0;
      if (m < M && k < khi && k >= klo) {
        const int64_t sr = TA ? k : m, sc = TA ? m : k;   // stored (row, col)
        if (!aul || sr > sc) v = A[sr + sc * g.lda];
        else if (sr == sc) v = 1.0;
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int64_t n, k;
      if (TB) { n = col0 + (tid & 127); k = k0 + (tid >> 7) + 2 * r; }
      else    { k = k0 + (tid & 15);    n = col0 + (tid >> 4) + 16 * r; }
      double v = 0.0;
      if (n < N && k < khi && k >= klo) {
        const int64_t sr = TB ? n : k, sc = TB ? k : n;
        if (!bul || sr > sc) v = B[sr + sc * g.ldb];
        else if (sr == sc) v = 1.0;
      }
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int m, k;
      if (!TA) { m = tid & 127; k = (tid >> 7) + 2 * r; }
      else     { k = tid & 15;  m = (tid >> 4) + 16 * r; }
      As[buf][k * SA + m] = ra[r];
    }
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      int n, k;
      if (TB) { n = tid & 127; k = (tid >> 7) + 2 * r; }
      else    { k = tid & 15;  n = (tid >> 4) + 16 * r; }
      Bs[buf][k * SB + n] = rb[r];
    }
  };

  if (khi > klo) {
    const int64_t kbeg = klo;
    const int64_t nk = (khi - klo + BK - 1) / BK;
    load(kbeg);
    store(0);
    __syncthreads();
    for (int64_t t = 0; t < nk; ++t) {
      const int cur = (int)(t & 1);
      const bool more = (t + 1 < nk);
      if (more) load(kbeg + (t + 1) * BK);
      const double* as = As[cur];
      const double* bs = Bs[cur];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        double a[4], b[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) a[i] = as[(kk + lk) * SA + wm * 64 + i * 16 + li];
#pragma unroll
        for (int j = 0; j < 4; ++j) b[j] = bs[(kk + lk) * SB + wn * 64 + j * 16 + li];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
    }
  }

  const double alpha = g.alpha, beta = g.beta, dg = g.diag;
  if (split) {   // raw partial product of this K share
    double* P = g.ws + (int64_t)blockIdx.z * M * N;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + wm * 64 + i * 16 + lk + 4 * r;
          const int64_t col = col0 + wn * 64 + j * 16 + li;
          if (row < M && col < N) P[row + col * M] = acc[i][j][r];
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * 64 + i * 16 + lk + 4 * r;
        const int64_t col = col0 + wn * 64 + j * 16 + li;
        if (row < M && col < N) {
          double* p = C + row + col * g.ldc;
          double v = alpha * acc[i][j][r];
          if (beta != 0.0) v += beta * Cin[row + col * ldcin];
          if (dg != 0.0 && row == col) v += dg;
          *p = v;
        }
      }
}

// C = alpha * sum_z P_z + beta * Cin (+ diag), summed in a fixed order.
__global__ void splitk_reduce(Gemm g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = g.M, N = g.N;
  const double* Cin = g.Cin ? g.Cin : g.C;
  const int64_t ldcin = g.Cin ? g.ldcin : g.ldc;
  for (int64_t j = blockIdx.y; j < N; j += gridDim.y) {
    if (i >= M) continue;
    double acc = 0.0;
    for (int z = 0; z < g.splitk; ++z) acc += g.ws[(int64_t)z * M * N + i + j * M];
    double v = g.alpha * acc;
    if (g.beta != 0.0) v += g.beta * Cin[i + j * ldcin];
    if (g.diag != 0.0 && i == j) v += g.diag;
    g.C[i + j * g.ldc] = v;
  }
}

}  // namespace

// sum over i in [0, rows) of max(0, min(hi_i, K) - max(lo_i, 0)) where exactly
// one bound depends on the row: lo_i = i + d (row_lo) or hi_i = i + d (else).
static double row_sum(int64_t rows, int64_t fixed, int64_t d, bool row_lo, int64_t K) {
  double t = 0.0;
  if (!row_lo) {            // count_i = clip(i + d, 0, K) - lo, lo = max(fixed, 0)
    const int64_t lo = std::max<int64_t>(fixed, 0);
    if (lo >= K) return 0.0;
    const int64_t i0 = std::max<int64_t>(0, lo - d + 1);        // first i with i + d > lo
    const int64_t i1 = std::max<int64_t>(0, K - d);             // first i with i + d >= K
    const int64_t a = i0, b = std::min(rows, i1);
    if (b > a) t += (double)(b - a) * ((double)(a + b - 1) / 2.0 + (double)(d - lo));
    const int64_t c0 = std::max(i0, i1);
    if (rows > c0) t += (double)(rows - c0) * (double)(K - lo);
  } else {                  // count_i = hi - clip(i + d, 0, hi), hi = min(fixed, K)
    const int64_t hi = std::min<int64_t>(fixed, K);
    if (hi <= 0) return 0.0;
    const int64_t i0 = std::max<int64_t>(0, -d);                // first i with i + d >= 0
    const int64_t i1 = std::max<int64_t>(0, hi - d);            // first i with i + d >= hi
    const int64_t a = std::min(rows, i0);
    t += (double)a * (double)hi;                                // lo clipped to 0
    const int64_t b = std::min(rows, i1);
    if (b > a) t += (double)(b - a) * ((double)hi - (double)d - (double)(a + b - 1) / 2.0);
  }
  return t;
}

double gemm_flops(const Gemm& g) {
  // per output column j: rows i in [0, M) (or [0, min(M, j+1)) for upper output);
  // each (i, j) needs k in [lo(i, j), hi(i, j)) clipped to [0, K).
  double total = 0.0;
  const int64_t K = g.K;
  for (int64_t j = 0; j < g.N; ++j) {
    const int64_t rows = (g.tiles == TILES_UPPER) ? std::min<int64_t>(g.M, j + 1) : g.M;
    if (g.khi == KHI_ROW) {
      const int64_t lo = (g.klo == KLO_COL) ? j - g.koff : 0;
      total += row_sum(rows, lo, 1 - g.koff, false, K);
    } else if (g.klo == KLO_ROW) {
      const int64_t hi = (g.khi == KHI_COL) ? j + 1 - g.koff : K;
      total += row_sum(rows, hi, -g.koff, true, K);
    } else {
      int64_t lo = (g.klo == KLO_COL) ? j - g.koff : 0;
      int64_t hi = (g.khi == KHI_COL) ? j + 1 - g.koff : K;
      lo = std::max<int64_t>(lo, 0); hi = std::min<int64_t>(hi, K);
      if (hi > lo) total += (double)rows * (double)(hi - lo);
    }
  }
  return 2.0 * total * g.batch;
}

void dgemm(const Gemm& g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return;
  void* tok = nullptr;
  const bool prof = prof_active();
  if (prof) prof_begin_launch(s, &tok);
  Gemm g = g0;
  g.splitk = 1;
  const int64_t tm = cdiv(g.M, BM), tn = cdiv(g.N, BN);
  const int64_t tiles = tm * tn * g.batch;
  if (g.batch == 1 && g.ws && g.tiles == TILES_ALL && tiles < 160 && g.K >= 4 * BK * 8) {
    int64_t S = cdiv(320, tiles);
    const int64_t kmax = g.K / (BK * 8);
    if (S > kmax) S = kmax;
    const int64_t cap = g.ws_doubles / (g.M * g.N);
    if (S > cap) S = cap;
    if (S > 64) S = 64;
    if (S >= 2) g.splitk = (int)S;
  }
  dim3 grid((unsigned)tm, (unsigned)tn, (unsigned)(g.splitk > 1 ? g.splitk : g.batch));
  dim3 block(256);
  if (!g.ta && !g.tb) dgemm_kernel<false, false><<<grid, block, 0, s>>>(g);
  else if (!g.ta && g.tb) dgemm_kernel<false, true><<<grid, block, 0, s>>>(g);
  else if (g.ta && !g.tb) dgemm_kernel<true, false><<<grid, block, 0, s>>>(g);
  else dgemm_kernel<true, true><<<grid, block, 0, s>>>(g);
  QDWHP_LAUNCH_CHECK();
  if (g.splitk > 1) {
    dim3 rg((unsigned)cdiv(g.M, 256), (unsigned)(g.N < 65535 ? g.N : 65535));
    splitk_reduce<<<rg, 256, 0, s>>>(g);
    QDWHP_LAUNCH_CHECK();
  }
  if (prof) prof_end_launch(s, tok, gemm_flops(g0));
}

}  // namespace qdwhp
