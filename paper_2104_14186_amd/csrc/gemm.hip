// FP64 MFMA GEMM for gfx950: C = alpha op(A) op(B) + beta C (+ diag I).
//
// Result layout of v_mfma_f64_16x16x4f64 (checked on gfx950): lane l, element r
// holds D[l/16 + 4r][l%16]; operands A[l%16][l/16] and B[l/16][l%16].
// v_mfma_f32_16x16x4f32 (the mixed-precision variant) takes the same operand
// layout but holds D[4(l/16) + r][l%16].
//
// Mixed precision (Gemm::f32): operands are rounded to FP32 when staged into
// LDS, or (Gemm::in32) are FP32 copies in HBM read at half the bytes;
// products accumulate in FP32 on the FP32 matrix cores (twice the FP64 rate),
// folded into FP64 every 32 k; alpha, beta, the C term and the diagonal shift
// are applied in FP64.
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

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"

namespace qdwhp {
namespace {

constexpr int BM = 128, BN = 128, BK = 16;
constexpr int PAD = 4;
constexpr int SA = BM + PAD;   // LDS row stride (elements) of the k-major A slice
constexpr int SB = BN + PAD;
constexpr int NLD = BM * BK / 256;   // elements of each operand slice loaded per thread (8)
constexpr int GM = 8;                // tile rows per group of the launch order

typedef float v4f __attribute__((ext_vector_type(4)));

template <bool F32> struct MfmaT;
template <> struct MfmaT<false> {
  typedef double elem; typedef v4d acc;
  static __device__ inline acc op(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int r) { return lk + 4 * r; }
};
template <> struct MfmaT<true> {
  typedef float elem; typedef v4f acc;
  static __device__ inline acc op(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int row(int lk, int r) { return 4 * lk + r; }
};

// Launch order.  The hardware deals consecutive workgroups round-robin to the
// 8 XCDs (each with its own L2); the linear id is remapped so each XCD gets a
// contiguous range of the tile list.  Full launches walk groups of GM tile
// rows column by column (workgroups resident together share A and B slices);
// upper-triangle launches enumerate exactly the tiles with tm <= tn, column by
// column, so every XCD gets the same number of tiles.  When the K range of an
// upper-triangle launch follows the tile column (order != 0), the tiles'
// work grows or shrinks along that enumeration and contiguous ranges would
// give the first XCD many times the work of the last: such launches deal
// the tiles round-robin in order of decreasing work instead (even shares
// per XCD, light tiles last).  Full launches whose K range follows the tile
// row (row groups are contiguous in the enumeration) are dealt the same way.
__device__ inline int64_t xcd_remap(int64_t w, int64_t W) {
  const int64_t q = W / 8, r = W % 8, xcd = w % 8, loc = w / 8;
  return (xcd < r) ? xcd * (q + 1) + loc : r * (q + 1) + (xcd - r) * q + loc;
}
__device__ inline void tile_of(int64_t w, int64_t gx, int64_t gy, bool upper, int order, int64_t* tm,
                               int64_t* tn) {
  if (upper) {
    const int64_t W = gx * (gx + 1) / 2;
    const int64_t L = (order == 0) ? xcd_remap(w, W) : (order > 0 ? w : W - 1 - w);
    int64_t c = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) / 2.0);
    while (c * (c + 1) / 2 > L) --c;
    while ((c + 1) * (c + 2) / 2 <= L) ++c;
    *tn = c;
    *tm = L - c * (c + 1) / 2;
    return;
  }
  const int64_t L = (order == 0) ? xcd_remap(w, gx * gy) : (order > 0 ? w : gx * gy - 1 - w);
  const int64_t per = (int64_t)GM * gy;
  const int64_t grp = L / per, first = grp * GM;
  const int64_t gm = (gx - first < GM) ? gx - first : GM;
  const int64_t in = L % per;
  *tm = first + in % gm;
  *tn = in / gm;
}

// One BT x BT output tile (tm, tn) of problem g (BT = 128 or 64); zi is the batch index, or
// the K share when g.splitk > 1.  As / Bs are the workgroup's LDS buffers.
template <bool TA, bool TB, bool F32, int BT, bool IN32 = false>
__device__ __forceinline__ void gemm_tile(const Gemm& g, int64_t tm, int64_t tn, int64_t zi,
                                          typename MfmaT<F32>::elem (*As)[BK * (BT + PAD)],
                                          typename MfmaT<F32>::elem (*Bs)[BK * (BT + PAD)]) {
  // tile geometry: 2x2 waves, each owning a (BT/2)^2 block of WT x WT MFMA tiles
  constexpr int TM = BT, TN = BT, TSA = BT + PAD, TSB = BT + PAD;
  constexpr int TNLD = BT * BK / 256;   // operand elements loaded per thread per slice
  constexpr int WT = BT / 32, HALF = BT / 2;
  constexpr int KS = 256 / BT;          // k rows covered by one pass of a k-major load
  typedef typename MfmaT<F32>::elem E;
  typedef typename MfmaT<F32>::acc ACC;

  const int tid = threadIdx.x;
  const int64_t row0 = tm * TM;
  const int64_t col0 = tn * TN;
  const bool split = g.splitk > 1;
  const int64_t bz = split ? 0 : zi;
  constexpr int ES = IN32 ? 4 : 8;      // bytes per stored operand element
  const char* __restrict__ A = (const char*)g.A + bz * g.sA * ES;
  const char* __restrict__ B = (const char*)g.B + bz * g.sB * ES;
  double* C = g.C + bz * g.sC;
  const double* Cin = g.Cin ? g.Cin + bz * g.sCin : C;
  const int64_t ldcin = g.Cin ? g.ldcin : g.ldc;
  const int64_t M = g.M, N = g.N;
  const bool aul = g.a_unit_lower, bul = g.b_unit_lower;
  const int64_t lda = g.lda, ldb = g.ldb;

  int64_t klo = 0, khi = g.K;
  if (g.klo == KLO_ROW) klo = row0 - g.koff;
  else if (g.klo == KLO_COL) klo = col0 - g.koff;
  if (g.khi == KHI_ROW) khi = row0 + TM - g.koff;
  else if (g.khi == KHI_COL) khi = col0 + TN - g.koff;
  if (klo < 0) klo = 0;
  if (khi > g.K) khi = g.K;
  if (split) {   // this workgroup's share of K, in whole BK slices
    const int64_t kc = ((g.K + g.splitk - 1) / g.splitk + BK - 1) / BK * BK;
    const int64_t z = zi;
    if (klo < z * kc) klo = z * kc;
    if (khi > (z + 1) * kc) khi = (z + 1) * kc;
  }
  // slices that need no bounds or structure masks use straight-line loads:
  // the tile lies inside C, the slice inside [klo, khi), and a unit-lower
  // operand's slice lies strictly below its diagonal (stored row > stored
  // column for every element), which for Householder vectors is all but
  // the slices that meet the top block
  const bool interior = row0 + TM <= M && col0 + TN <= N;
  auto mask_free = [&](int64_t k0) {
    const bool af = !aul || (TA ? k0 >= row0 + TM : row0 >= k0 + BK);
    const bool bf = !bul || (TB ? col0 >= k0 + BK : k0 >= col0 + TN);
    return af && bf;
  };

  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  const int li = lane & 15, lk = lane >> 4;

  // Operand slices are read with buffer loads: the 128-bit resource (scalar
  // registers) points at the slice's corner and each thread keeps one 32-bit
  // byte offset per element it loads.  Offsets at or beyond OOB read as zero,
  // which is how bounds, K ranges and structure masks are applied.
  //   A (m, k):  !TA: stored A[m + k lda] (thread: m = am, k = ak + KS r)
  //               TA: stored A[k + m lda] (thread: m = am + 16r, k = ak)
  //   B (k, n):  !TB: stored B[k + n ldb] (thread: n = bn + 16r, k = bk)
  //               TB: stored B[n + k ldb] (thread: n = bn, k = bk + KS r)
  const int am = TA ? (tid >> 4) : (tid & (BT - 1));
  const int ak = TA ? (tid & 15) : (tid / BT);
  const int bn = TB ? (tid & (BT - 1)) : (tid >> 4);
  const int bk = TB ? (tid / BT) : (tid & 15);
  constexpr uint32_t OOB = 0x80000000u, RECORDS = 0x7ffffff8u;
  uint32_t aoff[TNLD], boff[TNLD];
#pragma unroll
  for (int r = 0; r < TNLD; ++r) {
    aoff[r] = TA ? (uint32_t)((ak + (int64_t)(am + 16 * r) * lda) * ES)
                 : (uint32_t)((am + (int64_t)(ak + KS * r) * lda) * ES);
    boff[r] = TB ? (uint32_t)((bn + (int64_t)(bk + KS * r) * ldb) * ES)
                 : (uint32_t)((bk + (int64_t)(bn + 16 * r) * ldb) * ES);
  }
  auto slice_a = [&](int64_t k0) {
    const char* p = A + (TA ? row0 * lda + k0 : k0 * lda + row0) * ES;
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)RECORDS, 0x00020000);
  };
  auto slice_b = [&](int64_t k0) {
    const char* p = B + (TB ? k0 * ldb + col0 : col0 * ldb + k0) * ES;
    return __builtin_amdgcn_make_buffer_rsrc((void*)p, (short)0, (int)RECORDS, 0x00020000);
  };
  auto ld = [](__amdgpu_buffer_rsrc_t rs, uint32_t off) -> E {
    if constexpr (IN32)
      return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0));
    else
      return (E)__builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0));
  };

  ACC acc[WT][WT];
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j) acc[i][j] = ACC{0, 0, 0, 0};
  double acc64[F32 ? WT : 1][F32 ? WT : 1][4];   // FP32 path: slice sums added here in FP64
  if constexpr (F32) {
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
  }

  E ra[TNLD], rb[TNLD];

  auto load = [&](int64_t k0) {
    const __amdgpu_buffer_rsrc_t rsa = slice_a(k0), rsb = slice_b(k0);
    if (interior && k0 + BK <= khi && mask_free(k0)) {
#pragma unroll
      for (int r = 0; r < TNLD; ++r) ra[r] = ld(rsa, aoff[r]);
#pragma unroll
      for (int r = 0; r < TNLD; ++r) rb[r] = ld(rsb, boff[r]);
      return;
    }
#pragma unroll
    for (int r = 0; r < TNLD; ++r) {
      const int64_t m = row0 + am + (TA ? 16 * r : 0), k = k0 + ak + (TA ? 0 : KS * r);
      const int64_t sr = TA ? k : m, sc = TA ? m : k;   // stored (row, col)
      const bool in = m < M && k >= klo && k < khi;
      const bool take = in && (!aul || sr > sc);
      E v = ld(rsa, take ? aoff[r] : OOB);
      if (aul && in && sr == sc) v = (E)1.0;
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < TNLD; ++r) {
      const int64_t n = col0 + bn + (TB ? 0 : 16 * r), k = k0 + bk + (TB ? KS * r : 0);
      const int64_t sr = TB ? n : k, sc = TB ? k : n;
      const bool in = n < N && k >= klo && k < khi;
      const bool take = in && (!bul || sr > sc);
      E v = ld(rsb, take ? boff[r] : OOB);
      if (bul && in && sr == sc) v = (E)1.0;
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < TNLD; ++r)
      As[buf][(ak + (TA ? 0 : KS * r)) * TSA + am + (TA ? 16 * r : 0)] = ra[r];
#pragma unroll
    for (int r = 0; r < TNLD; ++r)
      Bs[buf][(bk + (TB ? KS * r : 0)) * TSB + bn + (TB ? 0 : 16 * r)] = rb[r];
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
      const E* as = As[cur];
      const E* bs = Bs[cur];
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        E a[WT], b[WT];
#pragma unroll
        for (int i = 0; i < WT; ++i) a[i] = as[(kk + lk) * TSA + wm * HALF + i * 16 + li];
#pragma unroll
        for (int j = 0; j < WT; ++j) b[j] = bs[(kk + lk) * TSB + wn * HALF + j * 16 + li];
#pragma unroll
        for (int i = 0; i < WT; ++i)
#pragma unroll
          for (int j = 0; j < WT; ++j)
            acc[i][j] = MfmaT<F32>::op(a[i], b[j], acc[i][j]);
      }
      if constexpr (F32) {
        if ((t & 1) || !more) {   // every 32 k: fold the FP32 sums into FP64
#pragma unroll
          for (int i = 0; i < WT; ++i)
#pragma unroll
            for (int j = 0; j < WT; ++j)
#pragma unroll
              for (int r = 0; r < 4; ++r) { acc64[i][j][r] += (double)acc[i][j][r]; acc[i][j][r] = 0.0f; }
        }
      }
      if (more) store(cur ^ 1);
      __syncthreads();
    }
  }

  auto result = [&](int i, int j, int r) -> double {
    if constexpr (F32) return acc64[i][j][r];
    else return acc[i][j][r];
  };
  const double alpha = (g.dscal && g.ia >= 0) ? g.dscal[g.ia] : g.alpha;
  const double beta = (g.dscal && g.ib >= 0) ? g.dscal[g.ib] : g.beta;
  const double dg = g.diag;
  if (split) {   // raw partial product of this K share
    double* P = g.ws + zi * M * N;
#pragma unroll
    for (int i = 0; i < WT; ++i)
#pragma unroll
      for (int j = 0; j < WT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t row = row0 + wm * HALF + i * 16 + MfmaT<F32>::row(lk, r);
          const int64_t col = col0 + wn * HALF + j * 16 + li;
          if (row < M && col < N) P[row + col * M] = result(i, j, r);
        }
    return;
  }
#pragma unroll
  for (int i = 0; i < WT; ++i)
#pragma unroll
    for (int j = 0; j < WT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = row0 + wm * HALF + i * 16 + MfmaT<F32>::row(lk, r);
        const int64_t col = col0 + wn * HALF + j * 16 + li;
        if (row < M && col < N) {
          double* p = C + row + col * g.ldc;
          double v = alpha * result(i, j, r);
          if (beta != 0.0) v += beta * Cin[row + col * ldcin];
          if (dg != 0.0 && row == col) v += dg;
          *p = v;
        }
      }
}

template <bool TA, bool TB, bool F32, int BT, bool IN32 = false>
__global__ __launch_bounds__(256, (F32 && BT == 128) ? 1 : 2) void dgemm_kernel(Gemm g, int64_t gx, int64_t gy) {
  __shared__ typename MfmaT<F32>::elem As[2][BK * (BT + PAD)];
  __shared__ typename MfmaT<F32>::elem Bs[2][BK * (BT + PAD)];
  int64_t tm, tn;
  // upper launches: k >= tile column puts the work in early columns, k < column
  // end in late ones; full launches: the same along rows (their enumeration
  // walks row groups), and k < column end puts it at the end of every row
  // group (reversed, the heavy tiles go first and the light ones fill the tail)
  const int order = (g.tiles == TILES_UPPER)
                        ? ((g.klo == KLO_COL) ? 1 : (g.khi == KHI_COL ? -1 : 0))
                        : ((g.klo == KLO_ROW) ? 1 : ((g.khi == KHI_ROW || g.khi == KHI_COL) ? -1 : 0));
  tile_of(blockIdx.x, gx, gy, g.tiles == TILES_UPPER, order, &tm, &tn);
  gemm_tile<TA, TB, F32, BT, IN32>(g, tm, tn, blockIdx.z, As, Bs);
}

// Persistent launch over a ragged list of FP64 problems (same transposes):
// tile t of the concatenated tile list belongs to the problem p with
// first[p] <= t < first[p + 1]; its tiles are numbered column by column.
// Each tile is computed exactly as by dgemm_kernel.
template <bool TA, bool TB>
__global__ __launch_bounds__(256, 2) void dgemm_grouped_kernel(const GroupedDesc* descs, const int64_t* first,
                                                               int count) {
  __shared__ double As[2][BK * SA];
  __shared__ double Bs[2][BK * SB];
  const int64_t total = first[count];
  for (int64_t t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (first[mid] <= t) lo = mid; else hi = mid - 1;
    }
    const GroupedDesc d = descs[lo];
    Gemm g;
    g.M = d.M; g.N = d.N; g.K = d.K; g.alpha = d.alpha; g.beta = d.beta;
    g.A = d.A; g.lda = d.lda; g.ta = TA; g.B = d.B; g.ldb = d.ldb; g.tb = TB; g.C = d.C; g.ldc = d.ldc;
    g.diag = d.diag; g.Cin = d.Cin; g.ldcin = d.ldcin; g.klo = d.klo; g.khi = d.khi; g.tiles = d.tiles;
    const int64_t local = t - first[lo];
    const int64_t gx = (g.M + BM - 1) / BM;
    int64_t tm = local % gx, tn = local / gx;
    if (d.tiles == TILES_UPPER) {   // column c holds tiles 0..c: local = c (c + 1) / 2 + tm
      int64_t c = (int64_t)((sqrt(8.0 * (double)local + 1.0) - 1.0) / 2.0);
      while (c * (c + 1) / 2 > local) --c;
      while ((c + 1) * (c + 2) / 2 <= local) ++c;
      tn = c;
      tm = local - c * (c + 1) / 2;
    }
    gemm_tile<TA, TB, false, 128>(g, tm, tn, 0, As, Bs);
    __syncthreads();
  }
}

// The descriptor table travels in kernel arguments (no host staging buffer
// whose lifetime would outlast the call): DESC_CHUNK entries per launch.
constexpr int DESC_CHUNK = 24;
struct DescChunk {
  GroupedDesc d[DESC_CHUNK];
  int64_t first[DESC_CHUNK + 1];
  int count, base;
};

__global__ void desc_write_kernel(GroupedDesc* table, int64_t* first, DescChunk c, int total_count) {
  const int i = threadIdx.x;
  if (i < c.count) {
    table[c.base + i] = c.d[i];
    first[c.base + i] = c.first[i];
  }
  if (i == 0 && c.base + c.count == total_count) first[total_count] = c.first[c.count];
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
    const double alpha = (g.dscal && g.ia >= 0) ? g.dscal[g.ia] : g.alpha;
    const double beta = (g.dscal && g.ib >= 0) ? g.dscal[g.ib] : g.beta;
    double v = alpha * acc;
    if (beta != 0.0) v += beta * Cin[i + j * ldcin];
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

template <int BT>
static void launch_tiles(const Gemm& g, int64_t tm, int64_t tn, hipStream_t s) {
  const int64_t ntile = (g.tiles == TILES_UPPER) ? tm * (tm + 1) / 2 : tm * tn;
  dim3 grid((unsigned)ntile, 1, (unsigned)(g.splitk > 1 ? g.splitk : g.batch));
  dim3 block(256);
  if (!g.f32) {
    if (!g.ta && !g.tb) dgemm_kernel<false, false, false, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else if (!g.ta && g.tb) dgemm_kernel<false, true, false, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else if (g.ta && !g.tb) dgemm_kernel<true, false, false, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else dgemm_kernel<true, true, false, BT><<<grid, block, 0, s>>>(g, tm, tn);
  } else if (!g.in32) {
    if (!g.ta && !g.tb) dgemm_kernel<false, false, true, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else if (!g.ta && g.tb) dgemm_kernel<false, true, true, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else if (g.ta && !g.tb) dgemm_kernel<true, false, true, BT><<<grid, block, 0, s>>>(g, tm, tn);
    else dgemm_kernel<true, true, true, BT><<<grid, block, 0, s>>>(g, tm, tn);
  } else {
    if (!g.ta && !g.tb) dgemm_kernel<false, false, true, BT, true><<<grid, block, 0, s>>>(g, tm, tn);
    else if (!g.ta && g.tb) dgemm_kernel<false, true, true, BT, true><<<grid, block, 0, s>>>(g, tm, tn);
    else if (g.ta && !g.tb) dgemm_kernel<true, false, true, BT, true><<<grid, block, 0, s>>>(g, tm, tn);
    else dgemm_kernel<true, true, true, BT, true><<<grid, block, 0, s>>>(g, tm, tn);
  }
}

void dgemm(const Gemm& g0, hipStream_t s) {
  if (g0.M <= 0 || g0.N <= 0 || g0.batch <= 0) return;
  void* tok = nullptr;
  const bool prof = prof_active();
  if (prof) prof_begin_launch(s, &tok);
  Gemm g = g0;
  g.splitk = 1;
  int64_t tm = cdiv(g.M, BM), tn = cdiv(g.N, BN);
  if (g.tiles == TILES_UPPER && tm != tn)
    throw HipError{hipErrorInvalidValue};   // upper-tile output must be square
  // every per-thread byte offset inside an operand slice must fit in 31 bits
  if ((g.lda > 0 && g.lda >= (int64_t(1) << 21)) || (g.ldb > 0 && g.ldb >= (int64_t(1) << 21)))
    throw HipError{hipErrorInvalidValue};   // leading dimension too large
  const int64_t tiles = ((g.tiles == TILES_UPPER) ? tm * (tm + 1) / 2 : tm * tn) * g.batch;
  if (g.batch == 1 && g.ws && g.tiles == TILES_ALL && tiles < 160 && g.K >= 4 * BK * 8) {
    // as many K shares as fill the chip's 512 resident workgroups (two per CU) in one pass
    int64_t S = 512 / tiles;
    const int64_t kmax = g.K / (BK * 8);
    if (S > kmax) S = kmax;
    const int64_t cap = g.ws_doubles / (g.M * g.N);
    if (S > cap) S = cap;
    if (S > 64) S = 64;
    if (S >= 2) g.splitk = (int)S;
  }
  // Launches with few 128x128 tiles run 64x64 tiles (4x the workgroups), and
  // so do shallow ones (K <= 128, e.g. block-reflector updates), whose time
  // goes to reading and writing C: more, lighter workgroups keep more of it
  // in flight (2.3 -> 1.8 ms for a 16384 x 16256 x 128 update).  The
  // per-element k order is the same for both, so the results are identical.
  // FP32-operand launches always take 64x64 tiles: the 128-wide FP32 tile
  // carries FP64 fold registers that limit it to one workgroup per CU (18
  // against 72 TF/s for a 16384^3 Gram).
  if (g.f32 || (g.splitk == 1 && (tiles < qdwhp_tune_get("gemm.small_tiles", 96) ||
                                  g.K <= qdwhp_tune_get("gemm.shallow_k", 128)))) {
    tm = cdiv(g.M, 64); tn = cdiv(g.N, 64);
    launch_tiles<64>(g, tm, tn, s);
  } else {
    launch_tiles<128>(g, tm, tn, s);
  }
  QDWHP_LAUNCH_CHECK();
  if (g.splitk > 1) {
    dim3 rg((unsigned)cdiv(g.M, 256), (unsigned)(g.N < 65535 ? g.N : 65535));
    splitk_reduce<<<rg, 256, 0, s>>>(g);
    QDWHP_LAUNCH_CHECK();
  }
  if (prof) prof_end_launch(s, tok, g0.f32 ? 0.0 : gemm_flops(g0));
}

size_t grouped_table_bytes(int count) {
  const size_t d = ((size_t)(count > 0 ? count : 1) * sizeof(GroupedDesc) + 255) / 256 * 256;
  return d + ((size_t)(count + 1) * sizeof(int64_t) + 255) / 256 * 256;
}

void dgemm_grouped(const GroupedDesc* descs, int count, bool ta, bool tb, void* table, hipStream_t s) {
  if (count <= 0) return;
  GroupedDesc* dt = (GroupedDesc*)table;
  int64_t* first = (int64_t*)((char*)table + ((size_t)count * sizeof(GroupedDesc) + 255) / 256 * 256);
  int64_t run = 0;
  for (int base = 0; base < count; base += DESC_CHUNK) {
    DescChunk c;
    c.base = base;
    c.count = std::min(DESC_CHUNK, count - base);
    for (int i = 0; i < c.count; ++i) {
      const GroupedDesc& d = descs[base + i];
      if (d.lda >= (int64_t(1) << 21) || d.ldb >= (int64_t(1) << 21)) throw HipError{hipErrorInvalidValue};
      if (d.tiles == TILES_UPPER && d.M != d.N) throw HipError{hipErrorInvalidValue};
      c.d[i] = d;
      c.first[i] = run;
      if (d.M > 0 && d.N > 0)
        run += (d.tiles == TILES_UPPER) ? cdiv(d.M, BM) * (cdiv(d.M, BM) + 1) / 2 : cdiv(d.M, BM) * cdiv(d.N, BN);
    }
    c.first[c.count] = run;
    desc_write_kernel<<<1, 64, 0, s>>>(dt, first, c, count);
    QDWHP_LAUNCH_CHECK();
  }
  if (run == 0) return;
  void* tok = nullptr;
  const bool prof = prof_active();
  if (prof) prof_begin_launch(s, &tok);
  const unsigned grid = (unsigned)std::min<int64_t>(run, 512);
  if (!ta && !tb) dgemm_grouped_kernel<false, false><<<grid, 256, 0, s>>>(dt, first, count);
  else if (!ta && tb) dgemm_grouped_kernel<false, true><<<grid, 256, 0, s>>>(dt, first, count);
  else if (ta && !tb) dgemm_grouped_kernel<true, false><<<grid, 256, 0, s>>>(dt, first, count);
  else dgemm_grouped_kernel<true, true><<<grid, 256, 0, s>>>(dt, first, count);
  QDWHP_LAUNCH_CHECK();
  if (prof) {
    double fl = 0.0;
    for (int i = 0; i < count; ++i) fl += 2.0 * (double)descs[i].M * (double)descs[i].N * (double)descs[i].K;
    prof_end_launch(s, tok, fl);
  }
}

}  // namespace qdwhp
