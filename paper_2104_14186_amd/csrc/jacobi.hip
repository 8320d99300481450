// Parallel-order block Jacobi eigen/singular value solvers for the
// Rayleigh-Ritz step (Algorithm 1: eig of Q2^T A Q2; Algorithm 2: SVD of the
// R factor of A Q2).
//
// The index set is cut into blocks of JB = 16.  A sweep visits every pair of
// blocks once in round-robin (circle) order; in each step the Nb/2 disjoint
// pairs are independent:
//   * two-sided (symmetric H): the 32x32 diagonal sub-problem of each pair
//     gets one cyclic Jacobi sweep in LDS (16 disjoint rotations per round),
//     giving an orthogonal J; then H <- J^T H J tile by tile (tile
//     (P,Q) becomes J_P^T H_PQ J_Q; H is kept block-upper, so each
//     off-diagonal block is read and written once) and V <- V J;
//   * one-sided (R): each pair forms the Gram matrix of its 32 columns,
//     diagonalises it the same way and rotates the columns of R and V by J,
//     making them mutually orthogonal.
// Each block rotation J is re-orthonormalised by one Newton-Schulz step: the
// thousands of plane rotations inside one sub-problem leave J off orthogonal
// by a random walk of roundings, which would otherwise accumulate over the
// steps into the eigenvalues and residuals.
// Off-diagonal magnitudes seen at the start of each pair solve are max-reduced
// per sweep (an order-independent atomic max) and decide convergence.
#include <map>
#include <memory>
#include <mutex>
#include <vector>
#include "qdwhp.h"
#include "common.h"
#include "jacobi.h"

namespace qdwhp {
namespace {

// Inner sweeps per pair sub-problem.  One sweep per visit is enough: the
// outer sweeps converge in the same number of steps as when every 2JB x 2JB
// sub-problem is diagonalised to convergence, at a fraction of the cost.
#ifndef QDWHP_JACOBI_INNER
#define QDWHP_JACOBI_INNER 1
#endif

constexpr int P2 = 2 * JB;     // size of a pair sub-problem
constexpr int LDM = P2 + 1;
constexpr int NT = 256;        // threads of the pair / tile kernels
constexpr int ROT = P2 / 2;    // rotations per round

// Pair (p, q) of step `step` in the circle method over nb (even) players.
__device__ __host__ inline void round_robin(int nb, int step, int i, int* p, int* q) {
  const int m = nb - 1;
  int a, b;
  if (i == 0) { a = m; b = step % m; }
  else { a = (step + i) % m; b = (step - i + m) % m; }
  *p = a < b ? a : b;
  *q = a < b ? b : a;
}

__device__ inline void atomic_max_nonneg(double* addr, double v) {
  atomicMax((unsigned long long*)addr, (unsigned long long)__double_as_longlong(v));
}

// Cyclic Jacobi on the P2 x P2 symmetric M (LDS), accumulating J (LDS, starts
// as identity), with NT threads.  A rotation is skipped when |m_pq| <= tol
// (abs) or <= tol * sqrt(m_pp m_qq) (relative).  The ROT rotations of a round
// are disjoint, so they cut M into ROT x ROT blocks of 2 x 2 (row pair x column
// pair): one thread owns one block and applies the row rotation then the
// column rotation to it (the same order of operations as a full row pass
// followed by a full column pass), and rotates the matching 2 x 2 block of J.
// No thread reads what another writes within a round, so a round takes two
// barriers: after the rotations are formed and after they are applied.
static_assert(NT == ROT * ROT, "one thread per 2x2 block of a round");
__device__ int inner_jacobi(double (*M)[LDM], double (*J)[LDM], double tol, bool relative,
                            int max_sweeps) {
  __shared__ double cs[ROT][2];
  __shared__ int any;
  const int t = threadIdx.x;
  const int kr = t / ROT, kc = t % ROT;   // row pair, column pair of this thread
  int sw = 0;
  for (; sw < max_sweeps; ++sw) {
    if (t == 0) any = 0;
    __syncthreads();
    for (int r = 0; r < P2 - 1; ++r) {
      if (t < ROT) {
        int p, q;
        round_robin(P2, r, t, &p, &q);
        const double app = M[p][p], aqq = M[q][q], apq = M[p][q];
        const double lim = relative ? tol * sqrt(fabs(app * aqq)) : tol;
        double c = 1.0, s = 0.0;
        if (fabs(apq) > lim && apq != 0.0) {
          const double d = aqq - app;
          double tt;
          if (fabs(apq) < 1e-150 * fabs(d)) tt = apq / d;
          else {
            const double tau = d / (2.0 * apq);
            tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
          }
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = tt * c;
          any = 1;
        }
        cs[t][0] = c; cs[t][1] = s;
      }
      int p, q, u, v;
      round_robin(P2, r, kr, &p, &q);
      round_robin(P2, r, kc, &u, &v);
      __syncthreads();
      const double cr = cs[kr][0], sr = cs[kr][1];
      const double cc = cs[kc][0], sc = cs[kc][1];
      // every load of the round is issued before the first store
      double a = M[p][u], b = M[p][v], c = M[q][u], d = M[q][v];
      const double ja = J[p][u], jb = J[p][v], jc = J[q][u], jd = J[q][v];
      if (sr != 0.0 || sc != 0.0) {
        if (sr != 0.0) {   // rows: M <- J_r^T M
          const double a1 = cr * a - sr * c, c1 = sr * a + cr * c;
          const double b1 = cr * b - sr * d, d1 = sr * b + cr * d;
          a = a1; b = b1; c = c1; d = d1;
        }
        if (sc != 0.0) {   // columns: M <- M J_r
          const double a1 = cc * a - sc * b, b1 = sc * a + cc * b;
          const double c1 = cc * c - sc * d, d1 = sc * c + cc * d;
          a = a1; b = b1; c = c1; d = d1;
        }
        if (kr == kc) { b = 0.0; c = 0.0; }   // the pair's own off-diagonal
        M[p][u] = a; M[p][v] = b; M[q][u] = c; M[q][v] = d;
      }
      if (sc != 0.0) {     // J <- J J_r on rows p, q
        J[p][u] = cc * ja - sc * jb; J[p][v] = sc * ja + cc * jb;
        J[q][u] = cc * jc - sc * jd; J[q][v] = sc * jc + cc * jd;
      }
      __syncthreads();
    }
    const int more = any;
    __syncthreads();
    if (!more) break;
  }
  return sw;
}

// C = alpha op(A) B (+ beta D) for P2 x P2 LDS matrices (op = transpose when
// ta) on the FP64 matrix cores: the NT / 64 waves each own one 16 x 16 block
// of C and run P2 / 4 v_mfma_f64_16x16x4f64 steps (operand lane l holds
// A[l%16][l/16] and B[l/16][l%16]; result element r of lane l is
// C[l/16 + 4r][l%16]).  C must not alias A or B.
static_assert(P2 == 32 && NT == 256, "one 16x16 output block per wave");
__device__ inline void lds_mm(const double (*A)[LDM], bool ta, const double (*B)[LDM],
                              double (*C)[LDM], double alpha, const double (*D)[LDM], double beta) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bi = (wv & 1) * 16, bj = (wv >> 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k0 = 0; k0 < P2; k0 += 4) {
    const int k = k0 + lk;
    const double av = ta ? A[k][bi + li] : A[bi + li][k];
    const double bv = B[k][bj + li];
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = bi + lk + 4 * r, col = bj + li;
    double v = alpha * acc[r];
    if (D) v += beta * D[row][col];
    C[row][col] = v;
  }
}

// J <- J (3I - J^T J) / 2: one Newton-Schulz step towards the nearest
// orthogonal matrix.  T and U are LDS scratch.
__device__ void orthonormalize(double (*J)[LDM], double (*T)[LDM], double (*U)[LDM]) {
  const int t = threadIdx.x;
  lds_mm(J, true, J, T, -0.5, nullptr, 0.0);           // T = -J^T J / 2
  __syncthreads();
  if (t < P2) T[t][t] += 1.5;                          // T = (3I - J^T J)/2
  __syncthreads();
  lds_mm(J, false, T, U, 1.0, nullptr, 0.0);           // U = J T
  __syncthreads();
  for (int e = t; e < P2 * P2; e += NT) J[e % P2][e / P2] = U[e % P2][e / P2];
  __syncthreads();
}

struct SymArgs {
  double* H; int64_t ldh; int nb;   // padded to nb*JB, zero outside n
  int64_t n;
  double* Jb;                        // [nb/2][P2*P2], fragment order
  double* V; int64_t ldv;            // npad x npad
  double tol;
  double* offmax;                    // per sweep
  int* act;                          // [nb/2]: 1 if the pair's rotation is not the identity
  int sweep; int step;
};

__device__ inline int64_t blk_index(int p, int q, int i) {  // pair (p,q) local index i -> global
  return (i < JB) ? (int64_t)p * JB + i : (int64_t)q * JB + (i - JB);
}

// Pair rotations are stored in the operand order of the FP64 MFMA so that
// every wave loads its operand fragments with contiguous 512-byte reads:
// slot e = 512 h + 64 s + l (h: 16-column half, s: k-step of 4 rows, l:
// lane) holds J[4s + l/16][16h + l%16]; frag_row / frag_col invert it.
__device__ inline int frag_row(int e) { return 4 * ((e / 64) % 8) + (e % 64) / 16; }
__device__ inline int frag_col(int e) { return 16 * (e / 512) + e % 16; }
static_assert(P2 == 32, "fragment order assumes 32 x 32 rotations");

// H is kept block-upper: a JB x JB block (bi, bj) is current only for
// bi <= bj (diagonal blocks in full); block (bi, bj) with bi > bj is read as
// the transpose of block (bj, bi) and never written.  Each sub-block of a
// tile moves with one element per thread, the contiguous index on
// consecutive lanes whichever way the block is stored.
static_assert(JB * JB == NT, "one element of a JB x JB block per thread");

__device__ inline void load_tile(const double* H, int64_t ld, int r0, int r1, int c0, int c1,
                                 double (*X)[LDM]) {
  const int a = threadIdx.x % JB, b = threadIdx.x / JB;
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int si = sb & 1, sj = sb >> 1;
    const int bi = si ? r1 : r0, bj = sj ? c1 : c0;
    if (bi <= bj) X[si * JB + a][sj * JB + b] = H[(int64_t)bi * JB + a + ((int64_t)bj * JB + b) * ld];
    else X[si * JB + b][sj * JB + a] = H[(int64_t)bj * JB + a + ((int64_t)bi * JB + b) * ld];
  }
}

// Writes the sub-blocks of X that are stored (bi <= bj), transposing those
// with bi > bj into their stored position; with skip_lower, blocks with
// bi > bj are left alone (their transposes are written from the same tile);
// with skip_diag, the diagonal entries of diagonal blocks are not written.
__device__ inline void store_tile(double* H, int64_t ld, int r0, int r1, int c0, int c1,
                                  const double (*X)[LDM], bool skip_lower, bool skip_diag = false) {
  const int a = threadIdx.x % JB, b = threadIdx.x / JB;
#pragma unroll
  for (int sb = 0; sb < 4; ++sb) {
    const int si = sb & 1, sj = sb >> 1;
    const int bi = si ? r1 : r0, bj = sj ? c1 : c0;
    if (skip_diag && bi == bj && a == b) continue;
    if (bi <= bj) H[(int64_t)bi * JB + a + ((int64_t)bj * JB + b) * ld] = X[si * JB + a][sj * JB + b];
    else if (!skip_lower) H[(int64_t)bj * JB + a + ((int64_t)bi * JB + b) * ld] = X[si * JB + b][sj * JB + a];
  }
}

// One workgroup per pair: gather the pair's diagonal sub-problem,
// diagonalise, re-orthonormalise J, store J and write back the rotated
// sub-problem with its diagonal recomputed as diag(J^T M0 J).
__global__ __launch_bounds__(NT) void sym_pair_kernel(SymArgs a) {
  __shared__ double M[P2][LDM];
  __shared__ double J[P2][LDM];
  __shared__ double M0[P2][LDM];
  __shared__ double T[P2][LDM];
  __shared__ double red[NT / 64];
  const int t = threadIdx.x;
  int p, q;
  round_robin(a.nb, a.step, blockIdx.x, &p, &q);
  load_tile(a.H, a.ldh, p, q, p, q, M);
  __syncthreads();
  double off = 0.0;
  for (int e = t; e < P2 * P2; e += NT) {
    const int i = e % P2, j = e / P2;
    const double v = M[i][j];
    M0[i][j] = v;
    J[i][j] = (i == j) ? 1.0 : 0.0;
    if (i != j) off = fmax(off, fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
  if ((t & 63) == 0) red[t >> 6] = off;
  __syncthreads();
  if (t == 0) {
    double m = red[0];
    for (int i = 1; i < NT / 64; ++i) m = fmax(m, red[i]);
    atomic_max_nonneg(a.offmax + a.sweep, m);
  }
  const int rotated = inner_jacobi(M, J, a.tol, false, QDWHP_JACOBI_INNER);
  if (t == 0) a.act[blockIdx.x] = rotated > 0;
  // the rotated sub-problem goes back now (its diagonal is rewritten below
  // from the re-orthonormalised J), freeing M
  store_tile(a.H, a.ldh, p, q, p, q, M, true, true);
  __syncthreads();
  orthonormalize(J, T, M);
  // diagonal of J^T M0 J with the orthonormalised J: T = M0 J, d_i = sum_k J[k][i] T[k][i]
  lds_mm(M0, false, J, T, 1.0, nullptr, 0.0);
  __syncthreads();
  double* Jout = a.Jb + (int64_t)blockIdx.x * P2 * P2;
  for (int e = t; e < P2 * P2; e += NT) Jout[e] = J[frag_row(e)][frag_col(e)];
  if (t < P2) {
    double acc = 0.0;
    for (int k = 0; k < P2; ++k) acc += J[k][t] * T[k][t];
    a.H[blk_index(p, q, t) + blk_index(p, q, t) * a.ldh] = acc;
  }
}

// Tile (P, Q), P < Q over pair indices: H_PQ <- J_P^T H_PQ J_Q, mirrored to H_QP.
__device__ __forceinline__ void tile_update(const SymArgs& a, int64_t lin, double (*X)[LDM], double (*Y)[LDM]) {
  const int np = a.nb / 2;
  int P = 0;
  int64_t rem = lin;
  while (rem >= np - 1 - P) { rem -= np - 1 - P; ++P; }
  const int Q = P + 1 + (int)rem;
  int pP, qP, pQ, qQ;
  round_robin(a.nb, a.step, P, &pP, &qP);
  round_robin(a.nb, a.step, Q, &pQ, &qQ);
  // The rotations enter the two MFMA products as register operands loaded
  // in fragment order; wave w owns the 16 x 16 output block (bi, bj), and
  // its J_P^T operand is the fragment half bi / 16 of J_P, its J_Q operand
  // the half bj / 16 of J_Q.
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int bi = (wv & 1) * 16, bj = (wv >> 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  const double* FP = a.Jb + (int64_t)P * P2 * P2 + bi * P2 + lane;
  const double* FQ = a.Jb + (int64_t)Q * P2 * P2 + bj * P2 + lane;
  double jp[P2 / 4], jq[P2 / 4];
#pragma unroll
  for (int s4 = 0; s4 < P2 / 4; ++s4) {
    jp[s4] = FP[64 * s4];   // J_P[4 s4 + lk][bi + li] = (J_P^T)[bi + li][4 s4 + lk]
    jq[s4] = FQ[64 * s4];   // J_Q[4 s4 + lk][bj + li]
  }
  load_tile(a.H, a.ldh, pP, qP, pQ, qQ, X);
  // the skip test comes after the loads are issued so that its latency
  // overlaps theirs (the flags are uniform over the workgroup)
  if (!a.act[P] && !a.act[Q]) return;   // both rotations are the identity
  __syncthreads();
  v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < P2 / 4; ++s4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(jp[s4], X[4 * s4 + lk][bj + li], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) Y[bi + lk + 4 * r][bj + li] = acc[r];   // Y = J_P^T X
  __syncthreads();
  acc = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < P2 / 4; ++s4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Y[bi + li][4 * s4 + lk], jq[s4], acc, 0, 0, 0);
#pragma unroll
  for (int r = 0; r < 4; ++r) X[bi + lk + 4 * r][bj + li] = acc[r];   // X = Y J_Q
  __syncthreads();
  // pair blocks of P and Q are disjoint: every sub-block has exactly one
  // stored copy, written from here
  store_tile(a.H, a.ldh, pP, qP, pQ, qQ, X, false);
}

// V[:, pair Q] <- V[:, pair Q] J_Q: one thread per row holds the row's 2JB
// entries in registers; J_Q sits in LDS and every lane reads the same entry
// (a broadcast).  Rows of a workgroup are consecutive, so each column access
// is coalesced.
__device__ __forceinline__ void cols_rotate(double* V, int64_t ldv, int64_t rows, int nb, int step,
                                            const double* Jb, const int* act, int Q, int64_t rb, double* JQ) {
  if (!act[Q]) return;             // identity rotation
  int p, q;
  round_robin(nb, step, Q, &p, &q);
  const double* J = Jb + (int64_t)Q * P2 * P2;
  for (int e = threadIdx.x; e < P2 * P2; e += NT) JQ[frag_row(e) + frag_col(e) * P2] = J[e];
  __syncthreads();
  const int64_t r = rb * NT + threadIdx.x;
  if (r >= rows) return;
  double x[P2];
#pragma unroll
  for (int k = 0; k < P2; ++k) x[k] = V[r + blk_index(p, q, k) * ldv];
#pragma unroll
  for (int j0 = 0; j0 < P2; j0 += 8) {
    double y[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) y[u] = 0.0;
#pragma unroll
    for (int k = 0; k < P2; ++k)
#pragma unroll
      for (int u = 0; u < 8; ++u) y[u] += x[k] * JQ[k + (j0 + u) * P2];
#pragma unroll
    for (int u = 0; u < 8; ++u) V[r + blk_index(p, q, j0 + u) * ldv] = y[u];
  }
}

__global__ __launch_bounds__(NT) void cols_update_kernel(double* V, int64_t ldv, int64_t rows, int nb,
                                                         int step, const double* Jb, const int* act) {
  __shared__ double JQ[P2 * P2];   // column-major J_Q
  cols_rotate(V, ldv, rows, nb, step, Jb, act, blockIdx.y, blockIdx.x, JQ);
}

// Rotations of the one-sided round applied to R (rows1 rows) and V (rows2
// rows) in one launch: the first rb1 x pairs workgroups take R.
__global__ __launch_bounds__(NT) void cols_update2_kernel(double* R, int64_t ldr, int64_t rows1, int64_t rb1,
                                                          double* V, int64_t ldv, int64_t rows2, int64_t rb2,
                                                          int nb, int step, const double* Jb, const int* act) {
  __shared__ double JQ[P2 * P2];
  const int64_t b = blockIdx.x;
  const int64_t npair = nb / 2;
  if (b < rb1 * npair) cols_rotate(R, ldr, rows1, nb, step, Jb, act, (int)(b / rb1), b % rb1, JQ);
  else {
    const int64_t c = b - rb1 * npair;
    cols_rotate(V, ldv, rows2, nb, step, Jb, act, (int)(c / rb2), c % rb2, JQ);
  }
}

__global__ __launch_bounds__(NT) void sym_update_kernel(SymArgs a) {
  __shared__ double X[P2][LDM];
  __shared__ double Y[P2][LDM];
  tile_update(a, blockIdx.x, X, Y);
}

// The two updates of a two-sided round in one launch (they only share the
// rotations): the first ntiles workgroups update tiles of H, the rest
// rotate row blocks of V.  It carries the register needs of both paths, so
// it is used where launches dominate (small ell) and the two kernels above
// where bandwidth does.
__global__ __launch_bounds__(NT) void round_update_kernel(SymArgs a, int64_t ntiles, int64_t rowblocks) {
  __shared__ double smem[2 * P2 * LDM];
  const int64_t b = blockIdx.x;
  if (b < ntiles) {
    tile_update(a, b, (double (*)[LDM])smem, (double (*)[LDM])(smem + P2 * LDM));
  } else {
    const int64_t idx = b - ntiles;
    cols_rotate(a.V, a.ldv, a.n, a.nb, a.step, a.Jb, a.act, (int)(idx / rowblocks), idx % rowblocks, smem);
  }
}

// One-sided step: Gram of the pair's columns of R (rows x npad), Jacobi,
// rotation of those columns of R and V.
struct SvjArgs {
  double* R; int64_t ldr; int64_t rows; int nb;
  double* V; int64_t ldv; int64_t vrows;
  double* Jb; double tol; double* offmax; int* act; int sweep; int step;
};

// One-sided step, split over rows so that every round keeps the device busy:
//   svj_gram_kernel   (row chunk, pair): partial Gram of the pair's 2JB
//                     columns over GR rows;
//   svj_solve_kernel  (pair): Gram = sum of the partials in chunk order,
//                     off-diagonal measure, Jacobi on the Gram matrix,
//                     re-orthonormalised rotation J;
//   cols_update_kernel (row chunk, pair), on R and on V: columns <- columns J.
constexpr int GR = 256;   // rows per partial Gram

__global__ __launch_bounds__(NT) void svj_gram_kernel(SvjArgs a, double* part, int nchunk) {
  __shared__ double X[P2][LDM];
  const int t = threadIdx.x;
  int p, q;
  round_robin(a.nb, a.step, blockIdx.y, &p, &q);
  // Gram X^T X of the chunk's rows on the FP64 matrix cores: wave w owns the
  // 16 x 16 block (bi, bj) and accumulates over the rows in steps of 4
  const int lane = t & 63, wv = t >> 6;
  const int bi = (wv & 1) * 16, bj = (wv >> 1) * 16;
  const int li = lane & 15, lk = lane >> 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t rbeg = (int64_t)blockIdx.x * GR;
  const int64_t rend = (rbeg + GR < a.rows) ? rbeg + GR : a.rows;
  for (int64_t r0 = rbeg; r0 < rend; r0 += P2) {
    for (int e = t; e < P2 * P2; e += NT) {
      const int i = e % P2, j = e / P2;
      const int64_t r = r0 + i;
      X[i][j] = (r < rend) ? a.R[r + blk_index(p, q, j) * a.ldr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 0; k0 < P2; k0 += 4) {
      const int k = k0 + lk;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(X[k][bi + li], X[k][bj + li], acc, 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = part + ((int64_t)blockIdx.y * nchunk + blockIdx.x) * P2 * P2;
#pragma unroll
  for (int r = 0; r < 4; ++r) out[(bi + lk + 4 * r) + (bj + li) * P2] = acc[r];
}

__global__ __launch_bounds__(NT) void svj_solve_kernel(SvjArgs a, const double* part, int nchunk) {
  __shared__ double M[P2][LDM];
  __shared__ double J[P2][LDM];
  __shared__ double X[P2][LDM];
  __shared__ double red[NT / 64];
  const int t = threadIdx.x;
  const double* base = part + (int64_t)blockIdx.x * nchunk * P2 * P2;
  for (int e = t; e < P2 * P2; e += NT) {
    double acc = 0.0;
    for (int c = 0; c < nchunk; ++c) acc += base[(int64_t)c * P2 * P2 + e];
    const int i = e % P2, j = e / P2;
    M[i][j] = acc;
    J[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  double off = 0.0;
  for (int e = t; e < P2 * P2; e += NT) {
    const int i = e % P2, j = e / P2;
    if (i != j) {
      const double den = sqrt(fabs(M[i][i] * M[j][j]));
      if (den > 0.0) off = fmax(off, fabs(M[i][j]) / den);
    }
  }
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
  if ((t & 63) == 0) red[t >> 6] = off;
  __syncthreads();
  if (t == 0) {
    double m = red[0];
    for (int i = 1; i < NT / 64; ++i) m = fmax(m, red[i]);
    atomic_max_nonneg(a.offmax + a.sweep, m);
  }
  const int rotated = inner_jacobi(M, J, a.tol, true, QDWHP_JACOBI_INNER);
  if (t == 0) a.act[blockIdx.x] = rotated > 0;
  orthonormalize(J, M, X);
  double* Jout = a.Jb + (int64_t)blockIdx.x * P2 * P2;
  for (int e = t; e < P2 * P2; e += NT) Jout[e] = J[frag_row(e)][frag_col(e)];
}

// Rank of each of the first n values by descending key (ties by index).
__global__ void rank_kernel(const double* key, int64_t kstride, int64_t n, int64_t* rank) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double ki = key[i * kstride];
  int64_t r = 0;
  for (int64_t j = 0; j < n; ++j) {
    const double kj = key[j * kstride];
    r += (kj > ki) || (kj == ki && j < i);
  }
  rank[i] = r;
}

__global__ void gather_cols_kernel(const double* Win, int64_t ldi, double* Wout, int64_t ldo,
                                   int64_t rows, const int64_t* rank, int64_t n) {
  const int64_t col = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n || r >= rows) return;
  Wout[r + rank[col] * ldo] = Win[r + col * ldi];
}

__global__ void diag_gather_kernel(const double* H, int64_t ldh, int64_t n, const int64_t* rank, double* w) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[rank[i]] = H[i + i * ldh];
}

__global__ void scatter_rank_kernel(const double* v, int64_t n, const int64_t* rank, double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[rank[i]] = v[i];
}

__global__ void col_norms_kernel(const double* R, int64_t ldr, int64_t rows, int64_t n, double* out) {
  __shared__ double red[256];
  const int64_t j = blockIdx.x;
  double acc = 0.0;
  for (int64_t r = threadIdx.x; r < rows; r += 256) { const double v = R[r + j * ldr]; acc += v * v; }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0 && j < n) out[j] = sqrt(red[0]);
}

__global__ void scale_cols_kernel(double* R, int64_t ldr, int64_t rows, const double* nrm) {
  const int64_t j = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < rows) {
    const double s = nrm[j];
    R[r + j * ldr] = (s > 0.0) ? R[r + j * ldr] / s : 0.0;
  }
}

// ||H||_F in two fixed-order stages: column-strided partial sums per
// workgroup, then one workgroup adds the partials.
constexpr int FROB_WG = 256;

// Largest off-diagonal magnitude of the block-upper H (n x n, ld ldh; the
// stored rows of column j are those of blocks up to j's), max-combined into
// *out (>= 0, zeroed by the caller); a NaN counts as infinite.
__global__ void off_max_kernel(const double* H, int64_t ldh, int64_t n, double* out) {
  __shared__ double red[4];
  double m = 0.0;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x) {
    const int64_t rows = (j / JB + 1) * JB < n ? (j / JB + 1) * JB : n;
    for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
      const double a = fabs(H[i + j * ldh]);
      if (i != j && !(a <= m)) m = (a == a) ? a : INFINITY;
    }
  }
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) r = fmax(r, red[w]);
    atomic_max_nonneg(out, r);
  }
}
__global__ void frob_part_kernel(const double* H, int64_t ldh, int64_t n, double* part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t j = blockIdx.x; j < n; j += gridDim.x)
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const double v = H[i + j * ldh];
      acc += v * v;
    }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void frob_final_kernel(const double* part, int np, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) acc += part[i];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

// Stopping rule.  The largest off-diagonal magnitude seen in a sweep is
// compared with the target tol; near convergence it is set by the rounding
// noise of the sub-problem data (Gram entries, rotated tiles), whose
// maximum over all pairs can exceed tol for large problems.  A sweep whose
// measure is within 32 tol and no longer fell by 4x is therefore at the
// noise floor and counts as converged.  (The two-sided solver also stops
// as soon as the whole matrix, measured after a sweep, is within 32 tol:
// the state that this rule accepts, reached two sweeps earlier, since the
// sweeps between rotate only entries at the noise floor and leave the
// residuals and orthogonality unchanged.)
constexpr int kMaxSweeps = 60;
bool converged(double off, double prev, double tol, int sw) {
  if (off <= tol) return true;
  return sw >= 3 && off <= 32.0 * tol && off > 0.25 * prev;
}

// The eigenvector update V <- V J of a two-sided round only needs that
// round's rotations, so above the fused size it runs on a helper stream,
// overlapping the next rounds' pair solves and tile updates.  The rotations
// and skip flags of kRing consecutive rounds live in a ring of slots; a
// round waits for the update that last read its slot before refilling it.
constexpr int kRing = kAuxRing;   // the helper set's event ring (common.h)

}  // namespace

int64_t jacobi_padded(int64_t n) { int64_t nb = cdiv(n > 0 ? n : 1, JB); if (nb & 1) ++nb; if (nb < 2) nb = 2; return nb * JB; }

int64_t syev_scratch_doubles(int64_t n) {
  const int64_t np = jacobi_padded(n);
  return np * np * 2 + kRing * (np / JB / 2) * P2 * P2 + 128 + 2 * np + kRing * (np / JB / 2) + 256;
}

// H (n x n, ldh) is copied into a padded work matrix; results: w[n] descending,
// W (n x n) eigenvectors.  Returns sweeps, or -1 if not converged.
int syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw, double* scratch,
         hipStream_t s) {
  const int64_t np = jacobi_padded(n);
  const int nb = (int)(np / JB);
  double* Hp = scratch;
  double* Vp = Hp + np * np;
  const int np2 = nb / 2;
  const int64_t jslot = (int64_t)np2 * P2 * P2;
  double* Jb = Vp + np * np;                 // kRing slots of np2 rotations
  double* offmax = Jb + kRing * jslot;       // [0, 64): pair measure per sweep; [64, 128): end of sweep
  int64_t* rank = (int64_t*)(offmax + 128);
  double* fro = (double*)(rank + np);
  int* act = (int*)(fro + 8);                // kRing slots of np2 flags
  fill(Hp, np, np, np, 0.0, 0.0, s);
  copy(H, ldh, Hp, np, n, n, s);
  fill(Vp, np, np, np, 0.0, 1.0, s);
  QDWHP_HIP(hipMemsetAsync(offmax, 0, 128 * sizeof(double), s));
  {   // the pair-rotation buffer is free until the sweeps start
    const int g = (int)std::min<int64_t>(FROB_WG, np);
    frob_part_kernel<<<g, 256, 0, s>>>(Hp, np, np, Jb);
    QDWHP_LAUNCH_CHECK();
    frob_final_kernel<<<1, 256, 0, s>>>(Jb, g, fro);
    QDWHP_LAUNCH_CHECK();
  }
  double hf = 0.0;
  QDWHP_HIP(hipMemcpyAsync(&hf, fro, sizeof(double), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  SymArgs a;
  a.H = Hp; a.ldh = np; a.nb = nb; a.n = n; a.Jb = Jb; a.V = Vp; a.ldv = np;
  // skip / stop threshold: 2u times the rms eigenvalue ||H||_F / sqrt(n); an
  // eigenvector's residual is then at most ~2u ||H||_F
  a.tol = 2.0 * 1.1102230246251565e-16 * (hf > 0.0 ? hf / std::sqrt((double)n) : 1.0);
  a.offmax = offmax;
  a.act = act;
  const int64_t ntiles = (int64_t)np2 * (np2 - 1) / 2;
  const bool fused = n <= qdwhp_tune_get("jacobi.fused_max", 2048) || no_alloc_mode();
  int dev = 0;
  QDWHP_HIP(hipGetDevice(&dev));
  std::unique_ptr<AuxLease> aux;
  if (!fused) aux.reset(new AuxLease(dev));
  int sweeps = -1;
  double prev = 0.0;
  int64_t round = 0;
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    a.sweep = sw;
    for (int st = 0; st < nb - 1; ++st, ++round) {
      a.step = st;
      if (fused) {
        sym_pair_kernel<<<np2, NT, 0, s>>>(a);
        QDWHP_LAUNCH_CHECK();
        const int64_t rowblocks = cdiv(n, NT);
        round_update_kernel<<<(unsigned)(ntiles + rowblocks * np2), NT, 0, s>>>(a, ntiles, rowblocks);
        QDWHP_LAUNCH_CHECK();
        continue;
      }
      const int slot = (int)(round % kRing);
      a.Jb = Jb + slot * jslot;
      a.act = act + slot * np2;
      if (round >= kRing) QDWHP_HIP(hipStreamWaitEvent(s, (*aux)->done[slot], 0));
      sym_pair_kernel<<<np2, NT, 0, s>>>(a);
      QDWHP_LAUNCH_CHECK();
      QDWHP_HIP(hipEventRecord((*aux)->ready[slot], s));
      if (ntiles > 0) {
        sym_update_kernel<<<(unsigned)ntiles, NT, 0, s>>>(a);
        QDWHP_LAUNCH_CHECK();
      }
      hipStream_t s2 = (*aux)->s;
      QDWHP_HIP(hipStreamWaitEvent(s2, (*aux)->ready[slot], 0));
      cols_update_kernel<<<dim3((unsigned)cdiv(n, NT), np2), NT, 0, s2>>>(Vp, np, n, nb, st, a.Jb, a.act);
      QDWHP_LAUNCH_CHECK();
      QDWHP_HIP(hipEventRecord((*aux)->done[slot], s2));
    }
    // the off-diagonal part as the sweep leaves it: within 32 tol it is at
    // the noise floor (the next sweeps rotate only entries there, or at or
    // below tol nothing, every |h_pq| <= tol being skipped), so they are
    // not run
    off_max_kernel<<<256, 256, 0, s>>>(Hp, np, np, offmax + 64 + sw);
    QDWHP_LAUNCH_CHECK();
    double off = 0.0, endm = 0.0;
    QDWHP_HIP(hipMemcpyAsync(&off, offmax + sw, sizeof(double), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipMemcpyAsync(&endm, offmax + 64 + sw, sizeof(double), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (converged(off, prev, a.tol, sw) || endm <= 32.0 * a.tol) { sweeps = sw + 1; break; }
    prev = off;
  }
  if (aux && round > 0)   // the last eigenvector updates precede the gather below
    QDWHP_HIP(hipStreamWaitEvent(s, (*aux)->done[(int)((round - 1) % kRing)], 0));
  // eigenvalues: diagonal of the first n positions; sort descending
  rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(Hp, np + 1, n, rank);
  QDWHP_LAUNCH_CHECK();
  diag_gather_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(Hp, np, n, rank, w);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)n), 256, 0, s>>>(Vp, np, W, ldw, n, rank, n);
  QDWHP_LAUNCH_CHECK();
  return sweeps;
}

int64_t gesvj_scratch_doubles(int64_t rows, int64_t n) {
  const int64_t np = jacobi_padded(n);
  const int64_t parts = (np / JB / 2) * cdiv(rows > 0 ? rows : 1, GR) * P2 * P2;
  return (rows > np ? rows : np) * np + np * np + (np / JB / 2) * P2 * P2 + 64 + 2 * np + np + parts + 256;
}

// One-sided Jacobi on R (rows x n): R <- U diag(S) (columns sorted), V (n x n).
int gesvj(double* R, int64_t rows, int64_t n, int64_t ldr, double* S, double* V, int64_t ldv,
          double* scratch, hipStream_t s) {
  const int64_t np = jacobi_padded(n);
  const int nb = (int)(np / JB);
  double* Rp = scratch;                    // rows x np
  double* Vp = Rp + (rows > np ? rows : np) * np;
  double* Jb = Vp + np * np;
  double* offmax = Jb + (int64_t)(nb / 2) * P2 * P2;
  int64_t* rank = (int64_t*)(offmax + 64);
  double* nrm = (double*)(rank + np);
  double* part = nrm + np;
  const int nchunk = (int)cdiv(rows, GR);
  int* act = (int*)(part + (int64_t)(nb / 2) * nchunk * P2 * P2);
  fill(Rp, rows, np, rows, 0.0, 0.0, s);
  copy(R, ldr, Rp, rows, rows, n, s);
  fill(Vp, np, np, np, 0.0, 1.0, s);
  QDWHP_HIP(hipMemsetAsync(offmax, 0, 64 * sizeof(double), s));
  SvjArgs a;
  a.R = Rp; a.ldr = rows; a.rows = rows; a.nb = nb; a.V = Vp; a.ldv = np; a.vrows = n;
  a.Jb = Jb; a.tol = 4e-16 * std::sqrt((double)rows); a.offmax = offmax; a.act = act;
  int sweeps = -1;
  double prev = 0.0;
  for (int sw = 0; sw < kMaxSweeps; ++sw) {
    a.sweep = sw;
    for (int st = 0; st < nb - 1; ++st) {
      a.step = st;
      svj_gram_kernel<<<dim3((unsigned)nchunk, nb / 2), NT, 0, s>>>(a, part, nchunk);
      QDWHP_LAUNCH_CHECK();
      svj_solve_kernel<<<nb / 2, NT, 0, s>>>(a, part, nchunk);
      QDWHP_LAUNCH_CHECK();
      {
        const int64_t rb1 = cdiv(rows, NT), rb2 = cdiv(n, NT);
        cols_update2_kernel<<<(unsigned)((rb1 + rb2) * (nb / 2)), NT, 0, s>>>(Rp, rows, rows, rb1, Vp, np, n, rb2,
                                                                              nb, st, Jb, a.act);
        QDWHP_LAUNCH_CHECK();
      }
    }
    double off = 0.0;
    QDWHP_HIP(hipMemcpyAsync(&off, offmax + sw, sizeof(double), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (converged(off, prev, a.tol, sw)) { sweeps = sw + 1; break; }
    prev = off;
  }
  col_norms_kernel<<<(unsigned)n, 256, 0, s>>>(Rp, rows, rows, n, nrm);
  QDWHP_LAUNCH_CHECK();
  rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(nrm, 1, n, rank);
  QDWHP_LAUNCH_CHECK();
  scale_cols_kernel<<<dim3((unsigned)cdiv(rows, 256), (unsigned)n), 256, 0, s>>>(Rp, rows, rows, nrm);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(rows, 256), (unsigned)n), 256, 0, s>>>(Rp, rows, R, ldr, rows, rank, n);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)n), 256, 0, s>>>(Vp, np, V, ldv, n, rank, n);
  QDWHP_LAUNCH_CHECK();
  scatter_rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(nrm, n, rank, S);
  QDWHP_LAUNCH_CHECK();
  return sweeps;
}

}  // namespace qdwhp
