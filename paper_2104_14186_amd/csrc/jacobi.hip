// Parallel-order block Jacobi eigen/singular value solvers for the
// Rayleigh-Ritz step (Algorithm 1: eig of Q2^T A Q2; Algorithm 2: SVD of the
// R factor of A Q2).
//
// The index set is cut into blocks of JB = 16.  A sweep visits every pair of
// blocks once in round-robin (circle) order; in each step the Nb/2 disjoint
// pairs are independent:
//   * two-sided (symmetric H): the 32x32 diagonal sub-problem of each pair is
//     diagonalised in LDS by cyclic Jacobi (one wave64 per pair, 16 disjoint
//     rotations per round), giving an orthogonal J; then H <- J^T H J tile by
//     tile (tile (P,Q) becomes J_P^T H_PQ J_Q) and V <- V J;
//   * one-sided (R): each pair forms the Gram matrix of its 32 columns,
//     diagonalises it the same way and rotates the columns of R and V by J,
//     making them mutually orthogonal.
// Off-diagonal magnitudes seen at the start of each pair solve are max-reduced
// per sweep (an order-independent atomic max) and decide convergence.
#include "common.h"
#include "jacobi.h"

namespace qdwhp {
namespace {

constexpr int P2 = 2 * JB;     // 32: size of a pair sub-problem
constexpr int LDM = P2 + 1;

// Pair (p, q) of step `step` in the circle method over nb (even) blocks.
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
// as identity).  Called by every thread of the block (blockDim.x >= 16).  A
// rotation is skipped when |m_pq| <= tol (abs) or <= tol * sqrt(m_pp m_qq)
// (relative).  Returns sweeps used.
__device__ int inner_jacobi(double (*M)[LDM], double (*J)[LDM], double tol, bool relative,
                            int max_sweeps) {
  __shared__ double cs[P2 / 2][2];
  __shared__ int pidx[P2 / 2][2];
  __shared__ int any;
  const int t = threadIdx.x, nt = blockDim.x;
  int sw = 0;
  for (; sw < max_sweeps; ++sw) {
    if (t == 0) any = 0;
    __syncthreads();
    for (int r = 0; r < P2 - 1; ++r) {
      if (t < P2 / 2) {
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
        cs[t][0] = c; cs[t][1] = s; pidx[t][0] = p; pidx[t][1] = q;
      }
      __syncthreads();
      // rows: M <- J^T M   (thread handles column j of rows p, q of rotation k)
      for (int e = t; e < (P2 / 2) * P2; e += nt) {
        const int k = e / P2, j = e % P2;
        const double c = cs[k][0], s = cs[k][1];
        if (s != 0.0) {
          const int p = pidx[k][0], q = pidx[k][1];
          const double mp = M[p][j], mq = M[q][j];
          M[p][j] = c * mp - s * mq;
          M[q][j] = s * mp + c * mq;
        }
      }
      __syncthreads();
      // columns: M <- M J and J <- J J_r
      for (int e = t; e < (P2 / 2) * P2; e += nt) {
        const int k = e / P2, i = e % P2;
        const double c = cs[k][0], s = cs[k][1];
        if (s != 0.0) {
          const int p = pidx[k][0], q = pidx[k][1];
          const double mp = M[i][p], mq = M[i][q];
          M[i][p] = c * mp - s * mq;
          M[i][q] = s * mp + c * mq;
          const double jp = J[i][p], jq = J[i][q];
          J[i][p] = c * jp - s * jq;
          J[i][q] = s * jp + c * jq;
        }
      }
      __syncthreads();
      if (t < P2 / 2 && cs[t][1] != 0.0) {
        const int p = pidx[t][0], q = pidx[t][1];
        M[p][q] = 0.0; M[q][p] = 0.0;
      }
      __syncthreads();
    }
    const int more = any;
    __syncthreads();
    if (!more) break;
  }
  return sw;
}

// J <- J (3I - J^T J) / 2: one Newton-Schulz step towards the nearest
// orthogonal matrix.  The thousands of rotations of a sub-problem leave J
// off orthogonal by a random walk of roundings; without this step that drift
// accumulates over the block steps into the eigenvalues and residuals.
__device__ void orthonormalize(double (*J)[LDM], double (*T)[LDM]) {
  const int t = threadIdx.x, nt = blockDim.x;
  for (int e = t; e < P2 * P2; e += nt) {      // T = (3I - J^T J) / 2
    const int i = e % P2, j = e / P2;
    double acc = 0.0;
    for (int k = 0; k < P2; ++k) acc += J[k][i] * J[k][j];
    T[i][j] = ((i == j) ? 1.5 : 0.0) - 0.5 * acc;
  }
  __syncthreads();
  double out[P2 * P2 / 64];
  int cnt = 0;
  for (int e = t; e < P2 * P2; e += nt) {      // J T
    const int i = e % P2, j = e / P2;
    double acc = 0.0;
    for (int k = 0; k < P2; ++k) acc += J[i][k] * T[k][j];
    out[cnt++] = acc;
  }
  __syncthreads();
  cnt = 0;
  for (int e = t; e < P2 * P2; e += nt) J[e % P2][e / P2] = out[cnt++];
  __syncthreads();
}

struct SymArgs {
  double* H; int64_t ldh; int nb;   // padded to nb*JB, zero outside n
  int64_t n;
  double* Jb;                        // [nb/2][P2*P2]
  double* V; int64_t ldv;            // npad x npad
  double tol;
  double* offmax;                    // per sweep
  int sweep; int step;
};

__device__ inline int64_t blk_index(int p, int q, int i) {  // pair (p,q) local index i -> global
  return (i < JB) ? (int64_t)p * JB + i : (int64_t)q * JB + (i - JB);
}

// One wave per pair: gather the pair's 32x32 diagonal sub-problem, diagonalise,
// store J and write the rotated (diagonal) sub-problem back.
__global__ __launch_bounds__(64) void sym_pair_kernel(SymArgs a) {
  __shared__ double M[P2][LDM];
  __shared__ double J[P2][LDM];
  __shared__ double M0[P2][LDM];
  __shared__ double T[P2][LDM];
  __shared__ double dg[P2];
  const int t = threadIdx.x;
  int p, q;
  round_robin(a.nb, a.step, blockIdx.x, &p, &q);
  double off = 0.0;
  for (int e = t; e < P2 * P2; e += 64) {
    const int i = e % P2, j = e / P2;
    const double v = a.H[blk_index(p, q, i) + blk_index(p, q, j) * a.ldh];
    M[i][j] = v;
    M0[i][j] = v;
    J[i][j] = (i == j) ? 1.0 : 0.0;
    if (i != j) off = fmax(off, fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
  if (t == 0) atomic_max_nonneg(a.offmax + a.sweep, off);
  __syncthreads();
  inner_jacobi(M, J, a.tol, false, 30);
  orthonormalize(J, T);
  // diagonal of J^T M0 J with the orthonormalised J (T = M0 J)
  for (int e = t; e < P2 * P2; e += 64) {
    const int i = e % P2, j = e / P2;
    double acc = 0.0;
    for (int k = 0; k < P2; ++k) acc += M0[i][k] * J[k][j];
    T[i][j] = acc;
  }
  __syncthreads();
  if (t < P2) {
    double acc = 0.0;
    for (int k = 0; k < P2; ++k) acc += J[k][t] * T[k][t];
    dg[t] = acc;
  }
  __syncthreads();
  double* Jout = a.Jb + (int64_t)blockIdx.x * P2 * P2;
  for (int e = t; e < P2 * P2; e += 64) {
    const int i = e % P2, j = e / P2;
    Jout[i + j * P2] = J[i][j];
    a.H[blk_index(p, q, i) + blk_index(p, q, j) * a.ldh] = (i == j) ? dg[i] : M[i][j];
  }
}

// Tile (P, Q), P < Q over pair indices: H_PQ <- J_P^T H_PQ J_Q, mirrored to H_QP.
__global__ __launch_bounds__(256) void sym_update_kernel(SymArgs a) {
  __shared__ double X[P2][LDM];
  __shared__ double Y[P2][LDM];
  __shared__ double JP[P2][LDM];
  __shared__ double JQ[P2][LDM];
  const int np = a.nb / 2;
  // linear index over pairs P < Q
  const int64_t lin = blockIdx.x;
  int P = 0;
  int64_t rem = lin;
  while (rem >= np - 1 - P) { rem -= np - 1 - P; ++P; }
  const int Q = P + 1 + (int)rem;
  int pP, qP, pQ, qQ;
  round_robin(a.nb, a.step, P, &pP, &qP);
  round_robin(a.nb, a.step, Q, &pQ, &qQ);
  const int t = threadIdx.x;
  const double* JbP = a.Jb + (int64_t)P * P2 * P2;
  const double* JbQ = a.Jb + (int64_t)Q * P2 * P2;
  for (int e = t; e < P2 * P2; e += 256) {
    const int i = e % P2, j = e / P2;
    X[i][j] = a.H[blk_index(pP, qP, i) + blk_index(pQ, qQ, j) * a.ldh];
    JP[i][j] = JbP[e];
    JQ[i][j] = JbQ[e];
  }
  __syncthreads();
  for (int e = t; e < P2 * P2; e += 256) {   // Y = J_P^T X
    const int i = e % P2, j = e / P2;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < P2; ++k) acc += JP[k][i] * X[k][j];
    Y[i][j] = acc;
  }
  __syncthreads();
  for (int e = t; e < P2 * P2; e += 256) {   // Z = Y J_Q
    const int i = e % P2, j = e / P2;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < P2; ++k) acc += Y[i][k] * JQ[k][j];
    const int64_t gi = blk_index(pP, qP, i), gj = blk_index(pQ, qQ, j);
    a.H[gi + gj * a.ldh] = acc;
    a.H[gj + gi * a.ldh] = acc;
  }
}

// V[:, pair Q] <- V[:, pair Q] J_Q for a chunk of 64 rows.
__global__ __launch_bounds__(256) void cols_update_kernel(double* V, int64_t ldv, int64_t rows, int nb,
                                                         int step, const double* Jb) {
  __shared__ double JQ[P2][LDM];
  __shared__ double X[64][LDM];
  const int Q = blockIdx.y;
  int p, q;
  round_robin(nb, step, Q, &p, &q);
  const int t = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * 64;
  const double* J = Jb + (int64_t)Q * P2 * P2;
  for (int e = t; e < P2 * P2; e += 256) JQ[e % P2][e / P2] = J[e];
  for (int e = t; e < 64 * P2; e += 256) {
    const int i = e % 64, j = e / 64;
    const int64_t r = r0 + i;
    X[i][j] = (r < rows) ? V[r + blk_index(p, q, j) * ldv] : 0.0;
  }
  __syncthreads();
  for (int e = t; e < 64 * P2; e += 256) {
    const int i = e % 64, j = e / 64;
    const int64_t r = r0 + i;
    double acc = 0.0;
#pragma unroll 8
    for (int k = 0; k < P2; ++k) acc += X[i][k] * JQ[k][j];
    if (r < rows) V[r + blk_index(p, q, j) * ldv] = acc;
  }
}

// One-sided step: Gram of the pair's 32 columns of R (rows x npad), Jacobi,
// rotation of those columns of R and V.  256 threads; the eigen-solve runs
// on the first wave.
struct SvjArgs {
  double* R; int64_t ldr; int64_t rows; int nb;
  double* V; int64_t ldv; int64_t vrows;
  double* Jb; double tol; double* offmax; int sweep; int step;
};

__global__ __launch_bounds__(256) void svj_pair_kernel(SvjArgs a) {
  __shared__ double M[P2][LDM];
  __shared__ double J[P2][LDM];
  __shared__ double X[64][LDM];
  const int t = threadIdx.x;
  int p, q;
  round_robin(a.nb, a.step, blockIdx.x, &p, &q);
  // Gram: each thread owns 4 entries of M (e = t + 256*u)
  double g[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t r0 = 0; r0 < a.rows; r0 += 64) {
    for (int e = t; e < 64 * P2; e += 256) {
      const int i = e % 64, j = e / 64;
      const int64_t r = r0 + i;
      X[i][j] = (r < a.rows) ? a.R[r + blk_index(p, q, j) * a.ldr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = t + 256 * u, i = e % P2, j = e / P2;
      double acc = g[u];
      for (int k = 0; k < 64; ++k) acc += X[k][i] * X[k][j];
      g[u] = acc;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    M[e % P2][e / P2] = g[u];
    J[e % P2][e / P2] = ((e % P2) == (e / P2)) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t < 64) {
    double off = 0.0;
    for (int e = t; e < P2 * P2; e += 64) {
      const int i = e % P2, j = e / P2;
      if (i != j) {
        const double den = sqrt(fabs(M[i][i] * M[j][j]));
        if (den > 0.0) off = fmax(off, fabs(M[i][j]) / den);
      }
    }
    for (int o = 32; o > 0; o >>= 1) off = fmax(off, __shfl_xor(off, o));
    if (t == 0) atomic_max_nonneg(a.offmax + a.sweep, off);
  }
  __syncthreads();
  inner_jacobi(M, J, a.tol, true, 30);
  orthonormalize(J, M);
  // rotate columns of R and V
  for (int pass = 0; pass < 2; ++pass) {
    double* Mat = pass == 0 ? a.R : a.V;
    const int64_t ld = pass == 0 ? a.ldr : a.ldv;
    const int64_t rows = pass == 0 ? a.rows : a.vrows;
    for (int64_t r0 = 0; r0 < rows; r0 += 64) {
      for (int e = t; e < 64 * P2; e += 256) {
        const int i = e % 64, j = e / 64;
        const int64_t r = r0 + i;
        X[i][j] = (r < rows) ? Mat[r + blk_index(p, q, j) * ld] : 0.0;
      }
      __syncthreads();
      for (int e = t; e < 64 * P2; e += 256) {
        const int i = e % 64, j = e / 64;
        const int64_t r = r0 + i;
        double acc = 0.0;
#pragma unroll 8
        for (int k = 0; k < P2; ++k) acc += X[i][k] * J[k][j];
        if (r < rows) Mat[r + blk_index(p, q, j) * ld] = acc;
      }
      __syncthreads();
    }
  }
}

// Rank of each of the first n values by descending key (ties by index), then
// gather: out[rank] = key, and column rank of Wout = column i of Win.
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
                                   int64_t rows, const int64_t* rank, int64_t n, double scale_by_norm) {
  const int64_t col = blockIdx.y;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n || r >= rows) return;
  Wout[r + rank[col] * ldo] = Win[r + col * ldi];
  (void)scale_by_norm;
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

__global__ void frob_kernel(const double* H, int64_t ldh, int64_t n, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int64_t e = threadIdx.x; e < n * n; e += 256) {
    const double v = H[(e % n) + (e / n) * ldh];
    acc += v * v;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(red[0]);
}

}  // namespace

int64_t jacobi_padded(int64_t n) { int64_t nb = cdiv(n > 0 ? n : 1, JB); if (nb & 1) ++nb; if (nb < 2) nb = 2; return nb * JB; }

int64_t syev_scratch_doubles(int64_t n) {
  const int64_t np = jacobi_padded(n);
  return np * np * 2 + (np / JB / 2) * P2 * P2 + 64 + 2 * np + 256;
}

// H (n x n, ldh) is copied into a padded work matrix; results: w[n] descending,
// W (n x n) eigenvectors.  Returns sweeps, or -1 if not converged.
int syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw, double* scratch,
         hipStream_t s) {
  const int64_t np = jacobi_padded(n);
  const int nb = (int)(np / JB);
  double* Hp = scratch;
  double* Vp = Hp + np * np;
  double* Jb = Vp + np * np;
  double* offmax = Jb + (int64_t)(nb / 2) * P2 * P2;
  int64_t* rank = (int64_t*)(offmax + 64);
  double* fro = (double*)(rank + np);
  fill(Hp, np, np, np, 0.0, 0.0, s);
  copy(H, ldh, Hp, np, n, n, s);
  fill(Vp, np, np, np, 0.0, 1.0, s);
  QDWHP_HIP(hipMemsetAsync(offmax, 0, 64 * sizeof(double), s));
  frob_kernel<<<1, 256, 0, s>>>(Hp, np, np, fro);
  QDWHP_LAUNCH_CHECK();
  double hf = 0.0;
  QDWHP_HIP(hipMemcpyAsync(&hf, fro, sizeof(double), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  SymArgs a;
  a.H = Hp; a.ldh = np; a.nb = nb; a.n = n; a.Jb = Jb; a.V = Vp; a.ldv = np;
  a.tol = 4.4e-16 * (hf > 0.0 ? hf : 1.0);
  a.offmax = offmax;
  const int np2 = nb / 2;
  const int64_t ntiles = (int64_t)np2 * (np2 - 1) / 2;
  int sweeps = -1;
  for (int sw = 0; sw < 40; ++sw) {
    a.sweep = sw;
    for (int st = 0; st < nb - 1; ++st) {
      a.step = st;
      sym_pair_kernel<<<np2, 64, 0, s>>>(a);
      QDWHP_LAUNCH_CHECK();
      if (ntiles > 0) {
        sym_update_kernel<<<(unsigned)ntiles, 256, 0, s>>>(a);
        QDWHP_LAUNCH_CHECK();
      }
      cols_update_kernel<<<dim3((unsigned)cdiv(np, 64), np2), 256, 0, s>>>(Vp, np, np, nb, st, Jb);
      QDWHP_LAUNCH_CHECK();
    }
    double off = 0.0;
    QDWHP_HIP(hipMemcpyAsync(&off, offmax + sw, sizeof(double), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (off <= a.tol) { sweeps = sw + 1; break; }
  }
  // eigenvalues: diagonal of the first n positions; sort descending
  rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(Hp, np + 1, n, rank);
  QDWHP_LAUNCH_CHECK();
  diag_gather_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(Hp, np, n, rank, w);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)n), 256, 0, s>>>(Vp, np, W, ldw, n, rank, n, 0.0);
  QDWHP_LAUNCH_CHECK();
  return sweeps;
}

int64_t gesvj_scratch_doubles(int64_t rows, int64_t n) {
  const int64_t np = jacobi_padded(n);
  return (rows > np ? rows : np) * np + np * np + (np / JB / 2) * P2 * P2 + 64 + 2 * np + np + 256;
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
  fill(Rp, rows, np, rows, 0.0, 0.0, s);
  copy(R, ldr, Rp, rows, rows, n, s);
  fill(Vp, np, np, np, 0.0, 1.0, s);
  QDWHP_HIP(hipMemsetAsync(offmax, 0, 64 * sizeof(double), s));
  SvjArgs a;
  a.R = Rp; a.ldr = rows; a.rows = rows; a.nb = nb; a.V = Vp; a.ldv = np; a.vrows = np;
  a.Jb = Jb; a.tol = 4e-16 * sqrt((double)rows); a.offmax = offmax;
  int sweeps = -1;
  for (int sw = 0; sw < 40; ++sw) {
    a.sweep = sw;
    for (int st = 0; st < nb - 1; ++st) {
      a.step = st;
      svj_pair_kernel<<<nb / 2, 256, 0, s>>>(a);
      QDWHP_LAUNCH_CHECK();
    }
    double off = 0.0;
    QDWHP_HIP(hipMemcpyAsync(&off, offmax + sw, sizeof(double), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (off <= a.tol) { sweeps = sw + 1; break; }
  }
  col_norms_kernel<<<(unsigned)n, 256, 0, s>>>(Rp, rows, rows, n, nrm);
  QDWHP_LAUNCH_CHECK();
  rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(nrm, 1, n, rank);
  QDWHP_LAUNCH_CHECK();
  scale_cols_kernel<<<dim3((unsigned)cdiv(rows, 256), (unsigned)n), 256, 0, s>>>(Rp, rows, rows, nrm);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(rows, 256), (unsigned)n), 256, 0, s>>>(Rp, rows, R, ldr, rows, rank, n, 0.0);
  QDWHP_LAUNCH_CHECK();
  gather_cols_kernel<<<dim3((unsigned)cdiv(n, 256), (unsigned)n), 256, 0, s>>>(Vp, np, V, ldv, n, rank, n, 0.0);
  QDWHP_LAUNCH_CHECK();
  scatter_rank_kernel<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(nrm, n, rank, S);
  QDWHP_LAUNCH_CHECK();
  return sweeps;
}

}  // namespace qdwhp
