// Internal entry points of the EIG / SVD drivers, shared by the public C ABI,
// the ragged-batch runtime and the serving engine.
#pragma once
#include "qdwhp.h"
#include "common.h"

namespace qdwhp {

// The last matrix product of a solve (V = Q2 W_k for EIG, V = Q2 V~_k for
// SVD) and the sign step that follows it.  When a driver is handed a
// Deferred, it fills it in instead of launching them; every other step,
// including the eigen/singular values, is complete on the stream.
struct Deferred {
  Gemm g;
  double* V = nullptr; int64_t ldv = 0, n = 0, k = 0;
  double* U = nullptr; int64_t ldu = 0, m = 0;   // SVD: left vectors flipped with V
};

// One solve split into phases (solver.cpp): setup (argument checks,
// workspace, estimator, threshold, schedule, X0), the DWH iterations, and
// finish (projector QR, subspace, Rayleigh-Ritz, threshold retry, vectors).
// A batch or the server may run the iterations of several solves together
// (iterations_grouped) instead of solve_iterate.  Each phase returns the
// status (0 or a QDWHP_ERR_* / negative argument code); info is filled as
// the standalone drivers fill it.
struct SolveState;
SolveState* solve_create(const qdwhp_problem& p, void* work, size_t lwork, const qdwhp_opts* opts,
                         hipStream_t s, qdwhp_info* info, Deferred* df);
void solve_destroy(SolveState* S);
int solve_status(const SolveState* S);
void solve_set_stream(SolveState* S, hipStream_t s);   // later phases run on s
int solve_setup(SolveState* S);
int solve_iterate(SolveState* S);
int solve_finish(SolveState* S);

int eig_impl(const double* A, int64_t n, int64_t lda, double fraction, int which, double* w,
             double* V, int64_t ldv, void* work, size_t lwork, const qdwhp_opts* opts,
             void* stream, qdwhp_info* info, Deferred* df);
int svd_impl(const double* A, int64_t m, int64_t n, int64_t lda, int64_t k, double* U,
             int64_t ldu, double* S, double* V, int64_t ldv, void* work, size_t lwork,
             const qdwhp_opts* opts, void* stream, qdwhp_info* info, Deferred* df);

// Ragged persistent GEMM (gemm.hip): FP64, all problems with the same
// transposes, plain C = alpha op(A) op(B) + beta C.  table holds
// grouped_table_bytes(count) bytes of device memory.
struct GroupedDesc {
  int64_t M, N, K;
  double alpha, beta;
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  double diag = 0.0;                 // added to C(i,i)
  const double* Cin = nullptr;       // beta term from Cin (ld ldcin) instead of C
  int64_t ldcin = 0;
  int klo = KLO_ZERO, khi = KHI_K;   // triangular K ranges, as for Gemm
  int tiles = TILES_ALL;             // TILES_UPPER: only tiles on or above the diagonal (M == N)
};
size_t grouped_table_bytes(int count);
void dgemm_grouped(const GroupedDesc* descs, int count, bool ta, bool tb, void* table, hipStream_t s);

// Cholesky-inversion (potrf.hip) of several matrices of one size n in
// lockstep: the recursion of chol_inverse_factor, each of its leaves one
// launch for all the matrices and each of its products one grouped GEMM, so
// every matrix gets bitwise the result of chol_inverse_factor.  Per item: Z
// (n x n, ld ldz, upper triangle read) gets W in its upper triangle; work
// (spd_inverse_doubles(n)) gets W^{-1} (n x n upper, zeros below, ld n) at
// its start, as for chol_inverse_factor; flag likewise.
struct CholItem {
  double* Z; int64_t ldz;
  double* work;
  int* flag;
};
void chol_inverse_grouped(const CholItem* items, int count, int64_t n, void* table, hipStream_t s);

// Phase 2 of a group of solves of one shape (solver.cpp; same type, rows and
// columns): the DWH steps of all of them on stream s.  Step i of every solve
// whose step i is Cholesky-based runs as one grouped step (grouped Gram,
// the lockstep Cholesky-inversion, grouped triangular products); QR-based
// steps run per solve.  table: grouped_table_bytes(count).  Every solve
// gets bitwise the result of its own standalone iterations.
void iterations_grouped(SolveState* const* v, int count, void* table, hipStream_t s);
// Shape key of a set-up solve: solves with equal keys may be grouped.
int64_t solve_shape(const SolveState* S);

}  // namespace qdwhp
