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
};
size_t grouped_table_bytes(int count);
void dgemm_grouped(const GroupedDesc* descs, int count, bool ta, bool tb, void* table, hipStream_t s);

}  // namespace qdwhp
