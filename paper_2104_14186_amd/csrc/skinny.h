// Products with few right-hand columns (see skinny.hip).
#pragma once
#include "common.h"

namespace qdwhp {

// Doubles of workspace for up to 16 splits of k (at least m * 8 allow one).
int64_t skinny_ws_doubles(int64_t m, int nv);
// C (m x nv, ldc) = alpha A (m x k, lda) B (k x nv, ldb); nv <= 32; ws holds
// the per-split partial sums (ws_doubles >= skinny_ws_doubles(m, nv)).
void skinny_gemm(const double* A, int64_t lda, int64_t m, int64_t k, const double* B, int64_t ldb, int nv,
                 double alpha, double* C, int64_t ldc, double* ws, int64_t ws_doubles, hipStream_t s);
// C (n x nv, ldc) = alpha A^T B for A m x n (lda) and B m x nv (ldb); nv <= 8.
void skinny_gemm_t(const double* A, int64_t lda, int64_t m, int64_t n, const double* B, int64_t ldb, int nv,
                   double alpha, double* C, int64_t ldc, hipStream_t s);

}  // namespace qdwhp
