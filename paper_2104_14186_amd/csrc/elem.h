// Elementwise kernels of the solve drivers (see elem.hip).
#pragma once
#include "common.h"

namespace qdwhp {

void eig_x0(const double* A, int64_t lda, double* X, int64_t ldx, int64_t n, double f, double tau,
            double sgn, double s, hipStream_t st);
void scale_copy(const double* A, int64_t lda, double* X, int64_t ldx, int64_t rows, int64_t cols,
                double inv, bool trans, hipStream_t st);
// W = [sc X; I] ((m + n) x n); sc is read from *dsc when dsc is set.
void stacked(const double* X, int64_t ldx, double* W, int64_t ldw, int64_t m, int64_t n, double sc,
             hipStream_t st, const double* dsc = nullptr);
void symmetrize(double* X, int64_t n, int64_t ld, hipStream_t st);
// Y (m x n, FP32) = X rounded to nearest
void to_f32(const double* X, int64_t ldx, float* Y, int64_t ldy, int64_t m, int64_t n, hipStream_t st);
void half_plus_identity(const double* X, int64_t ldx, double* B, int64_t ldb, int64_t n, hipStream_t st);
void diagonal(const double* A, int64_t lda, int64_t n, double* d, hipStream_t st);
void upper_copy(const double* A, int64_t lda, double* R, int64_t ldr, int64_t n, hipStream_t st);
void sign_normalize(double* V, int64_t ldv, int64_t rows, int64_t k, double* U, int64_t ldu,
                    int64_t urows, hipStream_t st);
void scale_vec(const double* x, double* y, int64_t n, double a, hipStream_t st);
void nonfinite(const double* A, int64_t lda, int64_t m, int64_t n, int* flag, hipStream_t st);

}  // namespace qdwhp
