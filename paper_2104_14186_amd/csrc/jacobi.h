// Block Jacobi eigen / singular value solvers (see jacobi.hip).
#pragma once
#include "common.h"

namespace qdwhp {

constexpr int JB = 16;   // Jacobi block size (pairs form 32x32 sub-problems)

int64_t jacobi_padded(int64_t n);
int64_t syev_scratch_doubles(int64_t n);
int64_t gesvj_scratch_doubles(int64_t rows, int64_t n);
// Eigenpairs of symmetric H (n x n): w descending, W eigenvectors.  H is read
// only.  Returns the sweep count, -1 if not converged.  Synchronises s.
int syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw, double* scratch,
         hipStream_t s);
// One-sided Jacobi SVD of R (rows x n, rows >= n): R <- U (columns sorted by
// descending S), S[n], V (n x n).  Returns sweeps, -1 if not converged.
int gesvj(double* R, int64_t rows, int64_t n, int64_t ldr, double* S, double* V, int64_t ldv,
          double* scratch, hipStream_t s);

}  // namespace qdwhp
