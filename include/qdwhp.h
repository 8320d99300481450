/*
 * qdwhp.h -- C ABI of the MI355X (gfx950) QDWHpartial-EIG / QDWHpartial-SVD
 * library (libqdwhp.so).
 *
 * Method: Keyes, Ltaief, Nakatsukasa, Sukkari, "High-Performance Partial
 * Spectrum Computation for Symmetric eigenvalue problems and the SVD"
 * (arXiv 2104.14186).  The solver runs a few dynamically weighted Halley
 * (QDWH) iterations whose weights are tuned only on the wanted part of the
 * spectrum (Sec. 3.1, Eqs. (1)-(3); Sec. 4), extracts a subspace containing
 * the wanted invariant subspace from a Householder QR of the spectral
 * projector (Sec. 4.1, Theorem 1 and "Choosing the subspace size"), and
 * finishes with a small Rayleigh-Ritz solve (Algorithms 1 and 2).
 *
 * Conventions shared by every entry point
 *   - Matrices are column-major IEEE FP64 in device memory (LAPACK layout,
 *     leading dimension >= number of rows).  Scalars and small result
 *     structures are host memory.
 *   - The caller owns every buffer: inputs, outputs and the workspace.  The
 *     library never allocates device memory on the solve path and keeps no
 *     pointer after a call returns.
 *   - Work is enqueued on `stream` (a hipStream_t passed as void*; NULL is the
 *     default stream).  Calls that need a data-dependent size from the device
 *     synchronise that stream internally; on return all results are complete.
 *   - Return value: 0 success; -i argument i (1-based) invalid; positive
 *     values are QDWHP_ERR_* below.  Output contents are unspecified on error.
 *   - Calls on one stream are serialised; calls that share a workspace must
 *     not overlap.
 */
#ifndef QDWHP_H
#define QDWHP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ----------------------------------------------------- */
#define QDWHP_OK                 0
#define QDWHP_ERR_NONFINITE      1  /* NaN/Inf in the input or in an iterate      */
#define QDWHP_ERR_NO_SUBSPACE    2  /* ell = 0 or fewer than k certified values   */
#define QDWHP_ERR_CHOL           3  /* Cholesky breakdown (non-positive pivot)    */
#define QDWHP_ERR_WORKSPACE      4  /* lwork smaller than the workspace query     */
#define QDWHP_ERR_HIP            5  /* a HIP runtime call failed                  */
#define QDWHP_ERR_NOCONV         6  /* small Jacobi solver did not converge       */

/* ---- selectors -------------------------------------------------------- */
#define QDWHP_LARGEST   0   /* wanted = k largest eigenvalues               */
#define QDWHP_SMALLEST  1   /* wanted = k smallest (Sec. 4.1: negate A)     */

#define QDWHP_FP64          0  /* every step in FP64                                  */
#define QDWHP_MIXED_FP32    1  /* Cholesky-step Gram/solve products in FP32 + polish  */

#define QDWHP_KIND_AUTO   0
#define QDWHP_KIND_QR     1    /* QR-based step, Eq. (2)       */
#define QDWHP_KIND_CHOL   2    /* Cholesky-based step, Eq. (3) */

/* ---- options (host struct; fill with qdwhp_opts_default) ------------- */
typedef struct {
  double   tol;            /* 0.05: threshold on |R_ii| (Sec. 4.1 after Theorem 1:
                              tol = Omega(1) trades ell against accuracy; the paper's
                              example value 0.01 leaves backward errors near 1e-13,
                              0.05 keeps them near 1e-14 for a few % larger ell)    */
  double   s_eig;          /* 0.2 : EIG shift / l_0 (Sec. 4.1, "Choosing s")         */
  int      eig_iters;      /* 3   : EIG iterations, type (27,26) (Sec. 4.1)          */
  double   kappa_max;      /* 100 : a step is QR-based when its bound on cond(Z)
                                    exceeds this (Sec. 4.2 advises QR when ill-conditioned) */
  int      svd_qr_first;   /* 1   : SVD step 0 QR-based (Table 1 counts one QR step)  */
  int      precision;      /* QDWHP_FP64, or QDWHP_MIXED_FP32: the Gram matrix and
                              the two triangular products of every Cholesky-based
                              step on FP32 matrix cores; QR-based steps, the
                              Cholesky-inversion, projector QR and Rayleigh-Ritz
                              stay FP64                                             */
  int      polish_steps;   /* 1   : FP64 polish steps after mixed iterations
                              (Newton-Schulz X(3I - X^T X)/2; EIG uses Halley's
                              (3,1,3) step when the unwanted side exceeds sqrt(3)) */
  uint64_t seed;           /* Philox key of the Lanczos start vectors               */
  int      lanczos_vectors;/* 8   : independent Lanczos runs of the estimator         */
  int      lanczos_steps;  /* 64  : steps per run (capped at n-1)                     */
  /* Replay / threshold overrides (NaN = choose automatically).  EIG: tau is
   * the threshold on the wanted side, mu > 0 the scale |mu|, rho the bound on
   * the unwanted side.  SVD: alpha ~ ||A||_2 and s the relative threshold. */
  double   tau, mu, rho;
  double   alpha, s_svd;
  int      kinds[16];      /* per-step QDWHP_KIND_*; QDWHP_KIND_AUTO = rule         */
} qdwhp_opts;

/* ---- per-call report (host struct) ------------------------------------ */
typedef struct {
  int64_t k;               /* number of returned pairs/triplets                     */
  int64_t ell;             /* subspace size n - ind + 1 (Sec. 4.1)                  */
  int64_t ind;             /* 1-based index of the first |R_ii| < tol               */
  int64_t n_above;         /* Rayleigh-Ritz values beyond the threshold             */
  double  tau, mu, rho;    /* EIG threshold, scale and unwanted-side bound          */
  double  alpha, s;        /* SVD norm estimate and relative threshold              */
  double  lmax, lmin;      /* estimator bounds (EIG: of A; SVD: of A^T A)           */
  int     n_iter;          /* DWH steps taken                                       */
  int     kinds[16];       /* QDWHP_KIND_QR / _CHOL per step                        */
  double  weights[16][3];  /* (a_k, b_k, c_k) per step (Sec. 3.1)                   */
  int     retries;         /* threshold retries (0 or 1)                            */
  int     jacobi_sweeps;   /* sweeps of the Rayleigh-Ritz Jacobi solver             */
  double  ms[8];           /* phase times: estimator, iterations, projector QR,
                              Q2, Rayleigh-Ritz products, small solve, vectors, total */
  double  flops_table1;    /* useful flops by the paper's Table 1 accounting        */
  int     status;          /* mirrors the return value                              */
} qdwhp_info;

void qdwhp_opts_default(qdwhp_opts* opts);
const char* qdwhp_strerror(int status);

/*
 * Workspace size in bytes (device memory, 256-byte aligned by the caller) for
 * a solve of the given shape.  Sized for the worst case ell = n, so a
 * successful query never under-sizes a call of the same shape and options.
 */
size_t qdwhp_eig_workspace(int64_t n, double fraction, const qdwhp_opts* opts);
size_t qdwhp_svd_workspace(int64_t m, int64_t n, int64_t k, const qdwhp_opts* opts);

/*
 * QDWHpartial-EIG (Algorithm 1): the k = floor(fraction*n + 1/2) (1 <= k <= n)
 * largest (which = QDWHP_LARGEST) or smallest (QDWHP_SMALLEST) eigenpairs of
 * the symmetric n x n matrix A.  Only the full matrix is read (both triangles);
 * A is not modified.  Outputs: w[k] (device; most wanted first: descending for
 * LARGEST, ascending for SMALLEST) and V (device, n x k, ldv >= n, orthonormal
 * eigenvectors, each column's largest-magnitude entry positive).  `info` may
 * be NULL.  Arguments: 1 A, 2 n, 3 lda, 4 fraction, 5 which, 6 w, 7 V, 8 ldv,
 * 9 work, 10 lwork, 11 opts (NULL = defaults), 12 stream, 13 info.
 */
int qdwhp_eig(const double* A, int64_t n, int64_t lda, double fraction, int which,
              double* w, double* V, int64_t ldv, void* work, size_t lwork,
              const qdwhp_opts* opts, void* stream, qdwhp_info* info);

/*
 * QDWHpartial-SVD (Algorithm 2): the k (1 <= k <= min(m,n)) largest singular
 * triplets of the m x n matrix A: A V = U diag(S).  Outputs (device): U
 * (m x k, ldu >= m), S[k] descending, V (n x k, ldv >= n); each column of V
 * has its largest-magnitude entry positive and U follows its sign.  m < n is
 * handled through A^T (Sec. 4.2).  Arguments: 1 A, 2 m, 3 n, 4 lda, 5 k, 6 U,
 * 7 ldu, 8 S, 9 V, 10 ldv, 11 work, 12 lwork, 13 opts, 14 stream, 15 info.
 */
int qdwhp_svd(const double* A, int64_t m, int64_t n, int64_t lda, int64_t k,
              double* U, int64_t ldu, double* S, double* V, int64_t ldv,
              void* work, size_t lwork, const qdwhp_opts* opts, void* stream,
              qdwhp_info* info);

/* ---- building blocks (same kernels as the solver; exported for tests and
 *      kernel-level measurement) ------------------------------------------ */

/*
 * C = alpha op(A) op(B) + beta C with op(X) = X (trans = 0) or X^T (1);
 * C is m x n, op(A) m x k, op(B) k x n, all column-major FP64 on the device.
 * The dense product behind every step of the method (Gram matrix of Eq. (3),
 * Q1 Q2^T of Eq. (2), the Rayleigh-Ritz projections of Algorithms 1 and 2).
 * flags bit 0 (QDWHP_GEMM_UPPER): compute only the 128x128 tiles of C that
 * meet the upper triangle (C square; the strictly-lower part of diagonal
 * tiles is written, other lower tiles are left untouched).
 * flags bit 1 (QDWHP_GEMM_F32): operands are rounded to FP32 and multiplied
 * on the FP32 matrix cores with FP32 accumulation; alpha, beta and C stay
 * FP64 (the mixed-precision Cholesky-based step).
 */
#define QDWHP_GEMM_UPPER 1
#define QDWHP_GEMM_F32   2
int qdwhp_dgemm(int transa, int transb, int64_t m, int64_t n, int64_t k,
                double alpha, const double* A, int64_t lda, const double* B,
                int64_t ldb, double beta, double* C, int64_t ldc, int flags,
                void* stream);

/*
 * In-place inverse of a symmetric positive definite n x n matrix Z through
 * its Cholesky factor Z = W^T W (W upper): on exit Z holds Z^{-1} (both
 * triangles).  This is the solve of the Cholesky-based step, Eq. (3), with
 * (X W^{-1}) W^{-T} = X Z^{-1}.  work: qdwhp_spd_inverse_workspace(n) bytes.
 * Returns QDWHP_ERR_CHOL if a pivot is not positive.
 */
size_t qdwhp_spd_inverse_workspace(int64_t n);
int qdwhp_spd_inverse(double* Z, int64_t n, int64_t ldz, void* work, size_t lwork,
                      void* stream);

/*
 * Householder QR without pivoting of the m x n matrix A (m >= n), in place:
 * R in the upper triangle, the essential parts of the reflectors below it,
 * tau[n] on the device (LAPACK geqrf layout).  Used on the stacked matrix of
 * Eq. (2) and on the spectral projector (Sec. 4.1, Theorem 1).
 * work: qdwhp_geqrf_workspace(m, n) bytes.
 */
size_t qdwhp_geqrf_workspace(int64_t m, int64_t n);
int qdwhp_geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau,
                void* work, size_t lwork, void* stream);

/*
 * Q(:, c0:c0+q) columns of Q = H_1 ... H_n from qdwhp_geqrf output, written
 * to Q (m x q, ldq >= m): applies the reflectors to the columns c0.. of the
 * identity (the thin Q of Eq. (2) for c0 = 0, q = n; the trailing columns Q2
 * of Algorithm 1 for c0 = ind - 1).  work: qdwhp_geqrf_workspace(m, n).
 */
int qdwhp_orgqr(const double* A, int64_t m, int64_t n, int64_t lda,
                const double* tau, int64_t c0, int64_t q, double* Q, int64_t ldq,
                void* work, size_t lwork, void* stream);

/*
 * All eigenpairs of the symmetric n x n matrix H by parallel-order block
 * Jacobi (the Rayleigh-Ritz solve of Algorithm 1): on exit w[n] holds the
 * eigenvalues in descending order and W (n x n, ldw >= n) the eigenvectors.
 * H is overwritten.  work: qdwhp_syev_workspace(n) bytes.
 */
size_t qdwhp_syev_workspace(int64_t n);
int qdwhp_syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw,
               void* work, size_t lwork, void* stream, int* sweeps);

/*
 * All singular triplets of the square n x n matrix R by one-sided block
 * Jacobi (the small SVD of Algorithm 2): R is overwritten by U diag(S),
 * S[n] descending, V (n x n).  work: qdwhp_gesvj_workspace(n) bytes.
 */
size_t qdwhp_gesvj_workspace(int64_t n);
int qdwhp_gesvj(double* R, int64_t n, int64_t ldr, double* S, double* V, int64_t ldv,
                void* work, size_t lwork, void* stream, int* sweeps);

/*
 * Kernel-level measurement: between qdwhp_profile_begin and
 * qdwhp_profile_end every launch of the FP64 MFMA GEMM kernel (the dense
 * products of Eqs. (2)-(3), Theorem 1's projector and the Rayleigh-Ritz step)
 * is bracketed by hipEvents on its own stream.  end synchronises those events
 * and returns the summed algorithmic flops (only the products the operation
 * needs: symmetric outputs count one triangle, triangular factors their
 * nonzero part), the summed kernel time in ms and the launch count.
 * Process-wide; not for concurrent use from several threads.
 */
void qdwhp_profile_begin(void);
int qdwhp_profile_end(double* flops, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* QDWHP_H */
