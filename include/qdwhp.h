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
#define QDWHP_PENDING          100  /* qdwhp_serve_poll: request not finished yet  */

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
                              tol = Omega(1) trades ell against accuracy).  The
                              paper's value 0.01 is accepted; with it the method
                              itself (as written, in plain FP64) leaves residuals
                              up to ~1.7e-13 ||A|| on kappa = 1e16 SVD inputs,
                              0.05 keeps them near 1e-14 for a few % larger ell  */
  double   s_eig;          /* 0.2 : EIG shift / l_0 (Sec. 4.1, "Choosing s")         */
  int      eig_iters;      /* 3   : EIG iterations, type (27,26) (Sec. 4.1)          */
  double   kappa_max;      /* 100 : a step is QR-based when its bound on cond(Z)
                                    exceeds this (Sec. 4.2 advises QR when ill-conditioned) */
  int      svd_qr_first;   /* 0   : SVD step 0 QR-based when s < 1e-3 (Sec. 4.2),
                                    any step QR-based while 1 + c_k > kappa_max;
                              1   : step 0 always QR-based (Table 1 counts one)     */
  int      precision;      /* QDWHP_FP64, or QDWHP_MIXED_FP32: the Gram matrix and
                              the two triangular products of every Cholesky-based
                              step except the last on FP32 matrix cores (the last
                              step, FP64, maps the wanted values back to FP64
                              accuracy); QR-based steps, the Cholesky-inversion,
                              projector QR and Rayleigh-Ritz stay FP64             */
  int      polish_steps;   /* 0   : extra FP64 polish steps after the iterations
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
  int      graphs;         /* 0   : 1 = run the DWH iterations as a captured hipGraph:
                              the first solve with given buffers, sizes and step kinds
                              records the launch sequence, later ones replay it with
                              new weights (pays off for repeated solves on one
                              workspace; results are identical either way)        */
  int      tau_policy;     /* 1   : EIG threshold by predicted cost: of the cuts at or
                                    below the plain one (a gap of the estimator's
                                    quadrature), the one whose step kinds and
                                    predicted subspace size cost the fewest flops by
                                    Table 1's accounting (a lower threshold can turn
                                    QR-based steps into Cholesky-based ones at the
                                    price of a larger ell);
                              0   : the plain cut (target count of the estimator)    */
  int      use_omega;      /* 0   : 1 = factor B Omega instead of the projector B,
                                    Omega an n x n Philox Gaussian (key seed + 3,
                                    entries of variance 1/n):
                                    the randomised rank-revealing QR of Sec. 4.1
                                    (costs one n^3 product more)                     */
  int      zolo_r;         /* 0   : DWH steps (Sec. 3.1);
                              r in 1..16: Zolotarev steps of type (2r+1, 2r), the
                                    higher-order rational functions named beside DWH
                                    (Sec. 3.1, Sec. 9), from l_0 = s until
                                    |l_k - 1| < 5u; each step is
                                    X+ = M (X + sum_j a_j X (X^T X + c_j I)^{-1}),
                                    its r terms Cholesky- or QR-based by the kappa_max
                                    rule (qdwhp_zolo_coeffs); FP64 only (precision,
                                    polish_steps, graphs and kinds are ignored), and
                                    the EIG threshold takes the plain cut (tau_policy
                                    is ignored); info->weights[k] = (M, r, l_k)       */
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
  int64_t rr_split;        /* EIG: size r of the exact spectral split of the
                              Rayleigh-Ritz matrix solved by Jacobi (0: the whole
                              ell x ell matrix was)                                */
} qdwhp_info;

void qdwhp_opts_default(qdwhp_opts* opts);
const char* qdwhp_strerror(int status);

/* QDWHpartial-EIG of a complex Hermitian matrix (Sec. 4: the Hermitian case
 * carries over from the real symmetric one with conjugate transposes).
 * A: n x n complex, interleaved (re, im) doubles, column-major, ld lda in
 * complex elements, read-only; the full matrix is read (Hermitian assumed).
 * k = floor(fraction n + 1/2) clamped to [1, n]; which as for qdwhp_eig.
 * Outputs (device, caller-owned): w[k] real (most wanted first), V (n x k
 * complex interleaved, ld ldv in complex elements), each column scaled so
 * that its largest-magnitude entry is real positive (lowest index on ties).
 * The solve runs the real path on the 2n x 2n real symmetric embedding
 * [Re A, -Im A; Im A, Re A] (every eigenvalue twice) and takes each cluster
 * of 2p real Ritz pairs back to p complex ones; info describes that real
 * solve (ell, kinds, ... of the embedding) with info->k = k.  work:
 * qdwhp_heig_workspace(n, fraction, opts) bytes.  Returns 0, -i for a bad
 * argument i, or QDWHP_ERR_* (QDWHP_ERR_NO_SUBSPACE also when a cluster
 * yields fewer complex vectors than its share). */
size_t qdwhp_heig_workspace(int64_t n, double fraction, const qdwhp_opts* opts);
int qdwhp_heig(const double* A, int64_t n, int64_t lda, double fraction, int which, double* w,
               double* V, int64_t ldv, void* work, size_t lwork, const qdwhp_opts* opts,
               void* stream, qdwhp_info* info);

/* Coefficients of the Zolotarev step of type (2r+1, 2r) for lower bound l
 * (host only, no GPU): c[2r] (c_1 .. c_2r), a[r] (partial fractions), *M and
 * *l_next = Z(l), Z(x) = M x prod_j (x^2 + c_{2j}) / (x^2 + c_{2j-1}), the
 * best approximation of sign on [l, 1] scaled to max 1 (Sec. 3.1 names these
 * beside DWH; r = 1 is the DWH map).  Returns 0, or -1 / -2 for l outside
 * (0, 1) / r outside 1..16, or QDWHP_ERR_NONFINITE. */
int qdwhp_zolo_coeffs(double l, int r, double* c, double* a, double* M, double* l_next);

/*
 * Workspace size in bytes (device memory, 256-byte aligned by the caller) for
 * a solve of the given shape.  Sized for the worst case ell = n, so a
 * successful query never under-sizes a call of the same shape and options.
 */
size_t qdwhp_eig_workspace(int64_t n, double fraction, const qdwhp_opts* opts);
size_t qdwhp_svd_workspace(int64_t m, int64_t n, int64_t k, const qdwhp_opts* opts);

/*
 * The number of eigenpairs that qdwhp_eig, qdwhp_eig_noalloc and qdwhp_heig
 * return for this n and fraction: k = floor(fraction*n + 1/2) clamped to
 * 1 <= k <= n (Algorithms 1 and 2 take k as given; a fraction of the order
 * is how the experiments of Sec. 7 state it).  Host only; 0 when n < 1 or
 * fraction is outside (0, 1], which those calls reject.  Callers size w and
 * V from it.
 */
int64_t qdwhp_eig_count(int64_t n, double fraction);

/*
 * QDWHpartial-EIG (Algorithm 1): the k = floor(fraction*n + 1/2) (1 <= k <= n)
 * largest (which = QDWHP_LARGEST) or smallest (QDWHP_SMALLEST) eigenpairs of
 * the symmetric n x n matrix A.  Only the full matrix is read (both triangles);
 * A is not modified.  Outputs: w[k] (device; most wanted first: descending for
 * LARGEST, ascending for SMALLEST) and V (device, n x k, ldv >= n, orthonormal
 * eigenvectors, each column's largest-magnitude entry positive).  `info` may
 * be NULL.  Arguments: 1 A, 2 n, 3 lda, 4 fraction, 5 which, 6 w, 7 V, 8 ldv,
 * 9 work, 10 lwork, 11 opts (NULL = defaults), 12 stream, 13 info.
 * A large ell x ell Rayleigh-Ritz matrix (tuning keys "rr.split_min",
 * "rr.split_pct") is first split exactly by the polar factor of a shifted
 * copy (Sec. 3.2) and only its wanted block goes to Jacobi; the split is
 * verified and otherwise the whole matrix is solved, so results meet the
 * same bounds either way (info->rr_split reports which).
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
 * flags bit 0 (QDWHP_GEMM_UPPER): C is square and only its upper triangle
 * is defined on exit (only the output tiles meeting it are computed; parts
 * of the strictly-lower triangle may be overwritten).
 * flags bit 1 (QDWHP_GEMM_F32): operands are rounded to FP32 and multiplied
 * on the FP32 matrix cores, the FP32 sums folded into FP64 every 32 terms of
 * k; alpha, beta and C stay FP64 (the mixed-precision Cholesky-based step).
 * Leading dimensions must be below 2^21 (QDWHP_ERR_HIP otherwise).  The
 * result does not depend on the tile size chosen (tuning key
 * "gemm.small_tiles").
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
 * work: qdwhp_geqrf_workspace(m, n) bytes.  Panels factored by the
 * reconstruction path hand the wide part of their trailing update to a
 * library-owned helper stream; the call's stream waits for it before the
 * call returns, so the result is ordered on `stream` as usual.
 */
size_t qdwhp_geqrf_workspace(int64_t m, int64_t n);
int qdwhp_geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau,
                void* work, size_t lwork, void* stream);

/*
 * Q(:, c0:c0+q) columns of Q = H_1 ... H_n from qdwhp_geqrf output, written
 * to Q (m x q, ldq >= m; q <= n, c0 + q <= m, else -7: the workspace holds
 * block products for at most n columns): applies the reflectors to the columns c0.. of the
 * identity (the thin Q of Eq. (2) for c0 = 0, q = n; the trailing columns Q2
 * of Algorithm 1 for c0 = ind - 1).  work must be the workspace of the
 * qdwhp_geqrf call that factored A, unchanged since: it holds the block
 * reflector (T) factors, which carry tau (the tau argument is not read).
 */
int qdwhp_orgqr(const double* A, int64_t m, int64_t n, int64_t lda,
                const double* tau, int64_t c0, int64_t q, double* Q, int64_t ldq,
                void* work, size_t lwork, void* stream);

/*
 * All eigenpairs of the symmetric n x n matrix H by parallel-order block
 * Jacobi (the Rayleigh-Ritz solve of Algorithm 1): on exit w[n] holds the
 * eigenvalues in descending order and W (n x n, ldw >= n) the eigenvectors.
 * H is read only (both triangles).  work: qdwhp_syev_workspace(n) bytes.
 * Stopping rule, with tol = 2u ||H||_F / sqrt(n): the largest off-diagonal
 * entry after a sweep is within 32 tol, or the largest seen during a sweep
 * is at or below tol, or within 32 tol and no longer falling by 4x (the
 * rounding floor).  *sweeps (optional) receives the sweep count;
 * QDWHP_ERR_NOCONV if the rule was not met within 60 sweeps.
 */
size_t qdwhp_syev_workspace(int64_t n);
int qdwhp_syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw,
               void* work, size_t lwork, void* stream, int* sweeps);

/*
 * All singular triplets of the square n x n matrix R by one-sided block
 * Jacobi (the small SVD of Algorithm 2): R is overwritten by U (columns
 * of unit norm, ordered like S), S[n] descending, V (n x n, ldv >= n).
 * work: qdwhp_gesvj_workspace(n) bytes.  *sweeps (optional) receives the
 * sweep count; QDWHP_ERR_NOCONV if the stopping rule was not met within 60
 * sweeps.
 */
size_t qdwhp_gesvj_workspace(int64_t n);
int qdwhp_gesvj(double* R, int64_t n, int64_t ldr, double* S, double* V, int64_t ldv,
                void* work, size_t lwork, void* stream, int* sweeps);

/* ---- ragged batches ---------------------------------------------------- */
#define QDWHP_PROBLEM_EIG  0
#define QDWHP_PROBLEM_SVD  1

/*
 * One independent problem: the arguments of qdwhp_eig (type EIG: A n x n,
 * fraction, which, w, V) or of qdwhp_svd (type SVD: A m x n, k, w = S, U, V).
 * Fields a type does not use are ignored.  Device pointers, column-major.
 */
typedef struct {
  int type;                  /* QDWHP_PROBLEM_EIG or QDWHP_PROBLEM_SVD                 */
  int which;                 /* EIG: QDWHP_LARGEST / QDWHP_SMALLEST                    */
  int64_t m, n;              /* SVD: m x n; EIG: n x n (m ignored)                     */
  const double* A; int64_t lda;
  double fraction;           /* EIG: k = floor(fraction n + 1/2), clamped to [1, n]     */
  int64_t k;                 /* SVD: number of wanted triplets                          */
  double* w;                 /* EIG eigenvalues / SVD singular values, length k         */
  double* U; int64_t ldu;    /* SVD left singular vectors (m x k); unused for EIG       */
  double* V; int64_t ldv;    /* EIG eigenvectors / SVD right singular vectors (n x k)   */
} qdwhp_problem;

/* Workspace bytes of one problem (qdwhp_eig_workspace / qdwhp_svd_workspace
 * of its type); 0 for an invalid type. */
size_t qdwhp_problem_workspace(const qdwhp_problem* p, const qdwhp_opts* opts);

/*
 * Solves `count` independent problems of uneven sizes (Algorithms 1 and 2
 * applied to each).  Instances run concurrently on `lanes` streams driven by
 * host threads (0: the tuned default, "batch.lanes"); each uses its own slice
 * of `work`.  The final products V = Q2 W of all instances run as one
 * persistent ragged GEMM launch on `stream`.  Every instance's results are
 * bitwise identical to a standalone qdwhp_eig / qdwhp_svd call with the same
 * options.  infos[i] / status[i] (optional, host arrays of `count`) receive
 * each instance's report and status; the return value is 0 if all succeeded,
 * else the first failing instance's status (or a negative argument index).
 * Synchronises `stream` like the single-problem calls; lanes start after the
 * work already queued on `stream`.
 */
size_t qdwhp_batched_workspace(int count, const qdwhp_problem* probs, const qdwhp_opts* opts);
int qdwhp_batched(int count, const qdwhp_problem* probs, void* work, size_t lwork,
                  const qdwhp_opts* opts, int lanes, void* stream, qdwhp_info* infos,
                  int* status);

/*
 * Persistent ragged GEMM: C_i = alpha_i op(A_i) op(B_i) + beta_i C_i for
 * i < count in one launch (shared transposes; m, n, k, alpha, A, lda, B, ldb,
 * beta, C, ldc are host arrays of `count` entries holding sizes, scalars and
 * device pointers).  Tiles of all problems form one list that a fixed grid
 * walks; each tile is computed exactly as by qdwhp_dgemm.  work: device
 * memory of qdwhp_dgemm_grouped_workspace(count) bytes for the descriptor
 * table.  Leading dimensions must be below 2^21.
 */
size_t qdwhp_dgemm_grouped_workspace(int count);
int qdwhp_dgemm_grouped(int count, int transa, int transb, const int64_t* m, const int64_t* n,
                        const int64_t* k, const double* alpha, const double* const* A,
                        const int64_t* lda, const double* const* B, const int64_t* ldb,
                        const double* beta, double* const* C, const int64_t* ldc,
                        void* work, size_t lwork, void* stream);

/* ---- continuous-batching server --------------------------------------- */
/*
 * A server owns one device arena of `arena_bytes` (its only allocation, made
 * here) and `lanes` worker threads with their own streams (0: the tuned
 * default, "serve.lanes").  submit() queues a problem (the descriptor is
 * copied; its buffers must stay valid until the request finishes) and
 * returns a ticket.  Requests are admitted in FIFO order when a lane is free
 * and the request's workspace fits in a free range of the arena.  An
 * admitted request's phases (setup, DWH iterations, subspace and
 * Rayleigh-Ritz) are taken by whichever lane is free; the iterations of all
 * requests of one shape (type, rows, columns) waiting at the same time run
 * as one group of grouped launches.  A request larger than the arena
 * finishes at once with QDWHP_ERR_WORKSPACE.  poll() returns QDWHP_PENDING
 * while the request runs (wait = 0) or blocks until it finishes (wait != 0);
 * a finished request returns its status, fills info, the latency from
 * submit to results ready and the time it queued (ms, host clock), and its
 * ticket is released.  destroy() finishes every queued request, then frees
 * the arena.  Results equal those of a standalone call bitwise, alone or in
 * any mix ("serve.grouped" = 0 runs every phase of a request on one lane).
 */
typedef struct qdwhp_server qdwhp_server;
int qdwhp_serve_create(size_t arena_bytes, int lanes, const qdwhp_opts* opts, qdwhp_server** srv);
int qdwhp_serve_submit(qdwhp_server* srv, const qdwhp_problem* p, int64_t* ticket);
int qdwhp_serve_poll(qdwhp_server* srv, int64_t ticket, int wait, qdwhp_info* info,
                     double* latency_ms, double* queue_ms);
int qdwhp_serve_destroy(qdwhp_server* srv);
/* Counters since creation or the last reset: the largest sum of the
 * footprints of requests running at once (bytes of the arena in use, i.e.
 * the server's HBM high-water mark inside its arena), the arena size (open
 * to requests), the most requests running at once, and the number of
 * iteration groups run with the number of requests they held (same-shape
 * requests waiting together share one group).  reset != 0 restarts the
 * marks from the current state and the group counts from zero.  Any pointer
 * may be NULL. */
int qdwhp_serve_stats(qdwhp_server* srv, size_t* peak_bytes, size_t* arena_bytes, int* peak_running,
                      int64_t* groups, int64_t* grouped_requests, int reset);

/* ---- full spectrum by QDWH-based spectral divide and conquer ---------- */
/*
 * All eigenpairs of the symmetric n x n matrix H (device, ld ldh, read only)
 * by the QDWH-EIG recursion (Sec. 3.2): a shift sigma at the median of the
 * spectrum (the count of a Lanczos quadrature), the sign function of
 * (H - sigma I)/alpha by a converged QDWH polar decomposition, orthonormal
 * bases of the ranges of the two spectral projectors (I +/- sign)/2, and the
 * same on the two restricted matrices, down to blocks of at most "dc.leaf"
 * rows (default 512), solved by block Jacobi.  A split whose check fails
 * (a column of H Q - Q Q^T H Q above 5e-14 ||H||) falls back to Jacobi on
 * that block.  Outputs: w[n] descending, W (n x n, ld ldw) eigenvectors.
 * levels (may be NULL) gets the recursion depth reached.  Workspace:
 * qdwhp_syev_dc_workspace(n) bytes.  Errors as for qdwhp_syev.
 */
size_t qdwhp_syev_dc_workspace(int64_t n);
int qdwhp_syev_dc(const double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw,
                  void* work, size_t lwork, void* stream, int* levels);

/* ---- solve without allocation ------------------------------------------ */
/*
 * For callers that cannot allocate device memory (code between graph-capture
 * boundaries, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as qdwhp_eig, arguments 1-8 and opts/stream/info alike, but with no
 * workspace argument.  The workspace is a fixed array of
 * QDWHP_NOALLOC_MAX_BYTES (128 MiB) that the library holds in the memory of
 * every GPU it runs on until the process ends (enough for n up to about
 * 1200); a problem whose qdwhp_eig_workspace exceeds it returns
 * QDWHP_ERR_WORKSPACE before any device work.  The call allocates nothing:
 * no device or pinned memory, no events, streams or graphs (info->ms stays
 * zero, opts->graphs is ignored).  Results equal those of qdwhp_eig bitwise.
 * Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents: calls that overlap on a GPU (from several threads or
 * streams) race and must be serialised by the caller.
 */
#define QDWHP_NOALLOC_MAX_BYTES (128u << 20)
size_t qdwhp_noalloc_max_bytes(void);
int qdwhp_eig_noalloc(const double* A, int64_t n, int64_t lda, double fraction, int which,
                      double* w, double* V, int64_t ldv, const qdwhp_opts* opts, void* stream,
                      qdwhp_info* info);

/* ---- tuning table ------------------------------------------------------ */
/*
 * Captured launch sequences (opts->graphs = 1) are kept per key (the
 * workspace buffers, sizes, step kinds and precision plan of a solve) so
 * that later solves on the same workspace replay them; they hold device
 * resources until the process ends.  qdwhp_graphs_clear waits for the
 * device (hipDeviceSynchronize, so no replay still runs) and destroys them
 * all; call it after freeing a workspace that solves with graphs used, or
 * to release the memory.  Returns 0 or QDWHP_ERR_HIP.  Later solves with
 * graphs = 1 capture again.  qdwhp_graphs_count: the number kept (host
 * only).  Neither may overlap a solve on another host thread.
 */
int qdwhp_graphs_clear(void);
int64_t qdwhp_graphs_count(void);

/*
 * Named integer parameters read by launch-shape decisions, written by the
 * autotuner (or by hand).  Keys: "gemm.small_tiles" (a GEMM whose 128x128
 * tile count is below this value runs with 64x64 tiles; default 96; GEMMs
 * with k <= 128 and FP32-operand GEMMs always take 64x64 tiles),
 * "batch.lanes" (default 8), "serve.lanes" (default 8), "jacobi.fused_max"
 * (two-sided Jacobi problems up to this size update H and V in one launch
 * per round; default 2048), "rr.split_min" and "rr.split_pct" (EIG
 * Rayleigh-Ritz matrices of at least split_min rows (default 3000) whose
 * wanted part, with a margin of max(16, k/32), is at most split_pct percent
 * of them (default 85) are first split exactly at a Lanczos-placed shift by
 * a converged QDWH polar decomposition, and only the wanted block goes to
 * Jacobi), "rr.svd_polar" (SVD Rayleigh-Ritz factors of at least this many
 * rows, default 256, are decomposed the QDWH-SVD way, Sec. 3.2: a converged
 * polar decomposition, then the symmetric eigenproblem of its Hermitian
 * factor; smaller ones, or 0, by one-sided Jacobi), "batch.grouped" and
 * "serve.grouped" (1, default: the iterations of same-shape instances run
 * as grouped launches; 0: each on its own lane), "qr.recon" (1, default:
 * Householder QR panels by Cholesky QR with Householder reconstruction
 * where they pass its checks; 0: one launch per column), "qr.stacked" (1,
 * default: the QR of [sqrt(c) X; I] in a QR-based step skips the rows of
 * the identity block that no reflector has reached; 0: the full stacked
 * matrix; the recon choice is read per panel height h as "qr.recon@b",
 * b = ceil(log2 h), when set), "qr.overlap" (1, default: with the
 * reconstruction path, the trailing update beyond the next panel runs on a
 * helper stream while the next panel is factored; 0: all on the call's
 * stream; the two agree to rounding), "rr.split2_min" (0, default: off;
 * from this many rows the wanted block of the Rayleigh-Ritz split is split
 * once more at the median of its spectrum, Jacobi on both halves, when at
 * least "rr.split2_pct" percent of it (12) lies in tight clusters by the
 * estimator's quadrature), "gemm.shallow_k" (GEMMs with k at most this
 * run 64x64 tiles; default 128), "batch.lanes.mixed" (lanes of a batch in
 * mixed precision; default batch.lanes).  Unset keys keep
 * their defaults.  Values apply to calls made after they are set.
 */
int qdwhp_tune_set(const char* key, int64_t value);
int64_t qdwhp_tune_get(const char* key, int64_t fallback);
/* Size-bucketed lookup: the value of "key@b" for b = ceil(log2(size)) when
 * set, else of "key", else fallback (sized keys: "qr.recon@b" by panel
 * height, "gemm.shallow_k" by none; see above). */
int64_t qdwhp_tune_get_sized(const char* key, int64_t size, int64_t fallback);
void qdwhp_tune_clear(void);

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
