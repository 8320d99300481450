// C ABI: options, error strings and the building-block entry points.
#include <cmath>
#include <cstring>
#include <limits>

#include "qdwhp.h"
#include "common.h"
#include "dwh_sched.h"

using namespace qdwhp;

extern "C" void qdwhp_opts_default(qdwhp_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  const double nan = std::numeric_limits<double>::quiet_NaN();
  o->tol = 0.05;
  o->s_eig = 0.2;
  o->eig_iters = 3;
  o->kappa_max = 100.0;
  o->svd_qr_first = 0;
  o->precision = QDWHP_FP64;
  o->polish_steps = 0;
  o->seed = 0;
  o->lanczos_vectors = 8;
  o->lanczos_steps = 64;
  o->tau = o->mu = o->rho = nan;
  o->alpha = o->s_svd = nan;
  for (int i = 0; i < 16; ++i) o->kinds[i] = QDWHP_KIND_AUTO;
  o->tau_policy = 1;
  o->use_omega = 0;
  o->zolo_r = 0;
}

extern "C" int qdwhp_zolo_coeffs(double l, int r, double* c, double* a, double* M, double* l_next) {
  if (!(l > 0.0 && l < 1.0)) return -1;
  if (r < 1 || r > kZoloMax) return -2;
  ZoloStep z;
  if (!zolo_coeffs(l, r, &z)) return QDWHP_ERR_NONFINITE;
  for (int i = 0; i < 2 * r && c; ++i) c[i] = z.c[i];
  for (int j = 0; j < r && a; ++j) a[j] = z.a[j];
  if (M) *M = z.M;
  if (l_next) *l_next = std::fmin(z.l_next, 1.0);
  return 0;
}

extern "C" const char* qdwhp_strerror(int st) {
  if (st < 0) return "invalid argument";
  switch (st) {
    case QDWHP_OK: return "success";
    case QDWHP_ERR_NONFINITE: return "non-finite value in input or iterate";
    case QDWHP_ERR_NO_SUBSPACE: return "no subspace: fewer than k certified values";
    case QDWHP_ERR_CHOL: return "Cholesky breakdown";
    case QDWHP_ERR_WORKSPACE: return "workspace too small";
    case QDWHP_ERR_HIP: return "HIP runtime error";
    case QDWHP_ERR_NOCONV: return "Jacobi solver did not converge";
    default: return "unknown status";
  }
}

extern "C" int qdwhp_dgemm(int transa, int transb, int64_t m, int64_t n, int64_t k,
                           double alpha, const double* A, int64_t lda, const double* B,
                           int64_t ldb, double beta, double* C, int64_t ldc, int upper,
                           void* stream) {
  if (transa != 0 && transa != 1) return -1;
  if (transb != 0 && transb != 1) return -2;
  if (m < 0) return -3;
  if (n < 0) return -4;
  if (k < 0) return -5;
  if (lda < (transa ? (k > 1 ? k : 1) : (m > 1 ? m : 1))) return -8;
  if (ldb < (transb ? (n > 1 ? n : 1) : (k > 1 ? k : 1))) return -10;
  if (ldc < (m > 1 ? m : 1)) return -13;
  if ((upper & 1) && m != n) return -14;
  if (m == 0 || n == 0) return QDWHP_OK;
  if ((k > 0 && (!A || !B)) || !C) return -7;
  try {
    Gemm g;
    g.M = m; g.N = n; g.K = k; g.alpha = alpha; g.beta = beta;
    g.A = A; g.lda = lda; g.ta = transa;
    g.B = B; g.ldb = ldb; g.tb = transb;
    g.C = C; g.ldc = ldc;
    g.tiles = (upper & 1) ? TILES_UPPER : TILES_ALL;
    g.f32 = (upper & 2) != 0;
    dgemm(g, (hipStream_t)stream);
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}
