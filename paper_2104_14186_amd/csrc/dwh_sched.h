// Host-side scalar layer: DWH weights, step schedules, threshold placement.
#pragma once
#include <cstdint>
#include <vector>

namespace qdwhp {

struct DwhStep {
  double a, b, c;    // weights of r(x) = x (a + b x^2) / (1 + c x^2)
  double l;          // lower bound l_k before the step
  double x;          // bound on the largest singular value before the step
  int kind;          // 1 = QR-based (Eq. (2)), 2 = Cholesky-based (Eq. (3))
};

// Weights of the scaled Zolotarev (3,2) approximation of sign on [l, 1]
// (Sec. 3.1; closed form as in Algorithm 3), with l clamped to <= 1.
void dwh_weights(double l, double* a, double* b, double* c);
double dwh_map(double x, double a, double b, double c);

// Algorithm 1: `iters` steps from l_0 = s; kinds from the bound
// 1 + c_k x_k^2 on cond(Z_k) against kappa_max.
std::vector<DwhStep> eig_schedule(double s, double rho, int iters, double kappa_max);
// Algorithm 2: steps from l_0 = s until |l_k - 1| < 5u; step 0 QR-based when
// qr_first or s < 1e-3 (Sec. 4.2), any step QR-based while 1 + c_k > kappa_max
// (1 + c_k bounds cond(I + c_k X^T X) since the singular values of X_k lie in
// [0, 1]).
std::vector<DwhStep> svd_schedule(double s, double kappa_max, bool qr_first);

// Zolotarev steps of type (2r+1, 2r): the higher-order rational functions
// the paper names beside DWH (Sec. 3.1; Sec. 9).  Z(x) = M x prod_j (x^2 +
// c_{2j}) / (x^2 + c_{2j-1}) is the best approximation of sign on [l, 1]
// scaled to max 1 (r = 1: the DWH map), with c_i = l^2 sc^2(i K'/(2r+1); l')
// (l' = sqrt(1 - l^2), K' = K(l')) and M = prod_j (1 + c_{2j-1})/(1 + c_{2j})
// (Nakatsukasa and Freund, SIAM Review 58, 2016).  One step is
// X+ = M (X + sum_j a_j X (X^T X + c_{2j-1} I)^{-1}), the a_j the partial
// fractions of the product in x^2.
constexpr int kZoloMax = 16;
struct ZoloStep {
  int r = 0;
  double M = 0.0;
  double c[2 * kZoloMax] = {};   // c_1 .. c_2r
  double a[kZoloMax] = {};       // a_1 .. a_r
  int kinds[kZoloMax] = {};      // per term: 1 = QR form, 2 = Cholesky form
  double l = 0.0, x = 1.0;       // lower bound and bound on the largest value before the step
  double l_next = 0.0;           // Z(l), from the coefficients in extended precision
};
// Jacobi's sn, cn, dn of argument u for the modulus k = sqrt(1 - kc^2), given
// the complementary modulus kc in (0, 1] (so that k next to 1 keeps its
// accuracy), and K(k): descending Landen transformation (Abramowitz and
// Stegun 16.12, 17.5).
void jacobi_sncndn(double u, double kc, double* sn, double* cn, double* dn);
double ellip_k(double kc);
// Coefficients (and l_next = Z(l)) for lower bound l in (0, 1), computed in
// long double and stored in double; false when they are not finite.
bool zolo_coeffs(double l, int r, ZoloStep* z);
double zolo_map(double x, const ZoloStep& z);
// Steps from l_0 = s until |l_k - 1| < 5u (at most 8).  A term is QR-based
// when 1 + x_k^2 / c_{2j-1} (its bound on cond(I + X^T X / c_{2j-1})) exceeds
// kappa_max, every term of step 0 when qr_first; x_0 = x0 and
// x_{k+1} = max(1, Z(x_k)) (x0 = 1 for the SVD).
std::vector<ZoloStep> zolo_schedule(double s, int r, double kappa_max, double x0, bool qr_first);

// Threshold below the pooled Lanczos quadrature node at which the estimated
// count first reaches kt; returns false when the count never reaches kt.
// nonneg: nodes of A^T A (>= 0, many decades): distinctness is relative to
// the node and, without a distinct node below, the cut is half the node.
bool cut_below(const std::vector<double>& nodes, const std::vector<double>& weights, int64_t n,
               int nv, double lmax, double lmin, int64_t kt, double* cut, bool nonneg = false);
int64_t target_count(int64_t n, int64_t k, int boost);

// Scaled value y in (-s, 0) at which the composite map of an EIG schedule
// reaches 2 tol - 1, i.e. where (r(y) + 1)/2 = tol: eigenvalues with scaled
// values above it form the band that the projector keeps besides the
// wanted ones (Sec. 4.1, "Choosing s" and "Choosing the subspace size").
double eig_band_edge(const std::vector<DwhStep>& sched, double s, double tol);
// Flops of a solve by the Table 1 accounting: the steps, the projector QR
// up to column n - ell, A Q2 and forming Q2 (6 n^2 ell), the ell x ell
// eigenproblem (9 ell^3).
double eig_cost_flops(const std::vector<DwhStep>& sched, double n, double ell);
// Threshold policy by predicted cost: every cut at or below the plain one
// (cut_below for kt) that falls in a gap between distinct quadrature nodes
// is a candidate; each is scored by eig_cost_flops with its step kinds (the
// kappa rule of eig_schedule) and its predicted subspace size (the
// quadrature count above the band edge).  The cheapest wins, ties go to the
// higher cut.  Returns false when the count never reaches kt.
bool choose_tau_cost(const std::vector<double>& nodes, const std::vector<double>& weights, int64_t n, int nv,
                     double lmax, double lmin, int64_t kt, double s, int iters, double kappa_max, double tol,
                     double* tau, int* candidates = nullptr);

}  // namespace qdwhp
