// Host-side scalar layer of the method (weights, schedules, threshold).
#include "dwh_sched.h"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace qdwhp {

static const double kUnitRoundoff = 1.1102230246251565e-16;   // 2^-53
// Sec. 4.2: for s << 1 ("say s < 1e-3") the first step should be QR-based.
static const double kQrFirstBelow = 1e-3;

void dwh_weights(double l, double* a, double* b, double* c) {
  if (l > 1.0) l = 1.0;
  const double l2 = l * l;
  const double dd = std::cbrt(4.0 * (1.0 - l2) / (l2 * l2));
  const double sqd = std::sqrt(1.0 + dd);
  const double aa = sqd + 0.5 * std::sqrt(8.0 - 4.0 * dd + 8.0 * (2.0 - l2) / (l2 * sqd));
  *a = aa;
  *b = (aa - 1.0) * (aa - 1.0) / 4.0;
  *c = aa + *b - 1.0;
}

double dwh_map(double x, double a, double b, double c) {
  const double x2 = x * x;
  return x * (a + b * x2) / (1.0 + c * x2);
}

std::vector<DwhStep> eig_schedule(double s, double rho, int iters, double kappa_max) {
  std::vector<DwhStep> out;
  double l = s;
  double x = std::max(1.0, (1.0 - s) * rho - s);
  for (int k = 0; k < iters; ++k) {
    DwhStep st;
    dwh_weights(l, &st.a, &st.b, &st.c);
    st.l = l; st.x = x;
    st.kind = (1.0 + st.c * x * x > kappa_max) ? 1 : 2;
    out.push_back(st);
    l = dwh_map(std::min(l, 1.0), st.a, st.b, st.c);
    x = std::max(1.0, dwh_map(x, st.a, st.b, st.c));
  }
  return out;
}

std::vector<DwhStep> svd_schedule(double s, double kappa_max, bool qr_first) {
  std::vector<DwhStep> out;
  if (s < kQrFirstBelow) qr_first = true;
  double l = s;
  while (std::fabs(l - 1.0) >= 5.0 * kUnitRoundoff && out.size() < 12) {
    DwhStep st;
    dwh_weights(l, &st.a, &st.b, &st.c);
    st.l = l; st.x = 1.0;
    st.kind = ((qr_first && out.empty()) || 1.0 + st.c > kappa_max) ? 1 : 2;
    out.push_back(st);
    l = dwh_map(std::min(l, 1.0), st.a, st.b, st.c);
  }
  return out;
}

int64_t target_count(int64_t n, int64_t k, int boost) {
  const int64_t extra = std::max<int64_t>(16, (k + 9) / 10);
  return std::min<int64_t>(n, (int64_t)boost * (k + extra));
}

bool cut_below(const std::vector<double>& nodes, const std::vector<double>& weights, int64_t n,
               int nv, double lmax, double lmin, int64_t kt, double* cut, bool nonneg) {
  if (kt >= n) return false;
  std::vector<size_t> order(nodes.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](size_t x, size_t y) { return nodes[x] > nodes[y]; });
  const double scale = (double)n / nv;
  double cum = 0.0;
  size_t j = order.size();
  for (size_t i = 0; i < order.size(); ++i) {
    cum += scale * weights[order[i]];
    if (cum >= (double)kt - 1e-9) { j = i; break; }
  }
  if (j == order.size()) return false;
  const double spread = std::max({lmax - lmin, std::fabs(lmax), std::fabs(lmin), 1e-300});
  const double tj = nodes[order[j]];
  // nonneg (nodes of A^T A, spanning many decades): distinct means more than
  // a relative 1e-6 below, and with no such node the cut is halfway to 0
  const double gap = nonneg ? 1e-6 * std::fabs(tj) : 1e-6 * spread;
  for (size_t i = j + 1; i < order.size(); ++i) {
    const double v = nodes[order[i]];
    if (v < tj - gap) { *cut = 0.5 * (tj + (nonneg ? std::max(v, 0.0) : v)); return true; }
  }
  if (nonneg && tj > 0.0) { *cut = 0.5 * tj; return true; }
  return false;
}

double eig_band_edge(const std::vector<DwhStep>& sched, double s, double tol) {
  auto image = [&](double y) {
    for (const DwhStep& st : sched) y = dwh_map(y, st.a, st.b, st.c);
    return y;
  };
  const double target = 2.0 * tol - 1.0;
  double lo = -s, hi = 0.0;
  if (!(image(lo) < target)) return lo;
  for (int it = 0; it < 200 && hi - lo > 1e-17; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (image(mid) < target) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

double eig_cost_flops(const std::vector<DwhStep>& sched, double n, double ell) {
  double f = 0.0;
  for (const DwhStep& st : sched) f += (st.kind == 1 ? 26.0 / 3.0 : 13.0 / 3.0) * n * n * n;
  const double j = std::max(0.0, n - ell);              // columns of the projector QR before ind
  f += 2.0 * n * j * j - 2.0 / 3.0 * j * j * j;
  f += 6.0 * n * n * ell + 9.0 * ell * ell * ell;        // A Q2, forming Q2, the small eigenproblem
  return f;
}

bool choose_tau_cost(const std::vector<double>& nodes, const std::vector<double>& weights, int64_t n, int nv,
                     double lmax, double lmin, int64_t kt, double s, int iters, double kappa_max, double tol,
                     double* tau, int* candidates) {
  if (candidates) *candidates = 0;
  if (kt >= n || nodes.empty()) return false;
  std::vector<size_t> order(nodes.size());
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](size_t x, size_t y) { return nodes[x] > nodes[y]; });
  const double scale = (double)n / nv;
  std::vector<double> th(order.size()), cum(order.size());
  double acc = 0.0;
  for (size_t i = 0; i < order.size(); ++i) {
    th[i] = nodes[order[i]];
    acc += scale * weights[order[i]];
    cum[i] = acc;
  }
  size_t j = th.size();
  for (size_t i = 0; i < th.size(); ++i)
    if (cum[i] >= (double)kt - 1e-9) { j = i; break; }
  if (j == th.size()) return false;
  const double spread = std::max({lmax - lmin, std::fabs(lmax), std::fabs(lmin), 1e-300});
  const double gap = 1e-6 * spread;
  auto count_above = [&](double t) {
    double c = 0.0;
    for (size_t i = 0; i < th.size() && th[i] >= t; ++i) c = cum[i];
    return c;
  };
  bool found = false;
  double best = 0.0;
  const double dn = (double)n;
  for (int cand = 0; cand < 4096; ++cand) {
    size_t nx = j + 1;
    while (nx < th.size() && !(th[nx] < th[j] - gap)) ++nx;
    if (nx >= th.size()) break;
    const double t = 0.5 * (th[j] + th[nx]);
    const double mu = std::max(lmax - t, 1e-3 * spread);
    const double rho = std::max(0.0, (t - lmin) / mu);
    const std::vector<DwhStep> sched = eig_schedule(s, rho, iters, kappa_max);
    const double edge = t - mu * (eig_band_edge(sched, s, tol) + s) / (1.0 - s);
    const double ell = std::min(dn, count_above(edge));
    const double cost = eig_cost_flops(sched, dn, ell);
    if (!found || cost < best * (1.0 - 1e-12)) { best = cost; *tau = t; found = true; }
    if (candidates) ++*candidates;
    j = nx;
  }
  return found;
}

// ---- Zolotarev steps ------------------------------------------------------
namespace {

constexpr long double kPiL = 3.14159265358979323846264338327950288L;

// Descending Landen (Gauss) transformation of the modulus k (complementary
// modulus kc = sqrt(1 - k^2), Abramowitz and Stegun 16.12, 17.5):
// k_{n+1} = (1 - kc_n)/(1 + kc_n), kc_{n+1} = 2 sqrt(kc_n)/(1 + kc_n), with
// 1 - k_{n+1} = 2 kc_n/(1 + kc_n) kept as well, so that a modulus next to 1
// (kc tiny) loses nothing to cancellation; stops once k_N < 1e-10 (then
// sn(v, k_N) = sin v to rounding).  Returns N; k[1..N], omk[1..N] = 1 - k.
// In long double: the coefficients decide the step count through
// |Z(l) - 1| < 5u, so they are carried to better than double accuracy.
int landen_chain(long double kc, long double* k, long double* omk) {
  int n = 0;
  long double kcn = kc;
  while (n < 40) {
    ++n;
    k[n] = (1.0L - kcn) / (1.0L + kcn);
    omk[n] = 2.0L * kcn / (1.0L + kcn);
    kcn = 2.0L * sqrtl(kcn) / (1.0L + kcn);
    if (k[n] < 1e-10L) break;
  }
  return n;
}

long double ellip_k_ld(long double kc) {
  long double k[41], omk[41];
  const int n = landen_chain(kc, k, omk);
  long double K = 0.5L * kPiL;
  for (int i = 1; i <= n; ++i) K *= 1.0L + k[i];
  return K;
}

void sncndn_ld(long double u, long double kc, long double* sn, long double* cn, long double* dn) {
  long double k[41], omk[41];
  const int n = landen_chain(kc, k, omk);
  long double v = u;
  for (int i = 1; i <= n; ++i) v /= 1.0L + k[i];
  long double s = sinl(v), c = cosl(v), d = 1.0L;
  for (int i = n; i >= 1; --i) {
    const long double den = 1.0L + k[i] * s * s;
    const long double s1 = (1.0L + k[i]) * s / den;
    const long double c1 = c * d / den;
    const long double d1 = (c * c + omk[i] * s * s) / den;
    s = s1; c = c1; d = d1;
  }
  *sn = s; *cn = c; *dn = d;
}

}  // namespace

// K(k) = (pi/2) prod_n (1 + k_n) over the Landen chain.
double ellip_k(double kc) { return (double)ellip_k_ld(kc); }

// sn, cn, dn by the Landen chain: v_n = u / prod_{i<=n} (1 + k_i); at the
// bottom sn = sin, cn = cos, dn = 1; then, going up with s, c, d of modulus
// k_{n+1}: D = 1 + k s^2, sn = (1 + k) s / D, cn = c d / D,
// dn = (1 - k s^2)/D = (c^2 + (1 - k) s^2)/D (the last form without the
// cancellation of 1 - k s^2 when k and s are both next to 1).
void jacobi_sncndn(double u, double kc, double* sn, double* cn, double* dn) {
  long double s, c, d;
  sncndn_ld(u, kc, &s, &c, &d);
  *sn = (double)s; *cn = (double)c; *dn = (double)d;
}

bool zolo_coeffs(double l, int r, ZoloStep* z) {
  if (!(l > 0.0 && l < 1.0) || r < 1 || r > kZoloMax) return false;
  const long double L = l;
  const long double kp = ellip_k_ld(L);        // K' = K(l'), l' = sqrt(1 - l^2): complementary modulus l
  const int d = 2 * r + 1;
  long double c[2 * kZoloMax];
  z->r = r;
  for (int i = 1; i <= 2 * r; ++i) {
    long double sn, cn, dn;
    if (2 * i <= d) {                          // argument below K'/2: c_i = l^2 sc^2(u)
      sncndn_ld(i * kp / d, L, &sn, &cn, &dn);
      c[i - 1] = L * L * (sn / cn) * (sn / cn);
    } else {                                   // u = K' - v: c_i = cs^2(v), v below K'/2
      sncndn_ld((d - i) * kp / d, L, &sn, &cn, &dn);
      c[i - 1] = (cn / sn) * (cn / sn);
    }
    z->c[i - 1] = (double)c[i - 1];
  }
  long double M = 1.0L;
  for (int j = 0; j < r; ++j) M *= (1.0L + c[2 * j]) / (1.0L + c[2 * j + 1]);
  z->M = (double)M;
  for (int j = 0; j < r; ++j) {
    const long double cj = c[2 * j];
    long double aj = c[2 * j + 1] - cj;
    for (int k = 0; k < r; ++k)
      if (k != j) aj *= (c[2 * k + 1] - cj) / (c[2 * k] - cj);
    z->a[j] = (double)aj;
  }
  // next lower bound from the extended-precision coefficients
  long double v = M * L;
  for (int j = 0; j < r; ++j) v *= (L * L + c[2 * j + 1]) / (L * L + c[2 * j]);
  z->l_next = (double)v;
  for (int i = 0; i < 2 * r; ++i)
    if (!std::isfinite(z->c[i]) || !(z->c[i] > 0.0)) return false;
  for (int j = 0; j < r; ++j)
    if (!std::isfinite(z->a[j])) return false;
  return std::isfinite(z->M) && z->M > 0.0 && std::isfinite(z->l_next);
}

double zolo_map(double x, const ZoloStep& z) {
  const double y = x * x;
  double v = z.M * x;
  for (int j = 0; j < z.r; ++j) v *= (y + z.c[2 * j + 1]) / (y + z.c[2 * j]);
  return v;
}

std::vector<ZoloStep> zolo_schedule(double s, int r, double kappa_max, double x0, bool qr_first) {
  std::vector<ZoloStep> sched;
  double l = s, x = std::max(1.0, x0);
  while (std::fabs(l - 1.0) >= 5.0 * kUnitRoundoff && sched.size() < 8) {
    ZoloStep z;
    if (!zolo_coeffs(std::min(l, 1.0 - 1e-16), r, &z)) break;
    z.l = l;
    z.x = x;
    for (int j = 0; j < r; ++j) {
      const bool force = qr_first && sched.empty();
      z.kinds[j] = (force || 1.0 + x * x / z.c[2 * j] > kappa_max) ? 1 : 2;
    }
    sched.push_back(z);
    l = std::min(z.l_next, 1.0);
    x = std::max(1.0, zolo_map(x, z));
  }
  return sched;
}

}  // namespace qdwhp
