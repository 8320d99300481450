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

}  // namespace qdwhp
