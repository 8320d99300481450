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

}  // namespace qdwhp
