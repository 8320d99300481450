// QDWHpartial-EIG (Algorithm 1) and QDWHpartial-SVD (Algorithm 2) drivers and
// the building-block entry points of the C ABI.
//
// Every matrix step runs in the library's HIP kernels; the host computes the
// scalar schedule (Sec. 3.1 weights), places the threshold from the Lanczos
// quadrature nodes, and reads back two data-dependent quantities: the
// estimator's Ritz data (to fix tau / s and the step kinds) and diag(R) of the
// projector QR (to fix ind and ell, Sec. 4.1 "Choosing the subspace size").
#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <limits>
#include <memory>
#include <thread>
#include <vector>

#include "qdwhp.h"
#include "common.h"
#include "drivers.h"
#include "dwh_sched.h"
#include "graphs.h"
#include "elem.h"
#include "jacobi.h"
#include "lanczos.h"
#include "skinny.h"
#include "qr.h"

using namespace qdwhp;

namespace {

struct WorkspaceError {};

// Bump allocator over the caller's workspace; with base == nullptr it only
// measures, so the size query and the solve share one carving routine.
struct Arena {
  char* base; size_t cap; size_t off = 0;
  Arena(void* b, size_t c) : base((char*)b), cap(c) {}
  double* take(int64_t count) {
    const size_t bytes = ((size_t)(count > 0 ? count : 1) * 8 + 255) / 256 * 256;
    if (base && off + bytes > cap) throw WorkspaceError{};
    double* p = base ? (double*)(base + off) : nullptr;
    off += bytes;
    return p;
  }
};

struct Events {
  hipEvent_t ev[9];
  bool on = false;
  int used = 0;
  explicit Events(bool enable) {
    if (!enable || no_alloc_mode()) return;
    for (auto& e : ev) QDWHP_HIP(hipEventCreate(&e));
    on = true;
  }
  ~Events() {
    if (on) for (auto& e : ev) (void)hipEventDestroy(e);
  }
  void mark(int i, hipStream_t s) {
    if (on) { QDWHP_HIP(hipEventRecord(ev[i], s)); used = std::max(used, i + 1); }
  }
  void fill(double* ms) {
    if (!on) return;
    QDWHP_HIP(hipEventSynchronize(ev[used - 1]));
    for (int i = 0; i + 1 < used && i < 7; ++i) {
      float t = 0.f;
      QDWHP_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
      ms[i] = t;
    }
    float tot = 0.f;
    QDWHP_HIP(hipEventElapsedTime(&tot, ev[0], ev[used - 1]));
    ms[7] = tot;
  }
};

bool is_nan(double x) { return std::isnan(x); }

int64_t lz_steps(const qdwhp_opts& o, int64_t n) {
  int64_t m = o.lanczos_steps > 0 ? o.lanczos_steps : 64;
  if (m > 126) m = 126;
  if (m > n - 1) m = n - 1;
  return m < 1 ? 1 : m;
}
int lz_vectors(const qdwhp_opts& o) { return o.lanczos_vectors > 0 ? std::min(o.lanczos_vectors, 32) : 8; }

// ---------------------------------------------------------------------------
// DWH steps on X (m x n, ld m).  X and Xn are exchanged by the Cholesky step.
struct StepBufs {
  double* Z;        // n x n
  double* spd;      // spd_inverse_doubles(n), then the step's product and FP32 staging
  int64_t spd_doubles = 0;   // size of that region (0: unknown, no FP32 staging)
  double* W;        // (m + n) x n stacked matrix
  double* Q;        // (m + n) x n thin Q
  double* tau;      // m + n
  double* Tall;     // qr_t_doubles(n)
  QrScratch qrs;
  int* flag;
  double* G = nullptr;   // n x n, Zolotarev steps only
};

// Eq. (3): Z = I + c X^T X = W^T W, X+ = (b/c) X + (a - b/c) (X W^{-1}) W^{-T}.
// W^{-1} comes from the recursive Cholesky-inversion; the two solves are
// triangular products (W^{-1} upper: X W^{-1} only needs k <= column,
// (.) W^{-T} only k >= column).  For symmetric X (EIG) only the upper tiles
// of the result are formed and then mirrored.
//
// f32: the Gram matrix and both triangular products run on the FP32 matrix
// cores (operands rounded to FP32, FP64 epilogue); the Cholesky-inversion
// stays FP64.
// Device weight block of one step (dw, optional): [c, a - b/c, b/c, sqrt(c),
// (a - b/c)/sqrt(c)]; when given, the products read their scalars from it so
// the same captured launches serve any weights.
constexpr int kStepParams = 8;
void step_params(double a, double b, double c, double* out) {
  out[0] = c; out[1] = a - b / c; out[2] = b / c; out[3] = std::sqrt(c);
  out[4] = (a - b / c) / std::sqrt(c);
  out[5] = out[6] = out[7] = 0.0;
}

// f32 with room for it: the operands are first rounded into FP32 copies
// (X, W^{-1}, then the product X W^{-1}), so the FP32 products read half the
// bytes of FP64 operands; the products' results stay FP64.
void chol_step(double*& X, double*& Xn, int64_t m, int64_t n, double a, double b, double c, bool sym,
               const StepBufs& B, hipStream_t s, bool f32 = false, const double* dw = nullptr) {
  const double* Wi = B.spd;
  double* T = B.spd + spd_inverse_doubles(n);
  // FP32 staging after T: X32 (m x n), T32 (m x n), W32 (n x n) floats
  float* X32 = (float*)(T + m * n);
  float* T32 = X32 + m * n;
  float* W32 = T32 + m * n;
  const bool staged = f32 && B.spd_doubles > 0 &&
                      spd_inverse_doubles(n) + m * n + (2 * m * n + n * n + 1) / 2 <= B.spd_doubles;
  if (staged) to_f32(X, m, X32, m, m, n, s);
  Gemm g;
  g.f32 = f32; g.in32 = staged;
  g.M = n; g.N = n; g.K = m; g.alpha = c; g.beta = 0.0; g.diag = 1.0;
  if (dw) { g.dscal = dw; g.ia = 0; }
  g.A = staged ? (const double*)X32 : X; g.lda = m; g.ta = true; g.B = g.A; g.ldb = m; g.C = B.Z; g.ldc = n;
  g.tiles = TILES_UPPER;
  dgemm(g, s);
  chol_inverse_factor(B.Z, n, n, B.spd, B.flag, s);
  if (staged) to_f32(Wi, n, W32, n, n, n, s);
  Gemm t;
  t.f32 = f32; t.in32 = staged;
  t.M = m; t.N = n; t.K = n; t.A = staged ? (const double*)X32 : X; t.lda = m;
  t.B = staged ? (const double*)W32 : Wi; t.ldb = n; t.C = T; t.ldc = m;
  t.khi = KHI_COL;
  dgemm(t, s);
  if (staged) to_f32(T, m, T32, m, m, n, s);
  Gemm u;
  u.f32 = f32; u.in32 = staged;
  u.M = m; u.N = n; u.K = n; u.alpha = a - b / c; u.beta = b / c;
  u.A = staged ? (const double*)T32 : T; u.lda = m; u.B = staged ? (const double*)W32 : Wi; u.ldb = n;
  u.tb = true; u.C = Xn; u.ldc = m; u.Cin = X; u.ldcin = m;
  u.klo = KLO_COL;
  if (dw) { u.dscal = dw; u.ia = 1; u.ib = 2; }
  if (sym) u.tiles = TILES_UPPER;
  dgemm(u, s);
  if (sym) mirror_upper(Xn, n, m, s);
  std::swap(X, Xn);
}

// FP64 Newton-Schulz step X <- X (3I - X^T X)/2 (polish after mixed-precision
// Cholesky steps: drives the singular values that the iteration mapped near 1
// back to 1 to FP64 accuracy).  Needs ||X||_2 < sqrt(3).
void ns_step(double*& X, double*& Xn, int64_t m, int64_t n, bool sym, const StepBufs& B, hipStream_t s) {
  Gemm g;
  g.M = n; g.N = n; g.K = m; g.A = X; g.lda = m; g.ta = true; g.B = X; g.ldb = m; g.C = B.Z; g.ldc = n;
  g.tiles = TILES_UPPER;
  dgemm(g, s);
  mirror_upper(B.Z, n, n, s);
  Gemm u;
  u.M = m; u.N = n; u.K = n; u.alpha = -0.5; u.beta = 1.5; u.A = X; u.lda = m; u.B = B.Z; u.ldb = n;
  u.C = Xn; u.ldc = m; u.Cin = X; u.ldcin = m;
  if (sym) u.tiles = TILES_UPPER;
  dgemm(u, s);
  if (sym) mirror_upper(Xn, n, m, s);
  std::swap(X, Xn);
}

// Eq. (2): [sqrt(c) X; I] = [Q1; Q2] R, X+ = (b/c) X + (a - b/c)/sqrt(c) Q1 Q2^T.
void qr_step(double* X, int64_t m, int64_t n, double a, double b, double c, bool sym,
             const StepBufs& B, hipStream_t s, const double* dw = nullptr) {
  const int64_t mn = m + n;
  stacked(X, m, B.W, mn, m, n, std::sqrt(c), s, dw ? dw + 3 : nullptr);
  // Cholesky-QR panels only where cond(W) <= sqrt(1 + c) keeps them well inside their checks;
  // the identity block's untouched rows are skipped (tuning key "qr.stacked", default on)
  const int64_t st = qdwhp_tune_get("qr.stacked", 1) ? m : 0;
  geqrf(B.W, mn, n, mn, B.tau, B.Tall, B.qrs, s, nullptr, c <= 1e8, st);
  orgqr(B.W, mn, mn, B.Tall, n, 0, n, B.Q, mn, B.qrs, s, st);
  Gemm g;
  g.M = m; g.N = n; g.K = n; g.alpha = (a - b / c) / std::sqrt(c); g.beta = b / c;
  g.A = B.Q; g.lda = mn; g.B = B.Q + m; g.ldb = mn; g.tb = true; g.C = X; g.ldc = m;
  if (dw) { g.dscal = dw; g.ia = 4; g.ib = 2; }
  dgemm(g, s);
  if (sym) symmetrize(X, n, m, s);
}

// One Zolotarev step (type (2r+1, 2r), the higher-order variant of Sec. 3.1):
// X+ = M X + sum_j (M a_j) X (X^T X + c_j I)^{-1}, c_j = c_{2j-1}.  The
// Cholesky-form terms share the Gram G = X^T X: Z = I + G / c_j = W^T W, and
// X (X^T X + c_j I)^{-1} = (1/c_j) (X W^{-1}) W^{-T} (the two triangular
// products of Eq. (3)); the QR-form terms take [X / sqrt(c_j); I] = [Q1; Q2] R,
// X (X^T X + c_j I)^{-1} = Q1 Q2^T / sqrt(c_j) (the structured QR of Eq. (2)).
// The terms accumulate into Xn (upper tiles and one mirror when sym).
void zolo_step(double*& X, double*& Xn, int64_t m, int64_t n, const ZoloStep& z, bool sym, const StepBufs& B,
               hipStream_t s) {
  const double* Wi = B.spd;
  double* T = B.spd + spd_inverse_doubles(n);
  bool first = true, have_gram = false;
  auto accumulate = [&](Gemm& u) {
    if (first) { u.beta = z.M; u.Cin = X; u.ldcin = m; }
    else { u.beta = 1.0; u.Cin = Xn; u.ldcin = m; }
    u.C = Xn; u.ldc = m;
    if (sym) u.tiles = TILES_UPPER;
    dgemm(u, s);
    first = false;
  };
  for (int pass = 0; pass < 2; ++pass) {          // Cholesky-form terms first: the QR ones reuse B.W
    for (int j = 0; j < z.r; ++j) {
      const bool qr = z.kinds[j] == 1;
      if (qr != (pass == 1)) continue;
      const double cj = z.c[2 * j];
      const double coef = z.M * z.a[j];
      if (!qr) {
        if (!have_gram) {
          Gemm g;
          g.M = n; g.N = n; g.K = m; g.A = X; g.lda = m; g.ta = true; g.B = X; g.ldb = m; g.C = B.G; g.ldc = n;
          g.tiles = TILES_UPPER;
          dgemm(g, s);
          have_gram = true;
        }
        eig_x0(B.G, n, B.Z, n, n, 1.0, 1.0, -1.0 / cj, 0.0, s);   // Z = I + G / c_j (upper part read)
        chol_inverse_factor(B.Z, n, n, B.spd, B.flag, s);
        Gemm t;
        t.M = m; t.N = n; t.K = n; t.A = X; t.lda = m; t.B = Wi; t.ldb = n; t.C = T; t.ldc = m;
        t.khi = KHI_COL;
        dgemm(t, s);
        Gemm u;
        u.M = m; u.N = n; u.K = n; u.alpha = coef / cj;
        u.A = T; u.lda = m; u.B = Wi; u.ldb = n; u.tb = true; u.klo = KLO_COL;
        accumulate(u);
      } else {
        const int64_t mn = m + n;
        stacked(X, m, B.W, mn, m, n, 1.0 / std::sqrt(cj), s);
        const int64_t st = qdwhp_tune_get("qr.stacked", 1) ? m : 0;
        geqrf(B.W, mn, n, mn, B.tau, B.Tall, B.qrs, s, nullptr, 1.0 / cj <= 1e8, st);
        orgqr(B.W, mn, mn, B.Tall, n, 0, n, B.Q, mn, B.qrs, s, st);
        Gemm g;
        g.M = m; g.N = n; g.K = n; g.alpha = coef / std::sqrt(cj);
        g.A = B.Q; g.lda = mn; g.B = B.Q + m; g.ldb = mn; g.tb = true;
        accumulate(g);
      }
    }
  }
  if (sym) mirror_upper(Xn, n, m, s);
  std::swap(X, Xn);
}

// ---------------------------------------------------------------------------
struct Plan {
  double *X, *Xn, *Z, *big;
  int64_t big_doubles;
  double *tau, *Tall, *diag, *vals, *lz, *wts;
  QrScratch qrs;
  int* flags;       // [0] Cholesky breakdown, [1] non-finite input
  double* G = nullptr;   // n x n Gram of the Zolotarev steps (only with zolo_r > 0)
};

Plan carve(Arena& ar, int64_t mm, int64_t nn, int nv, int64_t msteps, bool svd, bool zolo) {
  Plan p;
  const int64_t np = jacobi_padded(nn);
  p.X = ar.take(mm * nn);
  p.Xn = ar.take(mm * nn);
  p.Z = ar.take(nn * nn);
  int64_t big = std::max<int64_t>(spd_inverse_doubles(nn) + mm * nn, 2 * (mm + nn) * nn);
  if (svd) big = std::max<int64_t>(big, gesvj_scratch_doubles(nn, nn) + nn * nn);
  else big = std::max<int64_t>(big, nn * nn + syev_scratch_doubles(nn));
  big = std::max<int64_t>(big, np * np);
  p.big = ar.take(big);
  p.big_doubles = big;
  p.tau = ar.take(mm + nn);
  p.Tall = ar.take(qr_t_doubles(mm + nn));
  p.diag = ar.take(mm + nn);
  p.vals = ar.take(np);
  double* q = ar.take(qr_scratch_doubles(mm + nn, nn));
  p.qrs = ar.base ? carve_qr_scratch(q, mm + nn, nn) : QrScratch{};
  p.lz = ar.take(lanczos_doubles(nn, mm, nv, (int)msteps));
  p.flags = (int*)ar.take(8);
  p.wts = ar.take(16 * 8);
  if (zolo) p.G = ar.take(nn * nn);
  return p;
}

StepBufs step_bufs(const Plan& p, int64_t m, int64_t n) {
  StepBufs b;
  b.Z = p.Z; b.spd = p.big; b.spd_doubles = p.big_doubles; b.W = p.big; b.Q = p.big + (m + n) * n;
  b.tau = p.tau; b.Tall = p.Tall; b.qrs = p.qrs; b.flag = p.flags; b.G = p.G;
  return b;
}

void fill_info(qdwhp_info* info, const std::vector<DwhStep>& sched) {
  info->n_iter = (int)sched.size();
  for (size_t i = 0; i < sched.size() && i < 16; ++i) {
    info->kinds[i] = sched[i].kind;
    info->weights[i][0] = sched[i].a;
    info->weights[i][1] = sched[i].b;
    info->weights[i][2] = sched[i].c;
  }
}

void fill_info_zolo(qdwhp_info* info, const std::vector<ZoloStep>& zs) {
  info->n_iter = (int)zs.size();
  for (size_t i = 0; i < zs.size() && i < 16; ++i) {
    int kind = 2;
    for (int j = 0; j < zs[i].r; ++j) if (zs[i].kinds[j] == 1) kind = 1;
    info->kinds[i] = kind;
    info->weights[i][0] = zs[i].M;
    info->weights[i][1] = zs[i].r;
    info->weights[i][2] = zs[i].l;
  }
}

// Table 1's accounting for Zolotarev steps: the Gram 2mn^2 once per step with
// a Cholesky-form term, each Cholesky-form term n^3/3 + 2mn^2 (factor and
// the two triangular solves), each QR-form term 6mn^2 + 8/3 n^3.
double table1_zolo_flops(const std::vector<ZoloStep>& zs, double m, double n) {
  double f = 0.0;
  for (const auto& z : zs) {
    bool gram = false;
    for (int j = 0; j < z.r; ++j) {
      if (z.kinds[j] == 1) f += 6.0 * m * n * n + 8.0 / 3.0 * n * n * n;
      else { f += n * n * n / 3.0 + 2.0 * m * n * n; gram = true; }
    }
    if (gram) f += 2.0 * m * n * n;
  }
  return f;
}

// first 1-based i with |R_ii| < tol, n + 1 if none
int64_t find_ind(const std::vector<double>& d, double tol) {
  for (size_t i = 0; i < d.size(); ++i)
    if (std::fabs(d[i]) < tol) return (int64_t)i + 1;
  return (int64_t)d.size() + 1;
}

bool any_nonfinite(const std::vector<double>& d) {
  for (double v : d) if (!std::isfinite(v)) return true;
  return false;
}

double table1_iter_flops(const std::vector<DwhStep>& sched, double m, double n) {
  double f = 0.0;
  for (const auto& st : sched)
    f += (st.kind == 1) ? 6.0 * m * n * n + 8.0 / 3.0 * n * n * n : 4.0 * m * n * n + n * n * n / 3.0;
  return f;
}

// Columns of the projector QR that can matter: a solve for k values needs
// ell = n - ind + 1 >= k, i.e. its first small diagonal entry at index
// ind <= n - k + 1, and an attempt with a smaller ell is retried whatever
// the later columns hold.  The leading columns of a Householder QR do not
// depend on the later ones, so only the first n - k + 1 columns are
// factored and updated (the trailing updates of the rest are skipped); a
// threshold given by the caller (replay) bounds nothing and keeps all n.
int64_t projector_qr_cols(int64_t n, int64_t k, bool replay) {
  return replay ? n : std::max<int64_t>(1, std::min<int64_t>(n, n - k + 1));
}

// Projector QR watch: after each panel, read its part of diag(R) (final
// once the panel is factored) and stop at the first panel holding an entry
// below tol, or a non-finite one: ind is the first such index, and only the
// reflectors before it are used (Q2 = H_1 ... H_{ind-1} [0; I]).
PanelWatch diag_watch(double* B, int64_t ldb, double* dbuf, double tol, std::vector<double>* d, hipStream_t s) {
  return [=](int64_t c0, int w) -> bool {
    diagonal(B + c0 + c0 * ldb, ldb, w, dbuf, s);
    std::vector<double> part(w);
    QDWHP_HIP(hipMemcpyAsync(part.data(), dbuf, sizeof(double) * w, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    bool stop = false;
    for (double v : part) {
      d->push_back(v);
      if (!std::isfinite(v) || std::fabs(v) < tol) stop = true;
    }
    return stop;
  };
}

// The DWH steps of a solve, then the FP64 polish plan (0 = Newton-Schulz,
// 1 = Halley (3,1,3) in Cholesky form) of the mixed-precision variant.
// Mixed precision runs every Cholesky-based step but the last on the FP32
// matrix cores; the last step of the schedule stays FP64: its map is flat at
// 1 (|1 - r(1 + e)| = O(e^3) for l_k near 1), so the O(u_32) errors the
// low-precision steps leave on the wanted values vanish, while the unwanted
// values get the same map as in FP64 (the band, hence ell, stays as in FP64;
// a Newton-Schulz polish would push the band towards 1 and enlarge ell).
// With opts.graphs the sequence is captured once per (buffers, sizes, step
// kinds, plan) and replayed with this solve's weights.
void run_iterations(double*& X, double*& Xn, int64_t m, int64_t n, bool sym, const std::vector<DwhStep>& sched,
                    bool mixed, const std::vector<int>& polish, const Plan& P, const StepBufs& sb, bool graphs,
                    hipStream_t s) {
  std::vector<double> w(kStepParams * sched.size());
  for (size_t i = 0; i < sched.size(); ++i) step_params(sched[i].a, sched[i].b, sched[i].c, &w[kStepParams * i]);
  auto body = [&](double*& x, double*& xn, const double* dw) {
    for (size_t i = 0; i < sched.size(); ++i) {
      const DwhStep& st = sched[i];
      const double* d = dw ? dw + kStepParams * i : nullptr;
      if (st.kind == 1) qr_step(x, m, n, st.a, st.b, st.c, sym, sb, s, d);
      else chol_step(x, xn, m, n, st.a, st.b, st.c, sym, sb, s, mixed && i + 1 < sched.size(), d);
    }
    for (int p : polish) {
      if (p == 0) ns_step(x, xn, m, n, sym, sb, s);
      else chol_step(x, xn, m, n, 3.0, 1.0, 3.0, sym, sb, s, false);
    }
  };
  if (graphs && sched.size() <= 16 && !prof_active() && !no_alloc_mode()) {
    std::vector<int64_t> key = {(int64_t)(intptr_t)X, (int64_t)(intptr_t)Xn, (int64_t)(intptr_t)P.big,
                                (int64_t)(intptr_t)P.wts, m, n, sym, mixed};
    for (const auto& st : sched) key.push_back(st.kind);
    key.push_back(-1);
    for (int p : polish) key.push_back(p);
    write_params(P.wts, w.data(), (int)w.size(), s);
    double* x = X;
    double* xn = Xn;
    if (graph_replay(key, s, [&] { double* a = X; double* b = Xn; body(a, b, P.wts); })) {
      // the steps exchange X and Xn once per Cholesky-form or polish step
      int swaps = (int)polish.size();
      for (const auto& st : sched) swaps += (st.kind != 1);
      if (swaps & 1) std::swap(x, xn);
      X = x; Xn = xn;
      return;
    }
  }
  body(X, Xn, nullptr);
}

// Orthonormal basis of the columns of Y (rows x r, ld rows) by one Cholesky
// QR round: Q = Y W^{-1} with W^T W = Y^T Y.  gram: r x r; spd:
// spd_inverse_doubles(r).  Sets *flag on a non-positive pivot.
void chol_qr(const double* Y, int64_t rows, int64_t r, double* gram, double* spd, double* Q, int* flag,
             hipStream_t s) {
  Gemm g;
  g.M = r; g.N = r; g.K = rows; g.A = Y; g.lda = rows; g.ta = true; g.B = Y; g.ldb = rows;
  g.C = gram; g.ldc = r; g.tiles = TILES_UPPER;
  dgemm(g, s);
  chol_inverse_factor(gram, r, r, spd, flag, s);
  Gemm t;
  t.M = rows; t.N = r; t.K = r; t.A = Y; t.lda = rows; t.B = spd; t.ldb = r; t.C = Q; t.ldc = rows;
  t.khi = KHI_COL;
  dgemm(t, s);
}

// The step of Eq. (2) for the split's polar decomposition with the QR of
// W = [sqrt(c) X; I] (2n x n) taken by shifted Cholesky QR in three rounds
// (one round with the Gram shifted by 11 (2n^2 + n(n+1)) u ||W||^2 so that
// its Cholesky factor exists for any cond(W) <= 1/u, then two plain
// rounds): every round is a Gram, the Cholesky-inverse of Eq. (3)'s step
// and a triangular product, so the step has no per-column launches.  The
// published analysis of shifted Cholesky QR proves Q orthonormal to working
// accuracy only up to a smaller cond(W), which shrinks with the matrix size
// (about 1e6-1e7 for n near 5000); the first step from l0 = 1e-12 has
// cond(W) ~ sqrt(1 + c) ~ 1.3e8, beyond it.  There orthogonality is
// observed, not proved (FP64 emulation: max |Q^T Q - I| = 1.3e-15 at
// n = 2500).  Callers check the result of the whole polar decomposition
// (the split's residual test), so a loss of orthogonality costs a fallback
// to the plain solver, never a wrong result.  X+ = (b/c) X + (a - b/c)/sqrt(c)
// Q1 Q2^T as in Eq. (2).  W and Q: 2n x n each; G: n x n; spd:
// spd_inverse_doubles(n).  ||X||_2 <= 1 is assumed for the shift.
void cholqr_step(double* X, int64_t n, double a, double b, double c, double* W, double* Q, double* G,
                 double* spd, int* flag, hipStream_t s, bool sym = true) {
  const int64_t n2 = 2 * n;
  stacked(X, n, W, n2, n, n, std::sqrt(c), s);
  double* src = W;
  double* dst = Q;
  for (int round = 0; round < 3; ++round) {
    Gemm g;
    g.M = n; g.N = n; g.K = n2; g.A = src; g.lda = n2; g.ta = true; g.B = src; g.ldb = n2;
    g.C = G; g.ldc = n; g.tiles = TILES_UPPER;
    if (round == 0) g.diag = 11.0 * (double)(n2 * n + n * (n + 1)) * 1.1102230246251565e-16 * (c + 1.0);
    dgemm(g, s);
    chol_inverse_factor(G, n, n, spd, flag, s);
    Gemm t;
    t.M = n2; t.N = n; t.K = n; t.A = src; t.lda = n2; t.B = spd; t.ldb = n; t.C = dst; t.ldc = n2;
    t.khi = KHI_COL;
    dgemm(t, s);
    std::swap(src, dst);
  }
  Gemm f;   // src holds Q after the three rounds
  f.M = n; f.N = n; f.K = n; f.alpha = (a - b / c) / std::sqrt(c); f.beta = b / c;
  f.A = src; f.lda = n2; f.B = src + n; f.ldb = n2; f.tb = true; f.C = X; f.ldc = n;
  dgemm(f, s);
  if (sym) symmetrize(X, n, n, s);
}

// The SVD of the Rayleigh-Ritz factor R (ell x ell, ld ell) the QDWH-SVD
// way (Sec. 3.2): the polar factor U_p of R / alpha (||R|| <= alpha) by the
// scalar schedule of Sec. 3.1 run to convergence from l0 = 1e-12 (its
// QR-form steps by the shifted Cholesky QR of cholqr_step, the rest
// Cholesky-based), H = U_p^T R (symmetric positive semidefinite), the
// symmetric eigen decomposition H = W diag(sigma) W^T by block Jacobi, and
// U = U_p W.  Singular values below 1e-12 alpha are left unconverged (their
// vectors are not asked for).  On success R <- U (ell x ell), vals[0..ell)
// the singular values (descending), V (ell x ell, ld ell) the right vectors,
// and it returns the Jacobi sweeps; returns -1 (R untouched) when buf is too
// small or a pivot fails.  buf: buf_doubles of free device memory.
int polar_svd(double* R, int64_t ell, double alpha, double* vals, double*& V, double* buf, int64_t buf_doubles,
              const qdwhp_opts& o, int* flag, hipStream_t s) {
  const int64_t e2 = ell * ell;
  const int64_t spdn = spd_inverse_doubles(ell);
  double* Xp = buf;
  double* Xnp = Xp + e2;
  double* Zp = Xnp + e2;
  double* spd = Zp + e2;            // spd_inverse_doubles(ell) + ell^2 (the step's product)
  double* W = spd + spdn + e2;      // 2 ell^2
  double* Q = W + 2 * e2;           // 2 ell^2
  const int64_t need = 3 * e2 + spdn + e2 + 4 * e2;
  if (need > buf_doubles || syev_scratch_doubles(ell) > spdn + 5 * e2) return -1;
  scale_copy(R, ell, Xp, ell, ell, ell, 1.0 / alpha, false, s);
  StepBufs sb;
  sb.Z = Zp; sb.spd = spd; sb.W = W; sb.Q = Q; sb.flag = flag;
  double* X = Xp;
  double* Xn = Xnp;
  for (const DwhStep& st : svd_schedule(1e-12, o.kappa_max, false)) {
    if (st.kind == 1) cholqr_step(X, ell, st.a, st.b, st.c, W, Q, Zp, spd, flag, s, false);
    else chol_step(X, Xn, ell, ell, st.a, st.b, st.c, false, sb, s);
  }
  int hf = 0;
  QDWHP_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  if (hf) {
    QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    return -1;
  }
  // H = U_p^T R, symmetrised; its eigenvectors W land in Xn, U = U_p W in R
  Gemm h;
  h.M = ell; h.N = ell; h.K = ell; h.A = X; h.lda = ell; h.ta = true; h.B = R; h.ldb = ell; h.C = Zp; h.ldc = ell;
  dgemm(h, s);
  symmetrize(Zp, ell, ell, s);
  const int sweeps = syev(Zp, ell, ell, vals, Xn, ell, spd, s);
  if (sweeps < 0) return -1;
  Gemm u;
  u.M = ell; u.N = ell; u.K = ell; u.A = X; u.lda = ell; u.B = Xn; u.ldb = ell; u.C = R; u.ldc = ell;
  dgemm(u, s);
  V = Xn;
  return sweeps;
}

struct Bump {
  double* p = nullptr;
  int64_t left = 0;
  double* take(int64_t n) {
    n = (n + 31) / 32 * 32;      // 256-byte steps
    if (n > left) throw WorkspaceError{};
    double* r = p;
    p += n;
    left -= n;
    return r;
  }
};

constexpr int kDcSteps = 32;     // Lanczos steps of the shift estimate
constexpr int kDcVectors = 4;
struct DcStats { int splits = 0, leaves = 0, fallbacks = 0, depth = 0; };

// QDWH-based divide and conquer of a symmetric block (defined below).
int dc_eig(const double* H, int64_t ell, double* vals, double* W, Bump mem, const qdwhp_opts& o, int* flag,
           double* dbuf, int depth, DcStats* st, hipStream_t s, int64_t leaf);
int64_t dc_node_doubles(int64_t ell);

// Exact spectral split of the Rayleigh-Ritz matrix H (ell x ell, the
// Sec. 3.2 mechanism of QDWH-EIG): sigma is placed by a Lanczos estimate so
// that about k + margin eigenvalues lie above it; the polar factor of
// (H - sigma I) / alpha, taken to convergence by the scalar schedule of
// Sec. 3.1 from a lower bound 1e-12 (its QR-form steps by shifted Cholesky
// QR, cholqr_step), is sign(H - sigma I), so C = (I + X) / 2 projects onto
// the invariant subspace of the r eigenvalues above sigma.  Two subspace
// passes (C Omega, then C Q1, each orthonormalised) give an orthonormal
// basis Q1 of range(C); the r x r problem Q1^T H Q1 holds exactly those
// eigenvalues and is solved by Jacobi.  The split is checked: every column
// of H Q1 - Q1 (Q1^T H Q1) must be below 5e-14 ||H||, else (or when r < k,
// a pivot fails, or the buffers are too small) it returns 0 and H is
// untouched for the plain solve.  On success vals[0 .. r) holds the
// eigenvalues (descending), vals[r .. ell) -1e300, Wv (ell x r, ld ell)
// the eigenvectors; returns r.
//   top: the estimator's quadrature of the n x n operator (nullptr when
//   the solve replays a given threshold or retried it).  Every eigenvalue
//   of that operator above the threshold tau is an eigenvalue of H (Q2
//   contains its eigenvectors, Theorem 1), and a cut for k + margin < the
//   threshold's target lies at or above tau, so the counts the quadrature
//   gives there are counts of H's eigenvalues and its bounds bound H's
//   spectrum.  Without it a Lanczos run on H itself places sigma.
//   ybuf (ybuf_doubles): free during the call; zbuf = Wv (zbuf_doubles);
//   jscr: scratch of at least syev_scratch_doubles(ell).
int64_t rr_split(const double* H, int64_t ell, int64_t k, int64_t n, const LanczosResult* top, double top_lmax,
                 double top_lmin, const qdwhp_opts& o, const Plan& P, double* ybuf, int64_t ybuf_doubles,
                 double* Wv, int64_t zbuf_doubles, double* jscr, double* vals, int* sweeps, hipStream_t s) {
  const int64_t e2 = ell * ell;
  const int nv = lz_vectors(o);
  const int64_t margin = std::max<int64_t>(16, k / 32);
  if (ell < qdwhp_tune_get("rr.split_min", 3000) || 100 * (k + margin) > qdwhp_tune_get("rr.split_pct", 85) * ell)
    return 0;
  const int64_t wsd = skinny_ws_doubles(ell, nv);
  if (ybuf_doubles < 5 * e2 + wsd + 1024 || zbuf_doubles < 4 * e2 + spd_inverse_doubles(ell) + 2 * ell) return 0;
  double* Cp = ybuf + 2 * e2;    // Z of the steps, then the projector C (iterates X, Xn before it)
  double* Q1 = Cp + e2;          // ell x r
  double* H1 = Q1 + e2;          // r x r
  double* ws = H1 + e2;
  double* big = Wv;              // step buffers, then the subspace passes
  // ---- sigma from a Lanczos estimate (the estimator's quadrature first;
  // if that over-counts, so that fewer than k eigenvalues lie above sigma,
  // a Lanczos run on H itself places it again)
  const bool have_top = top && !top->nodes.empty();
  int64_t r = 0;
  double sigma = 0.0, alpha = 0.0, hnorm = 0.0;
  // eigenvalues above sigma in tight clusters: quadrature nodes that have
  // converged (residual bound within 1e-6 of the spread) and stand for at
  // least 8 eigenvalues each
  double clustered = 0.0;
  auto cluster_mass = [&](const LanczosResult& q, int64_t dim, double lmx, double lmn) {
    const double spread = std::max(lmx - lmn, 1e-300), scale = (double)dim / q.nv;
    double c = 0.0;
    for (size_t i = 0; i < q.nodes.size(); ++i) {
      const double cnt = scale * q.weights[i];
      if (q.nodes[i] > sigma && q.resid[i] <= 1e-6 * spread && cnt >= 8.0) c += cnt;
    }
    return c;
  };
  int hf = 0;
  auto failed = [&]() {
    QDWHP_HIP(hipMemsetAsync(P.flags, 0, sizeof(int), s));
    return (int64_t)0;
  };
  for (int attempt = have_top ? 0 : 1; attempt < 2; ++attempt) {
    double lmax = top_lmax, lmin = top_lmin;
    if (attempt == 0) {
      if (!cut_below(top->nodes, top->weights, n, top->nv, lmax, lmin, k + margin, &sigma)) continue;
      clustered = cluster_mass(*top, n, lmax, lmin);
    } else {
      LanczosOp op;
      op.rows_tmp = 1;
      op.apply = [&](const double* in, int64_t ldi, double* out, int64_t ldo, double*, hipStream_t st) {
        skinny_gemm(H, ell, ell, ell, in, ldi, nv, 1.0, out, ldo, ws, wsd, st);
      };
      const LanczosResult lz = lanczos(op, ell, nv, (int)lz_steps(o, ell), o.seed + 1, P.lz, s);
      if (lz.sweeps < 0) return 0;
      lmax = -std::numeric_limits<double>::infinity();
      lmin = std::numeric_limits<double>::infinity();
      for (size_t i = 0; i < lz.nodes.size(); ++i) {
        lmax = std::max(lmax, lz.nodes[i] + lz.resid[i]);
        lmin = std::min(lmin, lz.nodes[i] - lz.resid[i]);
      }
      if (!cut_below(lz.nodes, lz.weights, ell, nv, lmax, lmin, k + margin, &sigma)) return 0;
      clustered = cluster_mass(lz, ell, lmax, lmin);
    }
    alpha = 1.05 * std::max(lmax - sigma, sigma - lmin);
    hnorm = std::max(std::fabs(lmax), std::fabs(lmin));
    if (!(alpha > 0.0) || !std::isfinite(alpha)) return 0;
    // ---- X -> sign((H - sigma I) / alpha)
    double* X = ybuf;
    double* Xn = X + e2;
    eig_x0(H, ell, X, ell, ell, 1.0 / alpha, -sigma, -1.0, 0.0, s);
    StepBufs sb;
    sb.Z = Cp; sb.spd = big; sb.W = big; sb.Q = big + 2 * e2;
    sb.tau = P.tau; sb.Tall = P.Tall; sb.qrs = P.qrs; sb.flag = P.flags;
    for (const DwhStep& st : svd_schedule(1e-12, o.kappa_max, false)) {
      if (st.kind == 1) cholqr_step(X, ell, st.a, st.b, st.c, big, big + 2 * e2, Cp, big + 4 * e2, P.flags, s);
      else chol_step(X, Xn, ell, ell, st.a, st.b, st.c, true, sb, s);
    }
    half_plus_identity(X, ell, Cp, ell, ell, s);
    std::vector<double> d(ell);
    diagonal(Cp, ell, ell, P.diag, s);
    QDWHP_HIP(hipMemcpyAsync(d.data(), P.diag, sizeof(double) * ell, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipMemcpyAsync(&hf, P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (hf) return failed();
    double tr = 0.0;
    for (double v : d) tr += v;
    if (!std::isfinite(tr)) return 0;
    r = (int64_t)std::llround(tr);
    if (r >= ell) return 0;
    if (r >= k) break;
  }
  if (r < k) return 0;
  // ---- orthonormal basis of range(C): C Omega, then C Q1
  double* G = big;               // ell x r
  double* Yb = G + ell * r;      // ell x r
  double* gram = Yb + ell * r;   // r x r
  double* spd = gram + r * r;    // spd_inverse_doubles(r)
  if (zbuf_doubles < 2 * ell * r + r * r + spd_inverse_doubles(r)) return 0;
  gaussian_fill(G, ell * r, o.seed + 2, 0, s);
  for (int pass = 0; pass < 2; ++pass) {
    Gemm g;
    g.M = ell; g.N = r; g.K = ell; g.A = Cp; g.lda = ell; g.B = pass ? Q1 : G; g.ldb = ell;
    g.C = Yb; g.ldc = ell;
    dgemm(g, s);
    chol_qr(Yb, ell, r, gram, spd, Q1, P.flags, s);
  }
  // ---- H1 = Q1^T H Q1 and the check of the split
  {
    Gemm g;
    g.M = ell; g.N = r; g.K = ell; g.A = H; g.lda = ell; g.B = Q1; g.ldb = ell; g.C = Yb; g.ldc = ell;
    dgemm(g, s);
    Gemm h;
    h.M = r; h.N = r; h.K = ell; h.A = Q1; h.lda = ell; h.ta = true; h.B = Yb; h.ldb = ell;
    h.C = H1; h.ldc = r; h.tiles = TILES_UPPER;   // symmetric: the upper tiles, then mirrored
    dgemm(h, s);
    mirror_upper(H1, r, r, s);
    Gemm e;   // Yb <- H Q1 - Q1 H1
    e.M = ell; e.N = r; e.K = r; e.alpha = -1.0; e.beta = 1.0; e.A = Q1; e.lda = ell; e.B = H1; e.ldb = r;
    e.C = Yb; e.ldc = ell;
    dgemm(e, s);
    Gemm n2;  // column norms^2 of the residual on the diagonal of Yb^T Yb
    n2.M = r; n2.N = r; n2.K = ell; n2.A = Yb; n2.lda = ell; n2.ta = true; n2.B = Yb; n2.ldb = ell;
    n2.C = gram; n2.ldc = r; n2.tiles = TILES_UPPER;
    dgemm(n2, s);
    std::vector<double> cn(r);
    diagonal(gram, r, r, P.diag, s);
    QDWHP_HIP(hipMemcpyAsync(cn.data(), P.diag, sizeof(double) * r, hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipMemcpyAsync(&hf, P.flags, sizeof(int), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (hf) return failed();
    double worst = 0.0;
    for (double v : cn) worst = std::max(worst, std::isfinite(v) ? v : 1e300);
    if (!(std::sqrt(worst) <= 5e-14 * hnorm)) return 0;
  }
  // ---- the wanted block: Jacobi, or one more split at the median of its
  // spectrum (the same QDWH split, Sec. 3.2) with Jacobi on the two halves;
  // eigenvectors Q1 W1.  Jacobi needs many more sweeps when a good part of
  // the block lies in tight clusters (the rotations inside a cluster only
  // settle once everything else has converged); halving the rows of both
  // Jacobi problems then more than pays for the split.  Taken from
  // "rr.split2_min" rows when at least an eighth of the block is clustered
  // (cluster_mass above; "rr.split2_pct" = 0 drops that condition).
  double* W1 = ybuf;             // r x r (the iterates are no longer needed)
  const int64_t split2 = qdwhp_tune_get("rr.split2_min", 0);
  const int64_t pct2 = qdwhp_tune_get("rr.split2_pct", 12);
  if (split2 > 0 && r >= split2 && 100.0 * clustered >= (double)pct2 * (double)r &&
      dc_node_doubles(r) + r * r + syev_scratch_doubles(r) + 4096 <= zbuf_doubles) {
    DcStats st;
    Bump mem{Wv, zbuf_doubles};  // free until the final product
    // one level: the recursion's depth limit (24) makes both halves Jacobi leaves
    *sweeps = dc_eig(H1, r, vals, W1, mem, o, P.flags, P.diag, 23, &st, s, r - 1);
  } else {
    *sweeps = syev(H1, r, r, vals, W1, r, jscr, s);
  }
  if (*sweeps < 0) return 0;
  fill(vals + r, ell - r, 1, ell - r, -1e300, -1e300, s);
  Gemm v;
  v.M = ell; v.N = r; v.K = r; v.A = Q1; v.lda = ell; v.B = W1; v.ldb = r; v.C = Wv; v.ldc = ell;
  dgemm(v, s);
  return r;
}

}  // namespace

// ===========================================================================
// All eigenpairs of a symmetric matrix by QDWH-based spectral divide and
// conquer (the QDWH-EIG of Sec. 3.2, applied recursively).
namespace {


int64_t dc_node_doubles(int64_t ell) {
  const int64_t e2 = ell * ell;
  // polar phase: X, Xn, Z, spd + product, W, Q; then C; the shift's
  // Lanczos products
  return 3 * e2 + spd_inverse_doubles(ell) + e2 + 4 * e2 + e2 + 1024 + skinny_ws_doubles(ell, kDcVectors);
}

// Orthonormal basis (ell x r, ld ell) of range(P) for the projector P (ell x
// ell) of rank r: two subspace passes from a Philox Gaussian block, each
// orthonormalised by a Cholesky QR round.  gram: r x r, spd:
// spd_inverse_doubles(r), G, Y: ell x r.
void projector_basis(const double* P, int64_t ell, int64_t r, uint64_t key, double* Q, double* G, double* Y,
                     double* gram, double* spd, int* flag, hipStream_t s) {
  gaussian_fill(G, ell * r, key, 0, s);
  for (int pass = 0; pass < 2; ++pass) {
    Gemm g;
    g.M = ell; g.N = r; g.K = ell; g.A = P; g.lda = ell; g.B = pass ? Q : G; g.ldb = ell; g.C = Y; g.ldc = ell;
    dgemm(g, s);
    chol_qr(Y, ell, r, gram, spd, Q, flag, s);
  }
}

// Block Q^T H Q (r x r) of H (ell x ell), symmetrised, and the largest
// column norm of H Q - Q (Q^T H Q) (the split's check); Y: ell x r scratch,
// gram: r x r scratch.
double restricted(const double* H, int64_t ell, const double* Q, int64_t r, double* Hr, double* Y, double* gram,
                  double* dbuf, hipStream_t s) {
  Gemm g;
  g.M = ell; g.N = r; g.K = ell; g.A = H; g.lda = ell; g.B = Q; g.ldb = ell; g.C = Y; g.ldc = ell;
  dgemm(g, s);
  Gemm h;
  h.M = r; h.N = r; h.K = ell; h.A = Q; h.lda = ell; h.ta = true; h.B = Y; h.ldb = ell; h.C = Hr; h.ldc = r;
  h.tiles = TILES_UPPER;   // symmetric: the upper tiles, then mirrored
  dgemm(h, s);
  mirror_upper(Hr, r, r, s);
  Gemm e;
  e.M = ell; e.N = r; e.K = r; e.alpha = -1.0; e.beta = 1.0; e.A = Q; e.lda = ell; e.B = Hr; e.ldb = r;
  e.C = Y; e.ldc = ell;
  dgemm(e, s);
  Gemm n2;
  n2.M = r; n2.N = r; n2.K = ell; n2.A = Y; n2.lda = ell; n2.ta = true; n2.B = Y; n2.ldb = ell;
  n2.C = gram; n2.ldc = r; n2.tiles = TILES_UPPER;
  dgemm(n2, s);
  std::vector<double> cn(r);
  diagonal(gram, r, r, dbuf, s);
  QDWHP_HIP(hipMemcpyAsync(cn.data(), dbuf, sizeof(double) * r, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  double worst = 0.0;
  for (double v : cn) worst = std::max(worst, std::isfinite(v) ? v : 1e300);
  return std::sqrt(worst);
}


// H (ell x ell, ld ell) symmetric, read only; vals[ell] descending, W (ell x
// ell, ld ell) eigenvectors.  Returns the largest Jacobi sweep count of its
// leaves, or -1 if a leaf did not converge.
int dc_eig(const double* H, int64_t ell, double* vals, double* W, Bump mem, const qdwhp_opts& o, int* flag,
           double* dbuf, int depth, DcStats* st, hipStream_t s, int64_t leaf) {
  st->depth = std::max(st->depth, depth);
  const int64_t e2 = ell * ell;
  auto jacobi = [&]() {
    ++st->leaves;
    double* scr = mem.take(syev_scratch_doubles(ell));
    return syev(const_cast<double*>(H), ell, ell, vals, W, ell, scr, s);   // syev reads H only
  };
  if (ell <= leaf || depth >= 24) return jacobi();
  Bump m0 = mem;                        // released after the split
  // ---- shift at the median of the spectrum: a Lanczos quadrature of H
  const int64_t wsd = skinny_ws_doubles(ell, kDcVectors);
  double* ws = mem.take(wsd);
  double* lzb = mem.take(lanczos_doubles(ell, 1, kDcVectors, kDcSteps));
  LanczosOp op;
  op.rows_tmp = 1;
  op.apply = [&](const double* in, int64_t ldi, double* out, int64_t ldo, double*, hipStream_t t) {
    skinny_gemm(H, ell, ell, ell, in, ldi, kDcVectors, 1.0, out, ldo, ws, wsd, t);
  };
  const LanczosResult lz = lanczos(op, ell, kDcVectors, (int)std::min<int64_t>(kDcSteps, ell - 1),
                                   o.seed + 11 + (uint64_t)depth, lzb, s);
  if (lz.sweeps < 0) { ++st->fallbacks; mem = m0; return jacobi(); }
  double lmax = -std::numeric_limits<double>::infinity(), lmin = std::numeric_limits<double>::infinity();
  for (size_t i = 0; i < lz.nodes.size(); ++i) {
    lmax = std::max(lmax, lz.nodes[i] + lz.resid[i]);
    lmin = std::min(lmin, lz.nodes[i] - lz.resid[i]);
  }
  double sigma = 0.0;
  if (!cut_below(lz.nodes, lz.weights, ell, kDcVectors, lmax, lmin, ell / 2, &sigma)) {
    ++st->fallbacks; mem = m0; return jacobi();
  }
  const double alpha = 1.05 * std::max(lmax - sigma, sigma - lmin);
  if (!(alpha > 0.0) || !std::isfinite(alpha)) { ++st->fallbacks; mem = m0; return jacobi(); }
  mem = m0;
  // ---- X -> sign((H - sigma I) / alpha) by QDWH from l0 = 1e-12
  double* X = mem.take(e2);
  double* Xn = mem.take(e2);
  double* Z = mem.take(e2);
  double* spd = mem.take(spd_inverse_doubles(ell) + e2);
  double* Wb = mem.take(2 * e2);
  double* Qb = mem.take(2 * e2);
  eig_x0(H, ell, X, ell, ell, 1.0 / alpha, -sigma, -1.0, 0.0, s);
  StepBufs sb;
  sb.Z = Z; sb.spd = spd; sb.W = Wb; sb.Q = Qb; sb.flag = flag;
  for (const DwhStep& d : svd_schedule(1e-12, o.kappa_max, false)) {
    if (d.kind == 1) cholqr_step(X, ell, d.a, d.b, d.c, Wb, Qb, Z, spd, flag, s);
    else chol_step(X, Xn, ell, ell, d.a, d.b, d.c, true, sb, s);
  }
  // projectors C = (I + X)/2 onto the eigenvalues above sigma and I - C
  double* C = Xn;
  double* Cc = Z;
  half_plus_identity(X, ell, C, ell, ell, s);
  std::vector<double> dg(ell);
  diagonal(C, ell, ell, dbuf, s);
  int hf = 0;
  QDWHP_HIP(hipMemcpyAsync(dg.data(), dbuf, sizeof(double) * ell, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  double tr = 0.0;
  for (double v : dg) tr += v;
  const int64_t r = std::isfinite(tr) ? (int64_t)std::llround(tr) : -1;
  if (hf || r <= 0 || r >= ell) {
    if (hf) QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    ++st->fallbacks;
    mem = m0;
    return jacobi();
  }
  eig_x0(X, ell, Cc, ell, ell, 0.5, 1.0, 1.0, 0.0, s);   // Cc = (I - X)/2
  // ---- bases of the two ranges, the two blocks and the check of the split
  const int64_t r2 = ell - r;
  double* Q1 = Wb;                        // ell x r
  double* Q2 = Wb + ell * r;              // ell x r2
  double* H1 = C;                          // r x r (C no longer needed)
  double* H2 = Cc;                         // r2 x r2
  const double hnorm = std::max(std::fabs(lmax), std::fabs(lmin));
  // Each side: its basis, then its block and check (each reads only its own
  // projector and writes its block over it).  The two sides are independent
  // and latency bound, so unless it is off ("dc.concurrent" = 0) the second
  // runs from its own host thread on a helper stream, with scratch of its
  // own: the Y / G halves of Qb, its Gram after the first in X, its
  // Cholesky-inversion space after the first's, its diagonal after the
  // first's in dbuf.  The same kernels on the same data either way.
  double e1 = 0.0, e2n = 0.0;
  auto side = [&](const double* Cp, int64_t rr, uint64_t key, double* Qs, double* Hs, double* Y, double* G,
                  double* gr, double* sp, double* db, hipStream_t st) {
    projector_basis(Cp, ell, rr, key, Qs, G, Y, gr, sp, flag, st);
    return restricted(H, ell, Qs, rr, Hs, Y, gr, db, st);
  };
  const uint64_t key1 = o.seed + 21 + (uint64_t)depth * 2, key2 = o.seed + 22 + (uint64_t)depth * 2;
  if (!no_alloc_mode() && qdwhp_tune_get("dc.concurrent", 1) != 0) {
    int dev = 0;
    QDWHP_HIP(hipGetDevice(&dev));
    AuxLease aux(dev);
    QDWHP_HIP(hipEventRecord(aux->ready[0], s));          // both projectors are ready on s
    QDWHP_HIP(hipStreamWaitEvent(aux->s, aux->ready[0], 0));
    std::exception_ptr err2;
    std::thread th([&] {
      try {
        QDWHP_HIP(hipSetDevice(dev));
        e2n = side(Cc, r2, key2, Q2, H2, Qb + 2 * ell * r, Qb + 2 * ell * r + ell * r2, X + r * r,
                   spd + spd_inverse_doubles(r), dbuf + r, aux->s);
      } catch (...) {
        err2 = std::current_exception();
      }
    });
    std::exception_ptr err1;
    try {
      e1 = side(C, r, key1, Q1, H1, Qb, Qb + ell * r, X, spd, dbuf, s);
    } catch (...) {
      err1 = std::current_exception();
    }
    th.join();
    if (err1) std::rethrow_exception(err1);
    if (err2) std::rethrow_exception(err2);
    QDWHP_HIP(hipEventRecord(aux->done[0], aux->s));
    QDWHP_HIP(hipStreamWaitEvent(s, aux->done[0], 0));
  } else {
    e1 = side(C, r, key1, Q1, H1, Qb, Qb + e2, X, spd, dbuf, s);
    e2n = side(Cc, r2, key2, Q2, H2, Qb, Qb + e2, X, spd, dbuf, s);
  }
  QDWHP_HIP(hipMemcpyAsync(&hf, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  if (hf || !(e1 <= 5e-14 * hnorm) || !(e2n <= 5e-14 * hnorm)) {
    if (hf) QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    ++st->fallbacks;
    mem = m0;
    return jacobi();
  }
  ++st->splits;
  // ---- the two halves: Q1, Q2 (in Wb) and H1, H2 (in Xn, Z) stay; the rest is free
  Bump rest = m0;
  rest.take(e2);                            // X
  rest.take(e2);                            // Xn (H1)
  rest.take(e2);                            // Z (H2)
  rest.take(spd_inverse_doubles(ell) + e2);
  rest.take(2 * e2);                        // Wb (Q1, Q2)
  double* W1 = rest.take(r * r);
  double* W2 = rest.take(r2 * r2);
  int s1 = -1, s2 = -1;
  const bool leaf1 = r <= leaf || depth + 1 >= 24, leaf2 = r2 <= leaf || depth + 1 >= 24;
  if (leaf1 && leaf2 && !no_alloc_mode() && qdwhp_tune_get("dc.concurrent", 1) != 0) {
    // Both halves are Jacobi leaves, independent of each other, and each is
    // bound by the latency of its rounds: the second runs from a host thread
    // of its own on a helper stream (own scratch), beside the first.
    Bump rest2 = rest;
    double* scr1 = rest.take(syev_scratch_doubles(r));
    rest2.take(syev_scratch_doubles(r));
    double* scr2 = rest2.take(syev_scratch_doubles(r2));
    int dev = 0;
    QDWHP_HIP(hipGetDevice(&dev));
    AuxLease aux(dev);
    QDWHP_HIP(hipEventRecord(aux->ready[0], s));          // H2 is ready on s
    QDWHP_HIP(hipStreamWaitEvent(aux->s, aux->ready[0], 0));
    std::exception_ptr err2;
    std::thread th([&] {
      try {
        QDWHP_HIP(hipSetDevice(dev));
        s2 = syev(H2, r2, r2, vals + r, W2, r2, scr2, aux->s);
      } catch (...) {
        err2 = std::current_exception();
      }
    });
    std::exception_ptr err1;
    try {
      s1 = syev(H1, r, r, vals, W1, r, scr1, s);
    } catch (...) {
      err1 = std::current_exception();
    }
    th.join();
    if (err1) std::rethrow_exception(err1);
    if (err2) std::rethrow_exception(err2);
    QDWHP_HIP(hipEventRecord(aux->done[0], aux->s));      // s continues after both
    QDWHP_HIP(hipStreamWaitEvent(s, aux->done[0], 0));
    st->leaves += 2;
    st->depth = std::max(st->depth, depth + 1);   // as the leaves' own calls record it
    if (s1 < 0 || s2 < 0) return -1;
  } else {
    s1 = dc_eig(H1, r, vals, W1, rest, o, flag, dbuf, depth + 1, st, s, leaf);
    if (s1 < 0) return -1;
    s2 = dc_eig(H2, r2, vals + r, W2, rest, o, flag, dbuf, depth + 1, st, s, leaf);
    if (s2 < 0) return -1;
  }
  // eigenvectors [Q1 W1, Q2 W2]: the eigenvalues above sigma come first
  Gemm v1;
  v1.M = ell; v1.N = r; v1.K = r; v1.A = Q1; v1.lda = ell; v1.B = W1; v1.ldb = r; v1.C = W; v1.ldc = ell;
  dgemm(v1, s);
  Gemm v2;
  v2.M = ell; v2.N = r2; v2.K = r2; v2.A = Q2; v2.lda = ell; v2.B = W2; v2.ldb = r2; v2.C = W + ell * r;
  v2.ldc = ell;
  dgemm(v2, s);
  return std::max(s1, s2);
}

}  // namespace

extern "C" size_t qdwhp_syev_dc_workspace(int64_t n) {
  if (n < 1) return 0;
  // a node and, below it, its children; a leaf's Jacobi scratch
  const int64_t e2 = n * n;
  return (size_t)(2 * dc_node_doubles(n) + 2 * e2 + syev_scratch_doubles(n) + 4096) * 8;
}

extern "C" int qdwhp_syev_dc(const double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw,
                             void* work, size_t lwork, void* stream, int* levels) {
  if (!H) return -1;
  if (n < 1) return -2;
  if (ldh < n) return -3;
  if (!w) return -4;
  if (!W) return -5;
  if (ldw < n) return -6;
  if (!work) return -7;
  if (lwork < qdwhp_syev_dc_workspace(n)) return QDWHP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  try {
    qdwhp_opts o;
    qdwhp_opts_default(&o);
    Bump mem{(double*)work, (int64_t)(lwork / 8)};
    int* flag = (int*)mem.take(8);
    double* dbuf = mem.take(n + 64);
    double* Hc = mem.take(n * n);
    double* Wc = mem.take(n * n);
    QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    copy(H, ldh, Hc, n, n, n, s);
    DcStats st;
    const int sw = dc_eig(Hc, n, w, Wc, mem, o, flag, dbuf, 0, &st, s,
                          std::max<int64_t>(64, qdwhp_tune_get("dc.leaf", 512)));
    if (levels) *levels = st.depth;
    if (sw < 0) return QDWHP_ERR_NOCONV;
    copy(Wc, n, W, ldw, n, n, s);
    QDWHP_HIP(hipStreamSynchronize(s));
  } catch (const WorkspaceError&) {
    return QDWHP_ERR_WORKSPACE;
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

// ===========================================================================
extern "C" size_t qdwhp_eig_workspace(int64_t n, double fraction, const qdwhp_opts* opts) {
  (void)fraction;
  if (n < 1) return 0;
  qdwhp_opts o;
  if (opts) o = *opts; else qdwhp_opts_default(&o);
  Arena ar(nullptr, 0);
  carve(ar, n, n, lz_vectors(o), lz_steps(o, n), false, o.zolo_r > 0);
  return ar.off;
}

extern "C" size_t qdwhp_svd_workspace(int64_t m, int64_t n, int64_t k, const qdwhp_opts* opts) {
  (void)k;
  if (m < 1 || n < 1) return 0;
  qdwhp_opts o;
  if (opts) o = *opts; else qdwhp_opts_default(&o);
  const int64_t mm = std::max(m, n), nn = std::min(m, n);
  Arena ar(nullptr, 0);
  carve(ar, mm, nn, lz_vectors(o), lz_steps(o, nn), true, o.zolo_r > 0);
  return ar.off;
}

// ===========================================================================
// One solve in phases.  Everything a solve carries between its phases lives
// in SolveState, so that a batch or the server can run the DWH iterations of
// many solves together (iterations_grouped) between their setup and finish
// phases.  A standalone call runs the phases back to back.
namespace qdwhp {
struct SolveState {
  bool svd = false;
  // arguments
  const double* A = nullptr;
  int64_t m = 0, n = 0, lda = 0, k = 0;
  double fraction = 0.0;
  int which = QDWHP_LARGEST;
  double *w = nullptr, *U = nullptr, *V = nullptr;
  int64_t ldu = 0, ldv = 0;
  void* work = nullptr;
  size_t lwork = 0;
  qdwhp_opts o;
  hipStream_t s = nullptr;
  qdwhp_info* info = nullptr;
  Deferred* df = nullptr;
  // derived
  bool tr = false;                 // SVD of a wide A: the algorithm runs on M = A^T
  int64_t mm = 0, nn = 0;          // rows / columns of the iterate (EIG: n, n)
  int nv = 8;
  int64_t msteps = 64;
  double sgn = 1.0;                // EIG: -1 for the smallest eigenvalues
  Plan P;
  std::unique_ptr<Events> ev;
  LanczosResult lz;
  double lmax = 0.0, lmin = 0.0;
  bool replay = false;
  int boost = 1;
  std::vector<DwhStep> sched;
  std::vector<ZoloStep> zsched;    // Zolotarev steps instead of sched (opts.zolo_r > 0)
  std::vector<int> polish;
  bool mixed = false;
  double tau = 0.0, mu = 1.0, rho = 0.0;   // EIG threshold, scale, unwanted-side bound
  double alpha = 1.0, sthr = 0.5;          // SVD norm estimate, relative threshold
  double* X = nullptr;
  double* Xn = nullptr;
  StepBufs sb;
  int status = QDWHP_OK;
  int ret(int st) { info->status = st; status = st; return st; }
};

// The iterations of a set-up solve: its Zolotarev steps, or its DWH
// schedule (optionally as a captured graph) with the polish plan.
void iterate_state(SolveState& S, bool graphs, hipStream_t s) {
  if (!S.zsched.empty()) {
    for (const ZoloStep& z : S.zsched) zolo_step(S.X, S.Xn, S.mm, S.nn, z, !S.svd, S.sb, s);
    return;
  }
  run_iterations(S.X, S.Xn, S.mm, S.nn, !S.svd, S.sched, S.mixed, S.polish, S.P, S.sb, graphs, s);
}
}  // namespace qdwhp

namespace {

using qdwhp::SolveState;

// ---- EIG (Algorithm 1) -----------------------------------------------------
extern "C" int64_t qdwhp_eig_count(int64_t n, double fraction) {
  if (n < 1 || !(fraction > 0.0) || fraction > 1.0) return 0;
  const double k = std::floor(fraction * (double)n + 0.5);
  return k < 1.0 ? 1 : (k >= (double)n ? n : (int64_t)k);
}

int eig_setup(SolveState& S) {
  const qdwhp_opts& o = S.o;
  if (!(o.tol > 0.0) || !(o.s_eig > 0.0 && o.s_eig < 1.0) || o.eig_iters < 1 || o.eig_iters > 16 ||
      o.zolo_r < 0 || o.zolo_r > kZoloMax)
    return S.ret(-11);
  const int64_t n = S.n;
  const int64_t k = qdwhp_eig_count(n, S.fraction);
  S.k = k;
  S.info->k = k;
  S.nv = lz_vectors(o);
  S.msteps = lz_steps(o, n);
  S.sgn = (S.which == QDWHP_SMALLEST) ? -1.0 : 1.0;
  S.mm = S.nn = n;
  Arena ar(S.work, S.lwork);
  S.P = carve(ar, n, n, S.nv, S.msteps, false, o.zolo_r > 0);
  S.ev.reset(new Events(true));
  S.ev->mark(0, S.s);
  hipStream_t s = S.s;
  Plan& P = S.P;
  QDWHP_HIP(hipMemsetAsync(P.flags, 0, 8 * sizeof(int), s));
  nonfinite(S.A, S.lda, n, n, P.flags + 1, s);
  // ---- estimator (Algorithm 1 opens with a few Lanczos steps)
  S.replay = !is_nan(o.tau) && !is_nan(o.mu) && !is_nan(o.rho);
  if (!S.replay) {
    LanczosOp op;
    op.rows_tmp = 1;
    const double* A = S.A;
    const int64_t lda = S.lda;
    const double sgn = S.sgn;
    const int nv = S.nv;
    op.apply = [&](const double* in, int64_t ldi, double* out, int64_t ldo, double*, hipStream_t st) {
      // the big work block is free until the iterations start
      skinny_gemm(A, lda, n, n, in, ldi, nv, sgn, out, ldo, P.big, P.big_doubles, st);
    };
    S.lz = lanczos(op, n, S.nv, (int)S.msteps, o.seed, P.lz, s);
    if (S.lz.sweeps < 0) {   // a non-finite input shows up here first
      int hf[8];
      QDWHP_HIP(hipMemcpyAsync(hf, P.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
      QDWHP_HIP(hipStreamSynchronize(s));
      return S.ret(hf[1] ? QDWHP_ERR_NONFINITE : QDWHP_ERR_NOCONV);
    }
    S.lmax = -std::numeric_limits<double>::infinity();
    S.lmin = std::numeric_limits<double>::infinity();
    for (size_t i = 0; i < S.lz.nodes.size(); ++i) {
      S.lmax = std::max(S.lmax, S.lz.nodes[i] + S.lz.resid[i]);
      S.lmin = std::min(S.lmin, S.lz.nodes[i] - S.lz.resid[i]);
    }
  }
  S.info->lmax = S.lmax;
  S.info->lmin = S.lmin;
  S.ev->mark(1, s);
  return QDWHP_OK;
}

// Threshold for this attempt (boost), schedule, X0, polish plan.
void eig_prepare(SolveState& S) {
  const qdwhp_opts& o = S.o;
  const int64_t n = S.n;
  const double sfix = o.s_eig;
  if (S.replay) {
    S.tau = o.tau; S.mu = o.mu; S.rho = o.rho;
  } else {
    const double spread = std::max({S.lmax - S.lmin, std::fabs(S.lmax), std::fabs(S.lmin), 1e-300});
    if (!is_nan(o.tau)) {
      S.tau = S.sgn * o.tau;
    } else {
      double cut;
      const int64_t kt = target_count(n, S.k, S.boost);
      const bool ok = (o.tau_policy == 1 && o.zolo_r == 0)
          ? choose_tau_cost(S.lz.nodes, S.lz.weights, n, S.nv, S.lmax, S.lmin, kt, sfix, o.eig_iters,
                            o.kappa_max, o.tol, &cut)
          : cut_below(S.lz.nodes, S.lz.weights, n, S.nv, S.lmax, S.lmin, kt, &cut);
      S.tau = ok ? cut : S.lmin;
    }
    S.mu = std::max(S.lmax - S.tau, 1e-3 * spread);
    S.rho = std::max(0.0, (S.tau - S.lmin) / S.mu);
  }
  S.zsched.clear();
  if (o.zolo_r > 0) {
    S.sched.clear();
    S.zsched = zolo_schedule(sfix, o.zolo_r, o.kappa_max, std::max(1.0, (1.0 - sfix) * S.rho - sfix), false);
  } else {
    S.sched = eig_schedule(sfix, S.rho, o.eig_iters, o.kappa_max);
    for (size_t i = 0; i < S.sched.size() && i < 16; ++i)
      if (o.kinds[i] == QDWHP_KIND_QR || o.kinds[i] == QDWHP_KIND_CHOL) S.sched[i].kind = o.kinds[i];
  }
  S.info->retries = S.boost - 1;
  // ---- iterations on the scaled, shifted matrix (Sec. 4.1)
  S.X = S.P.X;
  S.Xn = S.P.Xn;
  eig_x0(S.A, S.lda, S.X, n, n, (1.0 - sfix) / S.mu, S.tau, S.sgn, sfix, S.s);
  S.sb = step_bufs(S.P, n, n);
  S.mixed = (o.precision == QDWHP_MIXED_FP32) && o.zolo_r == 0;
  double xbound = 1.0;
  for (const auto& st : S.sched) xbound = std::max(1.0, dwh_map(st.x, st.a, st.b, st.c));
  S.polish.clear();
  if (S.mixed) {
    // FP64 polish: Newton-Schulz while the unwanted side stays below
    // sqrt(3) (where it converges), else Halley's (3,1,3) step in
    // Cholesky form (monotone for any x)
    for (int p = 0; p < o.polish_steps; ++p) {
      if (xbound < 1.7) { S.polish.push_back(0); xbound = std::max(1.0, 0.5 * xbound * (3.0 - xbound * xbound)); }
      else { S.polish.push_back(1); xbound = std::max(1.0, dwh_map(xbound, 3.0, 1.0, 3.0)); }
    }
  }
}

// Projector, QR, ind/ell, Q2, Rayleigh-Ritz.  Returns 0 when this attempt
// is final (success or a final error in S.status), 1 when the threshold must
// be retried.
int eig_project(SolveState& S, std::vector<double>& theta, int64_t& ell, int64_t& ind, int64_t& n_above,
                double*& Q2, double*& Wv) {
  const qdwhp_opts& o = S.o;
  const int64_t n = S.n, k = S.k;
  hipStream_t s = S.s;
  Plan& P = S.P;
  double* X = S.X;
  S.ev->mark(2, s);
  // ---- projector (X + I)/2, QR, ind (Algorithm 1); with use_omega the
  // QR is of B Omega (the randomised rank-revealing form of Sec. 4.1)
  half_plus_identity(X, n, P.Z, n, n, s);
  double* Bq = P.Z;
  double* Q2buf = (X == P.X) ? P.Xn : P.X;
  if (o.use_omega) {
    gaussian_fill(Q2buf, n * n, o.seed + 3, 0, s);
    Gemm go;
    // Omega with N(0, 1/n) entries: B Omega keeps B's column norms on average
    go.M = n; go.N = n; go.K = n; go.alpha = 1.0 / std::sqrt((double)n);
    go.A = P.Z; go.lda = n; go.B = Q2buf; go.ldb = n; go.C = X; go.ldc = n;
    dgemm(go, s);
    Bq = X;
  }
  std::vector<double> d;
  const PanelWatch watch = diag_watch(Bq, n, P.diag, o.tol, &d, s);
  geqrf(Bq, n, projector_qr_cols(n, k, S.replay), n, P.tau, P.Tall, P.qrs, s, &watch);
  int hflags[8];
  QDWHP_HIP(hipMemcpyAsync(hflags, P.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  S.ev->mark(3, s);
  if (hflags[1]) { S.ret(QDWHP_ERR_NONFINITE); return 0; }
  if (hflags[0]) { S.ret(QDWHP_ERR_CHOL); return 0; }
  if (any_nonfinite(d)) { S.ret(QDWHP_ERR_NONFINITE); return 0; }
  ind = find_ind(d, o.tol);
  ell = n - ind + 1;
  if (ell <= 0 || (ell < k && !S.replay)) { S.status = QDWHP_ERR_NO_SUBSPACE; return S.replay ? 0 : 1; }
  // ---- Q2 = H_1 ... H_{ind-1} [0; I_ell]
  Q2 = Q2buf;
  double* Y = o.use_omega ? P.Z : X;          // the buffers free once Q2 is formed
  double* Wfree = o.use_omega ? X : P.Z;
  orgqr(Bq, n, n, P.Tall, ind - 1, ind - 1, ell, Q2, n, P.qrs, s);
  S.ev->mark(4, s);
  // ---- Rayleigh-Ritz on the original matrix: H = Q2^T (sgn A) Q2
  Gemm g1;
  g1.M = n; g1.N = ell; g1.K = n; g1.alpha = S.sgn; g1.A = S.A; g1.lda = S.lda; g1.B = Q2; g1.ldb = n;
  g1.C = Y; g1.ldc = n;
  dgemm(g1, s);
  double* H = P.big;
  Gemm g2;
  g2.M = ell; g2.N = ell; g2.K = n; g2.A = Q2; g2.lda = n; g2.ta = true; g2.B = Y; g2.ldb = n;
  g2.C = H; g2.ldc = ell; g2.tiles = TILES_UPPER;   // symmetric: the upper tiles, then mirrored
  dgemm(g2, s);
  mirror_upper(H, ell, ell, s);
  S.ev->mark(5, s);
  Wv = Wfree;
  int sweeps = -1;
  // the estimator's quadrature places the split unless it already
  // over-counted once (a retried threshold)
  S.info->rr_split = rr_split(H, ell, k, n, (S.replay || S.boost > 1) ? nullptr : &S.lz, S.lmax, S.lmin, o, P, Y,
                              n * n, Wv, n * n, P.big + ell * ell, P.vals, &sweeps, s);
  if (S.info->rr_split == 0) sweeps = syev(H, ell, ell, P.vals, Wv, ell, P.big + ell * ell, s);
  S.info->jacobi_sweeps = sweeps;
  if (sweeps < 0) { S.ret(QDWHP_ERR_NOCONV); return 0; }
  theta.resize(ell);
  QDWHP_HIP(hipMemcpyAsync(theta.data(), P.vals, sizeof(double) * ell, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  S.ev->mark(6, s);
  n_above = 0;
  for (double t : theta) n_above += (t >= S.tau);
  S.status = QDWHP_OK;
  if (n_above >= k || ell >= n || S.replay) return 0;
  S.status = QDWHP_ERR_NO_SUBSPACE;
  return 1;
}

int eig_finish(SolveState& S) {
  const int64_t n = S.n, k = S.k;
  hipStream_t s = S.s;
  std::vector<double> theta;
  int64_t ell = 0, ind = 0, n_above = 0;
  double* Q2 = nullptr;
  double* Wv = nullptr;
  while (eig_project(S, theta, ell, ind, n_above, Q2, Wv) == 1 && S.boost < 2) {
    ++S.boost;
    eig_prepare(S);
    iterate_state(S, S.o.graphs != 0, s);
  }
  qdwhp_info* info = S.info;
  info->tau = S.sgn * S.tau; info->mu = S.mu; info->rho = S.rho;
  info->ell = ell; info->ind = ind; info->n_above = n_above;
  if (S.zsched.empty()) fill_info(info, S.sched); else fill_info_zolo(info, S.zsched);
  if (S.status != QDWHP_OK) return S.ret(S.status);
  if (ell < k) return S.ret(QDWHP_ERR_NO_SUBSPACE);
  // ---- V = Q2 W(:, 1:k), w = sgn theta(1:k)
  Gemm g3;
  g3.M = n; g3.N = k; g3.K = ell; g3.A = Q2; g3.lda = n; g3.B = Wv; g3.ldb = ell; g3.C = S.V; g3.ldc = S.ldv;
  scale_vec(S.P.vals, S.w, k, S.sgn, s);
  if (S.df) {   // the caller launches the product and the sign step
    Deferred* df = S.df;
    df->g = g3; df->V = S.V; df->ldv = S.ldv; df->n = n; df->k = k; df->U = nullptr; df->ldu = 0; df->m = 0;
  } else {
    dgemm(g3, s);
    sign_normalize(S.V, S.ldv, n, k, nullptr, 0, 0, s);
  }
  S.ev->mark(7, s);
  S.ev->fill(info->ms);
  const double dn = (double)n, dl = (double)ell, dk = (double)k;
  info->flops_table1 = (S.zsched.empty() ? table1_iter_flops(S.sched, dn, dn) : table1_zolo_flops(S.zsched, dn, dn)) +
                       4.0 / 3.0 * dn * dn * dn +
                       2.0 * dn * dn * dl + 2.0 * dn * dl * dl + 9.0 * dl * dl * dl + 2.0 * dn * dl * dk;
  return S.ret(QDWHP_OK);
}

// ---- SVD (Algorithm 2) -----------------------------------------------------
int svd_setup(SolveState& S) {
  const qdwhp_opts& o = S.o;
  if (!(o.tol > 0.0) || o.zolo_r < 0 || o.zolo_r > kZoloMax) return S.ret(-13);
  hipStream_t s = S.s;
  const int64_t m = S.m, n = S.n;
  S.tr = m < n;                       // process M = A^T when A is wide
  const bool tr = S.tr;
  const int64_t mm = S.mm = std::max(m, n), nn = S.nn = std::min(m, n);
  S.info->k = S.k;
  S.nv = lz_vectors(o);
  S.msteps = lz_steps(o, nn);
  Arena ar(S.work, S.lwork);
  S.P = carve(ar, mm, nn, S.nv, S.msteps, true, o.zolo_r > 0);
  Plan& P = S.P;
  S.ev.reset(new Events(true));
  S.ev->mark(0, s);
  QDWHP_HIP(hipMemsetAsync(P.flags, 0, 8 * sizeof(int), s));
  nonfinite(S.A, S.lda, m, n, P.flags + 1, s);
  S.replay = !is_nan(o.alpha) && !is_nan(o.s_svd);
  if (!S.replay || is_nan(o.alpha)) {
    // operator M^T M on nn-vectors; M = A (tall) or A^T (wide)
    const double* A = S.A;
    const int64_t lda = S.lda;
    const int nv = S.nv;
    LanczosOp op;
    op.rows_tmp = mm;
    op.apply = [&](const double* in, int64_t ldi, double* out, int64_t ldo, double* tmp, hipStream_t st) {
      // tmp = M in (mm x nv), out = M^T tmp (nn x nv), as skinny products
      // (the big work block is free until the iterations start); the
      // transposed kernel takes up to 8 columns, wider blocks use the GEMM
      auto at_b = [&](int64_t rows, int64_t cols, const double* B, int64_t ldb, double* C, int64_t ldc) {
        if (nv <= 8) {
          skinny_gemm_t(A, lda, rows, cols, B, ldb, nv, 1.0, C, ldc, st);
        } else {
          Gemm g;
          g.M = cols; g.N = nv; g.K = rows; g.A = A; g.lda = lda; g.ta = true; g.B = B; g.ldb = ldb;
          g.C = C; g.ldc = ldc;
          dgemm(g, st);
        }
      };
      if (!tr) {
        skinny_gemm(A, lda, mm, nn, in, ldi, nv, 1.0, tmp, mm, P.big, P.big_doubles, st);
        at_b(mm, nn, tmp, mm, out, ldo);
      } else {
        at_b(nn, mm, in, ldi, tmp, mm);
        skinny_gemm(A, lda, nn, mm, tmp, mm, nv, 1.0, out, ldo, P.big, P.big_doubles, st);
      }
    };
    S.lz = lanczos(op, nn, S.nv, (int)S.msteps, o.seed, P.lz, s);
    if (S.lz.sweeps < 0) {   // a non-finite input shows up here first
      int hf[8];
      QDWHP_HIP(hipMemcpyAsync(hf, P.flags, sizeof(hf), hipMemcpyDeviceToHost, s));
      QDWHP_HIP(hipStreamSynchronize(s));
      return S.ret(hf[1] ? QDWHP_ERR_NONFINITE : QDWHP_ERR_NOCONV);
    }
    S.lmax = -std::numeric_limits<double>::infinity();
    S.lmin = std::numeric_limits<double>::infinity();
    for (size_t i = 0; i < S.lz.nodes.size(); ++i) {
      S.lmax = std::max(S.lmax, S.lz.nodes[i] + S.lz.resid[i]);
      S.lmin = std::min(S.lmin, S.lz.nodes[i] - S.lz.resid[i]);
    }
  }
  S.info->lmax = S.lmax;
  S.info->lmin = S.lmin;
  S.ev->mark(1, s);
  return QDWHP_OK;
}

void svd_prepare(SolveState& S) {
  const qdwhp_opts& o = S.o;
  const int64_t mm = S.mm, nn = S.nn;
  if (S.replay) {
    S.alpha = o.alpha; S.sthr = o.s_svd;
  } else {
    S.alpha = std::sqrt(std::max(S.lmax, 0.0));
    if (!(S.alpha > 0.0)) S.alpha = 1e-300;
    if (!is_nan(o.alpha)) S.alpha = o.alpha;
    if (!is_nan(o.s_svd)) {
      S.sthr = o.s_svd;
    } else {
      double cut;
      const double t = cut_below(S.lz.nodes, S.lz.weights, nn, S.nv, S.lmax, S.lmin,
                                 target_count(nn, S.k, S.boost), &cut, true) ? std::max(cut, 0.0) : 0.0;
      S.sthr = std::min(1.0, std::max(1e-15, std::sqrt(t) / S.alpha));
    }
  }
  S.zsched.clear();
  if (o.zolo_r > 0) {
    S.sched.clear();
    S.zsched = zolo_schedule(S.sthr, o.zolo_r, o.kappa_max, 1.0, o.svd_qr_first != 0 || S.sthr < 1e-3);
  } else {
    S.sched = svd_schedule(S.sthr, o.kappa_max, o.svd_qr_first != 0);
    for (size_t i = 0; i < S.sched.size() && i < 16; ++i)
      if (o.kinds[i] == QDWHP_KIND_QR || o.kinds[i] == QDWHP_KIND_CHOL) S.sched[i].kind = o.kinds[i];
  }
  S.info->retries = S.boost - 1;
  S.X = S.P.X;
  S.Xn = S.P.Xn;
  scale_copy(S.A, S.lda, S.X, mm, mm, nn, 1.0 / S.alpha, S.tr, S.s);
  S.sb = step_bufs(S.P, mm, nn);
  S.mixed = (o.precision == QDWHP_MIXED_FP32) && o.zolo_r == 0;
  // FP64 Newton-Schulz polish steps (singular values of X lie in [0, 1 + O(u_32)])
  S.polish.assign(S.mixed ? std::max(0, o.polish_steps) : 0, 0);
}

int svd_project(SolveState& S, std::vector<double>& sig, int64_t& ell, int64_t& ind, int64_t& n_above,
                double*& Q2, double*& Y, double*& Ut, double*& Vt) {
  const qdwhp_opts& o = S.o;
  const int64_t mm = S.mm, nn = S.nn, k = S.k;
  hipStream_t s = S.s;
  Plan& P = S.P;
  double* X = S.X;
  S.ev->mark(2, s);
  // ---- projector I - X^T X, QR, ind (Algorithm 2)
  Gemm gb;
  gb.M = nn; gb.N = nn; gb.K = mm; gb.alpha = -1.0; gb.diag = 1.0; gb.A = X; gb.lda = mm; gb.ta = true;
  gb.B = X; gb.ldb = mm; gb.C = P.Z; gb.ldc = nn; gb.tiles = TILES_UPPER;
  dgemm(gb, s);
  mirror_upper(P.Z, nn, nn, s);
  std::vector<double> d;
  const PanelWatch watch = diag_watch(P.Z, nn, P.diag, o.tol, &d, s);
  geqrf(P.Z, nn, projector_qr_cols(nn, k, S.replay), nn, P.tau, P.Tall, P.qrs, s, &watch);
  int hflags[8];
  QDWHP_HIP(hipMemcpyAsync(hflags, P.flags, sizeof(hflags), hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  S.ev->mark(3, s);
  if (hflags[1]) { S.ret(QDWHP_ERR_NONFINITE); return 0; }
  if (hflags[0]) { S.ret(QDWHP_ERR_CHOL); return 0; }
  if (any_nonfinite(d)) { S.ret(QDWHP_ERR_NONFINITE); return 0; }
  ind = find_ind(d, o.tol);
  ell = nn - ind + 1;
  if (ell <= 0 || (ell < k && !S.replay)) { S.status = QDWHP_ERR_NO_SUBSPACE; return S.replay ? 0 : 1; }
  Q2 = (X == P.X) ? P.Xn : P.X;
  Y = X;
  orgqr(P.Z, nn, nn, P.Tall, ind - 1, ind - 1, ell, Q2, nn, P.qrs, s);
  S.ev->mark(4, s);
  // ---- Y = M Q2 = Q_Y R_Y, SVD of R_Y (Algorithm 2 projection step)
  Gemm gy;
  gy.M = mm; gy.N = ell; gy.K = nn; gy.A = S.A; gy.lda = S.lda; gy.ta = S.tr; gy.B = Q2; gy.ldb = nn;
  gy.C = Y; gy.ldc = mm;
  dgemm(gy, s);
  geqrf(Y, mm, ell, mm, P.tau, P.Tall, P.qrs, s);
  Ut = P.Z;
  upper_copy(Y, mm, Ut, ell, ell, s);
  S.ev->mark(5, s);
  int sweeps = -1;
  // the small SVD: QDWH-SVD (polar factor, then the symmetric
  // eigenproblem) above "rr.svd_polar" rows, else one-sided Jacobi
  const int64_t polar_min = qdwhp_tune_get("rr.svd_polar", 256);
  if (polar_min > 0 && ell >= polar_min)
    sweeps = polar_svd(Ut, ell, S.alpha, P.vals, Vt, P.big, P.big_doubles, o, P.flags, s);
  if (sweeps < 0) {
    Vt = P.big + gesvj_scratch_doubles(ell, ell);
    sweeps = gesvj(Ut, ell, ell, ell, P.vals, Vt, ell, P.big, s);
  }
  S.info->jacobi_sweeps = sweeps;
  if (sweeps < 0) { S.ret(QDWHP_ERR_NOCONV); return 0; }
  sig.resize(ell);
  QDWHP_HIP(hipMemcpyAsync(sig.data(), P.vals, sizeof(double) * ell, hipMemcpyDeviceToHost, s));
  QDWHP_HIP(hipStreamSynchronize(s));
  S.ev->mark(6, s);
  n_above = 0;
  for (double v : sig) n_above += (v >= S.sthr * S.alpha);
  S.status = QDWHP_OK;
  if (n_above >= k || ell >= nn || S.replay) return 0;
  S.status = QDWHP_ERR_NO_SUBSPACE;
  return 1;
}

int svd_finish(SolveState& S) {
  const int64_t mm = S.mm, nn = S.nn, k = S.k;
  hipStream_t s = S.s;
  std::vector<double> sig;
  int64_t ell = 0, ind = 0, n_above = 0;
  double *Q2 = nullptr, *Y = nullptr, *Ut = nullptr, *Vt = nullptr;
  while (svd_project(S, sig, ell, ind, n_above, Q2, Y, Ut, Vt) == 1 && S.boost < 2) {
    ++S.boost;
    svd_prepare(S);
    iterate_state(S, S.o.graphs != 0, s);
  }
  qdwhp_info* info = S.info;
  info->alpha = S.alpha; info->s = S.sthr;
  info->ell = ell; info->ind = ind; info->n_above = n_above;
  if (S.zsched.empty()) fill_info(info, S.sched); else fill_info_zolo(info, S.zsched);
  if (S.status != QDWHP_OK) return S.ret(S.status);
  if (ell < k) return S.ret(QDWHP_ERR_NO_SUBSPACE);
  Plan& P = S.P;
  // ---- U_M = Q_Y [U~_k; 0], V_M = Q2 V~_k; A = M or M^T
  double* Um = S.tr ? S.V : S.U;
  const int64_t ldum = S.tr ? S.ldv : S.ldu;
  double* Vm = S.tr ? S.U : S.V;
  const int64_t ldvm = S.tr ? S.ldu : S.ldv;
  fill(Um, mm, k, ldum, 0.0, 0.0, s);
  copy(Ut, ell, Um, ldum, ell, k, s);
  apply_q(Y, mm, mm, P.Tall, ell, Um, k, ldum, P.qrs, s);
  Gemm gv;
  gv.M = nn; gv.N = k; gv.K = ell; gv.A = Q2; gv.lda = nn; gv.B = Vt; gv.ldb = ell; gv.C = Vm; gv.ldc = ldvm;
  scale_vec(P.vals, S.w, k, 1.0, s);
  if (S.df) {
    Deferred* df = S.df;
    df->g = gv; df->V = S.V; df->ldv = S.ldv; df->n = S.n; df->k = k; df->U = S.U; df->ldu = S.ldu; df->m = S.m;
  } else {
    dgemm(gv, s);
    sign_normalize(S.V, S.ldv, S.n, k, S.U, S.ldu, S.m, s);
  }
  S.ev->mark(7, s);
  S.ev->fill(info->ms);
  const double dm = (double)mm, dn = (double)nn, dl = (double)ell, dk = (double)k;
  info->flops_table1 = (S.zsched.empty() ? table1_iter_flops(S.sched, dm, dn) : table1_zolo_flops(S.zsched, dm, dn)) +
                       dm * dn * dn + 4.0 / 3.0 * dn * dn * dn +
                       2.0 * dm * dn * dl + 2.0 * dm * dl * dl + 17.0 * dl * dl * dl +
                       2.0 * dm * dl * dk + 2.0 * dn * dl * dk;
  return S.ret(QDWHP_OK);
}

// Argument checks of the two drivers (LAPACK-style negative codes).
int check_eig(const double* A, int64_t n, int64_t lda, double fraction, int which, const double* w,
              const double* V, int64_t ldv, const void* work) {
  if (!A) return -1;
  if (n < 1) return -2;
  if (lda < n) return -3;
  if (!(fraction > 0.0) || fraction > 1.0) return -4;
  if (which != QDWHP_LARGEST && which != QDWHP_SMALLEST) return -5;
  if (!w) return -6;
  if (!V) return -7;
  if (ldv < n) return -8;
  if (!work) return -9;
  return 0;
}

int check_svd(const double* A, int64_t m, int64_t n, int64_t lda, int64_t k, const double* U, int64_t ldu,
              const double* S, const double* V, int64_t ldv, const void* work) {
  if (!A) return -1;
  if (m < 1) return -2;
  if (n < 1) return -3;
  if (lda < m) return -4;
  if (k < 1 || k > std::min(m, n)) return -5;
  if (!U) return -6;
  if (ldu < m) return -7;
  if (!S) return -8;
  if (!V) return -9;
  if (ldv < n) return -10;
  if (!work) return -11;
  return 0;
}

// Runs f, mapping the library's exceptions to status codes.
template <class F>
int guarded(SolveState& S, F&& f) {
  try {
    return f();
  } catch (const WorkspaceError&) {
    return S.ret(QDWHP_ERR_WORKSPACE);
  } catch (const HipError&) {
    return S.ret(QDWHP_ERR_HIP);
  }
}

}  // namespace

namespace qdwhp {

SolveState* solve_create(const qdwhp_problem& p, void* work, size_t lwork, const qdwhp_opts* opts,
                         hipStream_t s, qdwhp_info* info, Deferred* df) {
  auto* S = new SolveState();
  S->svd = (p.type == QDWHP_PROBLEM_SVD);
  S->A = p.A; S->lda = p.lda; S->n = p.n; S->m = S->svd ? p.m : p.n;
  S->fraction = p.fraction; S->which = p.which; S->k = p.k;
  S->w = p.w; S->U = p.U; S->ldu = p.ldu; S->V = p.V; S->ldv = p.ldv;
  S->work = work; S->lwork = lwork;
  if (opts) S->o = *opts; else qdwhp_opts_default(&S->o);
  S->s = s;
  S->info = info;
  S->df = df;
  std::memset(info, 0, sizeof(*info));
  return S;
}

void solve_destroy(SolveState* S) { delete S; }
int solve_status(const SolveState* S) { return S->status; }
void solve_set_stream(SolveState* S, hipStream_t s) { S->s = s; }

int solve_setup(SolveState* S) {
  SolveState& st = *S;
  const int bad = st.svd ? check_svd(st.A, st.m, st.n, st.lda, st.k, st.U, st.ldu, st.w, st.V, st.ldv, st.work)
                         : check_eig(st.A, st.n, st.lda, st.fraction, st.which, st.w, st.V, st.ldv, st.work);
  if (bad) return st.ret(bad);
  return guarded(st, [&] {
    const int r = st.svd ? svd_setup(st) : eig_setup(st);
    if (r != QDWHP_OK) return r;
    if (st.svd) svd_prepare(st); else eig_prepare(st);
    return QDWHP_OK;
  });
}

int solve_iterate(SolveState* S) {
  SolveState& st = *S;
  return guarded(st, [&] {
    iterate_state(st, st.o.graphs != 0, st.s);
    return QDWHP_OK;
  });
}

int solve_finish(SolveState* S) {
  SolveState& st = *S;
  return guarded(st, [&] { return st.svd ? svd_finish(st) : eig_finish(st); });
}

int eig_impl(const double* A, int64_t n, int64_t lda, double fraction, int which, double* w, double* V,
             int64_t ldv, void* work, size_t lwork, const qdwhp_opts* opts, void* stream, qdwhp_info* info,
             Deferred* df) {
  qdwhp_info dummy;
  qdwhp_problem p{};
  p.type = QDWHP_PROBLEM_EIG; p.which = which; p.m = n; p.n = n; p.A = A; p.lda = lda; p.fraction = fraction;
  p.w = w; p.V = V; p.ldv = ldv;
  std::unique_ptr<SolveState> S(solve_create(p, work, lwork, opts, (hipStream_t)stream, info ? info : &dummy, df));
  int r = solve_setup(S.get());
  if (r == QDWHP_OK) r = solve_iterate(S.get());
  if (r == QDWHP_OK) r = solve_finish(S.get());
  return r;
}

int svd_impl(const double* A, int64_t m, int64_t n, int64_t lda, int64_t k, double* U, int64_t ldu, double* S_,
             double* V, int64_t ldv, void* work, size_t lwork, const qdwhp_opts* opts, void* stream,
             qdwhp_info* info, Deferred* df) {
  qdwhp_info dummy;
  qdwhp_problem p{};
  p.type = QDWHP_PROBLEM_SVD; p.m = m; p.n = n; p.A = A; p.lda = lda; p.k = k;
  p.w = S_; p.U = U; p.ldu = ldu; p.V = V; p.ldv = ldv;
  std::unique_ptr<SolveState> S(solve_create(p, work, lwork, opts, (hipStream_t)stream, info ? info : &dummy, df));
  int r = solve_setup(S.get());
  if (r == QDWHP_OK) r = solve_iterate(S.get());
  if (r == QDWHP_OK) r = solve_finish(S.get());
  return r;
}

}  // namespace qdwhp

extern "C" int qdwhp_eig(const double* A, int64_t n, int64_t lda, double fraction, int which,
                         double* w, double* V, int64_t ldv, void* work, size_t lwork,
                         const qdwhp_opts* opts, void* stream, qdwhp_info* info) {
  return eig_impl(A, n, lda, fraction, which, w, V, ldv, work, lwork, opts, stream, info, nullptr);
}

extern "C" int qdwhp_svd(const double* A, int64_t m, int64_t n, int64_t lda, int64_t k,
                         double* U, int64_t ldu, double* S, double* V, int64_t ldv,
                         void* work, size_t lwork, const qdwhp_opts* opts, void* stream,
                         qdwhp_info* info) {
  return svd_impl(A, m, n, lda, k, U, ldu, S, V, ldv, work, lwork, opts, stream, info, nullptr);
}

// ===========================================================================
// Building blocks.

extern "C" size_t qdwhp_spd_inverse_workspace(int64_t n) {
  return n < 1 ? 0 : (size_t)(spd_inverse_doubles(n) + 64) * 8;
}

extern "C" int qdwhp_spd_inverse(double* Z, int64_t n, int64_t ldz, void* work, size_t lwork, void* stream) {
  if (!Z) return -1;
  if (n < 1) return -2;
  if (ldz < n) return -3;
  if (!work) return -4;
  if (lwork < qdwhp_spd_inverse_workspace(n)) return QDWHP_ERR_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  try {
    double* ws = (double*)work;
    int* flag = (int*)(ws + spd_inverse_doubles(n));
    QDWHP_HIP(hipMemsetAsync(flag, 0, sizeof(int), s));
    spd_inverse(Z, n, ldz, ws, flag, s);
    int h = 0;
    QDWHP_HIP(hipMemcpyAsync(&h, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    QDWHP_HIP(hipStreamSynchronize(s));
    if (h) return QDWHP_ERR_CHOL;
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

extern "C" size_t qdwhp_geqrf_workspace(int64_t m, int64_t n) {
  if (m < 1 || n < 1) return 0;
  return (size_t)(qr_t_doubles(n) + qr_scratch_doubles(m, n) + 64) * 8 + 512;
}

extern "C" int qdwhp_geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, void* work,
                           size_t lwork, void* stream) {
  if (!A) return -1;
  if (m < 1) return -2;
  if (n < 1 || n > m) return -3;
  if (lda < m) return -4;
  if (!tau) return -5;
  if (!work) return -6;
  if (lwork < qdwhp_geqrf_workspace(m, n)) return QDWHP_ERR_WORKSPACE;
  try {
    double* Tall = (double*)work;
    QrScratch sc = carve_qr_scratch(Tall + qr_t_doubles(n), m, n);
    fill(Tall, QB, cdiv(n, QB) * QB, QB, 0.0, 0.0, (hipStream_t)stream);
    geqrf(A, m, n, lda, tau, Tall, sc, (hipStream_t)stream);
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

extern "C" int qdwhp_orgqr(const double* A, int64_t m, int64_t n, int64_t lda, const double* tau,
                           int64_t c0, int64_t q, double* Q, int64_t ldq, void* work, size_t lwork,
                           void* stream) {
  (void)tau;
  if (!A) return -1;
  if (m < 1) return -2;
  if (n < 1 || n > m) return -3;
  if (lda < m) return -4;
  if (c0 < 0 || c0 > m) return -6;
  if (q < 0 || q > n || c0 + q > m) return -7;
  if (!Q) return -8;
  if (ldq < m) return -9;
  if (!work) return -10;
  if (lwork < qdwhp_geqrf_workspace(m, n)) return QDWHP_ERR_WORKSPACE;
  try {
    double* Tall = (double*)work;
    QrScratch sc = carve_qr_scratch(Tall + qr_t_doubles(n), m, n);
    orgqr(A, m, lda, Tall, n, c0, q, Q, ldq, sc, (hipStream_t)stream);
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

extern "C" size_t qdwhp_syev_workspace(int64_t n) {
  return n < 1 ? 0 : (size_t)(syev_scratch_doubles(n) + 64) * 8;
}

extern "C" int qdwhp_syev(double* H, int64_t n, int64_t ldh, double* w, double* W, int64_t ldw,
                          void* work, size_t lwork, void* stream, int* sweeps) {
  if (!H) return -1;
  if (n < 1) return -2;
  if (ldh < n) return -3;
  if (!w) return -4;
  if (!W) return -5;
  if (ldw < n) return -6;
  if (!work) return -7;
  if (lwork < qdwhp_syev_workspace(n)) return QDWHP_ERR_WORKSPACE;
  try {
    const int sw = syev(H, n, ldh, w, W, ldw, (double*)work, (hipStream_t)stream);
    if (sweeps) *sweeps = sw;
    if (sw < 0) return QDWHP_ERR_NOCONV;
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

extern "C" size_t qdwhp_gesvj_workspace(int64_t n) {
  return n < 1 ? 0 : (size_t)(gesvj_scratch_doubles(n, n) + 64) * 8;
}

extern "C" int qdwhp_gesvj(double* R, int64_t n, int64_t ldr, double* S, double* V, int64_t ldv,
                           void* work, size_t lwork, void* stream, int* sweeps) {
  if (!R) return -1;
  if (n < 1) return -2;
  if (ldr < n) return -3;
  if (!S) return -4;
  if (!V) return -5;
  if (ldv < n) return -6;
  if (!work) return -7;
  if (lwork < qdwhp_gesvj_workspace(n)) return QDWHP_ERR_WORKSPACE;
  try {
    const int sw = gesvj(R, n, n, ldr, S, V, ldv, (double*)work, (hipStream_t)stream);
    QDWHP_HIP(hipStreamSynchronize((hipStream_t)stream));
    if (sweeps) *sweeps = sw;
    if (sw < 0) return QDWHP_ERR_NOCONV;
  } catch (const HipError&) {
    return QDWHP_ERR_HIP;
  }
  return QDWHP_OK;
}

// ===========================================================================
// DWH steps of a group of solves of one shape (phase 2 of a batch or a server
// group): the operations of chol_step for all Cholesky-based members at once.
int64_t qdwhp::solve_shape(const SolveState* S) {
  // solves with Zolotarev steps never share a key (they are not grouped)
  if (!S->zsched.empty()) return -1 - (int64_t)(intptr_t)S;
  return ((S->svd ? 1 : 0) | ((int64_t)(S->mixed ? 1 : 0) << 1)) + 4 * (S->mm * 2000003 + S->nn);
}

void qdwhp::iterations_grouped(SolveState* const* v, int count, void* table, hipStream_t s) {
  if (count <= 0) return;
  if (count == 1) {    // a group of one is the solve's own iterations
    iterate_state(*v[0], false, s);
    return;
  }
  const int64_t m = v[0]->mm, n = v[0]->nn;
  const bool sym = !v[0]->svd;
  for (int q = 1; q < count; ++q)
    if (solve_shape(v[q]) != solve_shape(v[0])) throw HipError{hipErrorInvalidValue};
  size_t steps = 0;
  for (int q = 0; q < count; ++q) steps = std::max(steps, v[q]->sched.size());
  std::vector<GroupedDesc> gram, prod1, prod2;
  std::vector<CholItem> chol;
  std::vector<SolveState*> grp;
  for (size_t i = 0; i < steps; ++i) {
    grp.clear();
    for (int q = 0; q < count; ++q) {
      SolveState& S = *v[q];
      if (i >= S.sched.size()) continue;
      const DwhStep& st = S.sched[i];
      const bool f32 = S.mixed && i + 1 < S.sched.size();
      if (st.kind == 1) qr_step(S.X, m, n, st.a, st.b, st.c, sym, S.sb, s);
      else if (f32) chol_step(S.X, S.Xn, m, n, st.a, st.b, st.c, sym, S.sb, s, true);
      else grp.push_back(&S);
    }
    if (grp.empty()) continue;
    gram.clear(); prod1.clear(); prod2.clear(); chol.clear();
    for (SolveState* p : grp) {
      SolveState& S = *p;
      const DwhStep& st = S.sched[i];
      double* Wi = S.sb.spd;
      double* T = S.sb.spd + spd_inverse_doubles(n);
      GroupedDesc g{n, n, m, st.c, 0.0, S.X, m, S.X, m, S.sb.Z, n};   // Z = I + c X^T X (upper tiles)
      g.diag = 1.0;
      g.tiles = TILES_UPPER;
      gram.push_back(g);
      chol.push_back(CholItem{S.sb.Z, n, S.sb.spd, S.sb.flag});
      GroupedDesc t{m, n, n, 1.0, 0.0, S.X, m, Wi, n, T, m};          // T = X W^{-1}
      t.khi = KHI_COL;
      prod1.push_back(t);
      GroupedDesc u{m, n, n, st.a - st.b / st.c, st.b / st.c, T, m, Wi, n, S.Xn, m};   // X+ = (b/c) X + (a - b/c) T W^{-T}
      u.Cin = S.X; u.ldcin = m; u.klo = KLO_COL;
      if (sym) u.tiles = TILES_UPPER;
      prod2.push_back(u);
    }
    const int cnt = (int)grp.size();
    dgemm_grouped(gram.data(), cnt, true, false, table, s);
    chol_inverse_grouped(chol.data(), cnt, n, table, s);
    dgemm_grouped(prod1.data(), cnt, false, false, table, s);
    dgemm_grouped(prod2.data(), cnt, false, true, table, s);
    for (SolveState* p : grp) {
      if (sym) mirror_upper(p->Xn, n, m, s);
      std::swap(p->X, p->Xn);
    }
  }
  for (int q = 0; q < count; ++q) {
    SolveState& S = *v[q];
    for (int pl : S.polish) {
      if (pl == 0) ns_step(S.X, S.Xn, m, n, sym, S.sb, s);
      else chol_step(S.X, S.Xn, m, n, 3.0, 1.0, 3.0, sym, S.sb, s, false);
    }
  }
}
