// Householder QR building blocks (see qr.hip).
#pragma once
#include <functional>

#include "common.h"

namespace qdwhp {

constexpr int QB = 128;   // panel width and T-factor block

struct QrScratch {
  double* part; double* piv; double* G; double* W1; double* W2;
  double* ws; int64_t ws_doubles;
  // Cholesky-QR / Householder-reconstruction panels: partial Grams, small
  // factors, failure flag, and a copy of the panel (backup_rows x QB)
  double* cq_part = nullptr; double* cq_small = nullptr; int* cq_flag = nullptr;
  double* backup = nullptr; int64_t backup_rows = 0;
  // the trailing updates' buffers on the helper stream (W1, W2, split-K scratch)
  double* W1b = nullptr; double* W2b = nullptr; double* wsb = nullptr; int64_t wsb_doubles = 0;
};

int64_t qr_scratch_doubles(int64_t m, int64_t n);
QrScratch carve_qr_scratch(double* w, int64_t m, int64_t n);
inline int64_t qr_t_doubles(int64_t n) { return cdiv(n > 0 ? n : 1, QB) * QB * QB; }

// Called after each panel (columns c0 .. c0+w-1 factored, their T built,
// trailing columns not yet updated); returning true ends the factorization.
using PanelWatch = std::function<bool(int64_t c0, int w)>;

// In-place QR of A (m x n, m >= n): R above, reflectors below, tau[n];
// per-panel T factors in Tall (QB x QB each, zero below the diagonal).
// Returns the number of columns factored (n unless `watch` stopped early).
// recon: factor sub-panels by Cholesky QR with Householder reconstruction
// where they pass its checks (not while the stream is being captured; the
// tuning key "qr.recon" = 0 turns it off); the host then waits for the
// stream once per panel.  Then the trailing updates also run on a helper
// stream, overlapping the factorization of the next panel ("qr.overlap" =
// 0 turns that off; the next panel's columns then go through a narrower
// product whose K split differs, so results agree to rounding, not bits).
// stacked > 0: A is [A1; I] with A1 the first `stacked` rows and an n x n
// identity below (the QR-based step's [sqrt(c) X; I]); panels and updates
// then skip the rows of the identity block no reflector has reached yet
// (pass the same value to apply_q / orgqr).
int64_t geqrf(double* A, int64_t m, int64_t n, int64_t lda, double* tau, double* Tall,
              const QrScratch& sc, hipStream_t s, const PanelWatch* watch = nullptr, bool recon = true,
              int64_t stacked = 0);
// Q (m x q) = H_1 ... H_upto E, E = columns c0 .. c0+q-1 of the identity.
// C (m x q) <- H_1 ... H_upto C.
void apply_q(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
             double* C, int64_t q, int64_t ldc, const QrScratch& sc, hipStream_t s, int64_t stacked = 0);
void orgqr(const double* A, int64_t m, int64_t lda, const double* Tall, int64_t upto,
           int64_t c0, int64_t q, double* Q, int64_t ldq, const QrScratch& sc, hipStream_t s,
           int64_t stacked = 0);

}  // namespace qdwhp
