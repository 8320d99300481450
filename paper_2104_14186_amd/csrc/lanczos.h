// Lanczos estimator (see lanczos.hip).
//
// Philox stream layout: entry i of stream `stream` uses pair index p = i/2,
// counter (p mod 2^32, p >> 32, stream, 0), key (seed mod 2^32, seed >> 32);
// words (w0, w1) and (w2, w3) give u1, u2 = ((w >> 5) 2^26 + (w' >> 6) + 1/2) 2^-53;
// entry 2p = sqrt(-2 ln u1) cos(2 pi u2), entry 2p+1 = sqrt(-2 ln u1) sin(2 pi u2).
// Run i starts from stream i; a restart of run i at step j draws stream
// nv + i*m + j.
#pragma once
#include <algorithm>
#include <cmath>
#include <functional>
#include <vector>

#include "common.h"

namespace qdwhp {

struct LanczosOp {
  // out (n x nv, ld ldo) = Op(in) for in = n x nv columns with column stride ldi
  std::function<void(const double* in, int64_t ldi, double* out, int64_t ldo, double* tmp,
                     hipStream_t s)> apply;
  int64_t rows_tmp = 1;   // rows of the temporary (e.g. m for A^T A)
};

struct LanczosResult {
  std::vector<double> nodes, weights, resid, alpha, beta;
  int nv = 0, m = 0; int64_t n = 0;
  int sweeps = 0;   // -1 if a tridiagonal eigenproblem did not converge
};

int64_t lanczos_doubles(int64_t n, int64_t rows_op, int nv, int m);
// out[0 .. count) = Gaussian entries 0 .. count-1 of Philox stream `stream`
// (the layout above).
void gaussian_fill(double* out, int64_t count, uint64_t seed, uint64_t stream, hipStream_t s);
LanczosResult lanczos(const LanczosOp& op, int64_t n, int nv, int m, uint64_t seed, double* ws,
                      hipStream_t s);

}  // namespace qdwhp
