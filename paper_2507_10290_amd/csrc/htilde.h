// The per-segment system matrix of eq. QpSubProblem in the normalised-time
// basis c~_j = c_j T^j, and its inverse, in float64:
//   Htilde = 2 T^(1-2p) Q(1) + rho [ left knot rows + right knot rows + 2 sum_s tau_s tau_s^T
//                                    + T^-2 sum_s tau'_s tau'_s^T ]
// (the box rows come in upper/lower pairs, hence the 2; the velocity rows carry 1/T).
#pragma once

#include "common.h"

namespace top {

// iTp[o] = T^-o for o < 2N at least up to 2p - 1.
template <int P, int S, bool BOX, bool VEL>
__device__ inline void build_htilde(const double* iTp, double iT, double rho, bool first, bool last,
                                    double (&H)[2 * P][2 * P]) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  const double sq = 2.0 * iTp[2 * P - 1];
#pragma unroll
  for (int j = 0; j < N; ++j)
#pragma unroll
    for (int k = 0; k < N; ++k) H[j][k] = sq * cgram(P, j, k);
  const int nL = first ? P : S;
  const int nR = last ? P : S;
  for (int o = 0; o < nL; ++o) {
    const double v = cfact(o) * iTp[o];
    H[o][o] += rho * v * v;
  }
  for (int o = 0; o < nR; ++o) {
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int k = 0; k < N; ++k) H[j][k] += rho * (cfall(o, j) * iTp[o]) * (cfall(o, k) * iTp[o]);
  }
  if (BOX) {
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 0; k < N; ++k) H[j][k] += rho * 2.0 * cpos(s, j) * cpos(s, k);
  }
  if (VEL) {
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 0; k < N; ++k) H[j][k] += rho * iT * iT * cvel(s, j) * cvel(s, k);
  }
}

// Inverse of a symmetric positive definite matrix by Cholesky H = L L^T, then Hi = L^-T L^-1.
// H is overwritten (its lower triangle holds L).
template <int N>
__device__ inline void spd_inverse(double (&H)[N][N], double (&Hi)[N][N]) {
  for (int j = 0; j < N; ++j) {
    double d = H[j][j];
    for (int k = 0; k < j; ++k) d -= H[j][k] * H[j][k];
    d = sqrt(d);
    H[j][j] = d;
    for (int r = j + 1; r < N; ++r) {
      double v = H[r][j];
      for (int k = 0; k < j; ++k) v -= H[r][k] * H[j][k];
      H[r][j] = v / d;
    }
  }
  double Li[N][N];
  for (int c = 0; c < N; ++c) {
    for (int r = 0; r < N; ++r) {
      if (r < c) { Li[r][c] = 0.0; continue; }
      double v = (r == c) ? 1.0 : 0.0;
      for (int k = c; k < r; ++k) v -= H[r][k] * Li[k][c];
      Li[r][c] = v / H[r][r];
    }
  }
  for (int r = 0; r < N; ++r) {
    for (int c = r; c < N; ++c) {
      double v = 0.0;
      for (int k = c; k < N; ++k) v += Li[k][r] * Li[k][c];
      Hi[r][c] = Hi[c][r] = v;
    }
  }
}

}  // namespace top
