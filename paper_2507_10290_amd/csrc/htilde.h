// The per-segment system matrix of eq. QpSubProblem in the normalised-time
// basis c~_j = c_j T^j, and its inverse, in float64:
//   Htilde = 2 T^(1-2p) Q(1) + rho [ left knot rows + right knot rows + w sum_s tau_s tau_s^T
//                                    + T^-2 sum_s tau'_s tau'_s^T ]
// The velocity rows carry 1/T.  w weighs the corridor's sample rows: a box has an upper and a
// lower row per axis and sample (w = 2); a polytope's rows a_k (x) tau_s add
// (sum_k a_k a_k^T) (x) (sum_s tau_s tau_s^T), which the rotation to the eigenvectors of
// sum_k a_k a_k^T splits into one matrix per rotated axis with w = its eigenvalue.
#pragma once

#include "common.h"

namespace top {

// iTp[o] = T^-o for o < 2N at least up to 2p - 1.
template <int P, int S, bool VEL>
__device__ inline void build_htilde(const double* iTp, double iT, double rho, bool first, bool last,
                                    double wpos, double (&H)[2 * P][2 * P]) {
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
  if (wpos != 0.0) {
#pragma unroll
    for (int s = 0; s < M; ++s)
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int k = 0; k < N; ++k) H[j][k] += rho * wpos * cpos(s, j) * cpos(s, k);
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

// Symmetric 3 x 3 eigen-decomposition A = V diag(w) V^T by cyclic Jacobi rotations (a fixed
// number of sweeps; each zeroes one off-diagonal entry, convergence is quadratic).  A is destroyed.
__device__ inline void sym3_eig(double (&A)[3][3], double (&V)[3][3], double (&w)[3]) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 10; ++sweep) {
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = A[p][q];
      if (fabs(apq) <= 1e-300) continue;
      const double theta = (A[q][q] - A[p][p]) / (2.0 * apq);
      const double t = fabs(theta) > 1e150 ? 0.5 / theta
                                           : (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
      for (int k = 0; k < 3; ++k) {  // A <- A J (columns p, q)
        const double akp = A[k][p], akq = A[k][q];
        A[k][p] = c * akp - s * akq;
        A[k][q] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {  // A <- J^T A (rows p, q)
        const double apk = A[p][k], aqk = A[q][k];
        A[p][k] = c * apk - s * aqk;
        A[q][k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {  // V <- V J
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  for (int i = 0; i < 3; ++i) w[i] = A[i][i];
}

}  // namespace top
