// One-time per-segment work: input validation, the float64 precompute of
// rho * Htilde^-1 (the inverse in eq. QpSubProblem, in the normalised-time
// basis), and Init of Algorithm 1.
//
// Init (the paper only says that Init sets up every variable): each segment
// starts on its chord as the rest-to-rest step polynomial of degree 2p-1;
// interior knots hold the waypoint position with zero higher derivatives; the
// end knots hold the trajectory's end states; all scaled duals are zero; the
// box slack starts at max(0, b - A^o c^0) with a zero dual, stored as
// y = min(0, A^o c^0 - b); the velocity split starts at Proj(A^v c^0) with a
// zero dual, stored as g = Proj(A^v c^0).
#include "common.h"
#include "htilde.h"

namespace top {

// Every input array is checked as a flat array, one element per lane and grid-stride, so the loads
// are coalesced whatever the array's row length (a polytope row is 4 * n_faces doubles).
__global__ void __launch_bounds__(256) validate_kernel(SetupArgs a, int p, int* bad) {
  const int64_t n_box = 3 * a.S, n_faces = a.faces != nullptr ? (int64_t)4 * a.n_faces * a.S : 0;
  const int64_t n_wp = 3 * (a.S + a.B), n_bc = a.bc != nullptr ? (int64_t)6 * p * a.B : 0;
  int64_t n = a.S > n_box ? a.S : n_box;
  n = n > n_faces ? n : n_faces;
  n = n > n_wp ? n : n_wp;
  n = n > n_bc ? n : n_bc;
  int flag = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < a.S) {
      const double T = a.durations[i];
      if (!(T > 0.0) || !isfinite(T)) flag |= 1;
    }
    if (a.box_lo != nullptr && i < n_box) {
      const double lo = a.box_lo[i], hi = a.box_hi[i];
      if (!isfinite(lo) || !isfinite(hi) || !(lo < hi)) flag |= 2;
    }
    if (i < n_faces && !isfinite(a.faces[i])) flag |= 64;
    if (i < n_wp && !isfinite(a.waypoints[i])) flag |= 4;
    if (i < a.B) {
      const double r = a.rho[i];
      if (!(r > 0.0) || !isfinite(r)) flag |= 8;
      if (a.vmax != nullptr) {
        const double v = a.vmax[i];
        if (!(v > 0.0) || !isfinite(v)) flag |= 16;
      }
    }
    if (i < n_bc && !isfinite(a.bc[i])) flag |= 32;
  }
  if (flag) atomicOr(bad, flag);
}

hipError_t launch_validate(const SetupArgs& a, int p, int* bad, hipStream_t st) {
  const int64_t n = 4 * (int64_t)(a.faces != nullptr ? a.n_faces : 1) * a.S + 3 * (int64_t)a.B;
  const int bs = 256;
  int64_t nb = (n + bs - 1) / bs;
  if (nb > 4096) nb = 4096;  // grid-stride beyond 4096 workgroups
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)nb), dim3(bs), 0, st, a, p, bad);
  return hipGetLastError();
}

// End state (order o, axis c) of trajectory b at its start (side 0) or end (side 1).
__device__ inline double end_state(const SetupArgs& a, int P, int b, int side, int o, int c, int64_t wp_row) {
  if (a.bc != nullptr) return a.bc[(((int64_t)b * 2 + side) * P + o) * 3 + c];
  return o == 0 ? a.waypoints[wp_row * 3 + c] : 0.0;
}

// KF = kFaces: general polytope corridor (BOX is then false).  NUM: NumericSolve state (velocity
// multipliers w = 0 and the Init c~ kept as the first L-BFGS start) instead of the velocity split g.
template <typename R, int P, int S, bool BOX, bool VEL, int KF = 0, bool NUM = false>
__global__ void __launch_bounds__(128) setup_kernel(SetupArgs a, SetupOut<R> out) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_G = 9 * S + (BOX ? 6 * M : KF * M);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t ld = out.ld;
  if (i >= a.S) {
    // padding columns S..ld-1: owned by no lane; zeroed so that exported states are deterministic
    if (i < ld)
      for (int f = 0; f < out.nf; ++f) {
        out.state[(int64_t)f * ld + i] = R(0);
        if (out.state1 != nullptr) out.state1[(int64_t)f * ld + i] = R(0);
      }
    return;
  }

  // trajectory of segment i: last b with seg_off[b] <= i
  int lo_b = 0, hi_b = a.B;  // invariant seg_off[lo_b] <= i < seg_off[hi_b]
  while (hi_b - lo_b > 1) {
    const int mid = (lo_b + hi_b) / 2;
    if (a.seg_off[mid] <= i) lo_b = mid; else hi_b = mid;
  }
  const int b = lo_b;
  const bool first = i == a.seg_off[b];
  const bool last = i == a.seg_off[b + 1] - 1;
  const double T = a.durations[i];
  const double iT = 1.0 / T;
  const double rho = a.rho[b];
  double iTp[2 * N];  // powers of 1/T up to 2N-1 (the T-derivative rows need 2o+1 <= 2s-1)
  iTp[0] = 1.0;
  for (int o = 1; o < 2 * N; ++o) iTp[o] = iTp[o - 1] * iT;

  // ---- Htilde = 2 T^(1-2p) Q(1) + rho [boundary rows + corridor rows + velocity rows], inverted
  double H[N][N], Hi[N][N];
  if constexpr (KF > 0) {
    // faces (padded with a = 0, b = 1, which never bind and add nothing), G = sum_k a_k a_k^T,
    // G = U diag(lam) U^T, and one matrix per rotated axis
    double G[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, Um[3][3], lam[3];
    for (int k = 0; k < KF; ++k) {
      double f[4] = {0.0, 0.0, 0.0, 1.0};
      if (k < a.n_faces)
        for (int q = 0; q < 4; ++q) f[q] = a.faces[(i * a.n_faces + k) * 4 + q];
      for (int q = 0; q < 4; ++q) out.fa[(int64_t)(k * 4 + q) * ld + i] = (R)f[q];
      for (int q = 0; q < 3; ++q)
        for (int r = 0; r < 3; ++r) G[q][r] += f[q] * f[r];
    }
    sym3_eig(G, Um, lam);
    constexpr int NH = N * (N + 1) / 2;
    for (int ax = 0; ax < 3; ++ax) {
      build_htilde<P, S, VEL>(iTp, iT, rho, first, last, lam[ax], H);
      spd_inverse<N>(H, Hi);
      for (int r = 0; r < N; ++r)
        for (int c = r; c < N; ++c) out.Hr[(int64_t)(ax * NH + tri(N, r, c)) * ld + i] = (R)(rho * Hi[r][c]);
      out.lam[ax * ld + i] = lam[ax];
    }
    for (int q = 0; q < 3; ++q)
      for (int ax = 0; ax < 3; ++ax) out.U[(int64_t)(3 * q + ax) * ld + i] = (R)Um[q][ax];
  } else {
    build_htilde<P, S, VEL>(iTp, iT, rho, first, last, BOX ? 2.0 : 0.0, H);
    spd_inverse<N>(H, Hi);
    for (int r = 0; r < N; ++r)
      for (int c = r; c < N; ++c) out.Hr[(int64_t)tri(N, r, c) * ld + i] = (R)(rho * Hi[r][c]);
  }
  const int nL = first ? P : S;
  const int nR = last ? P : S;
  if (KF == 0 && out.Hd != nullptr) {
    // d(rho Htilde^-1)/dT = -rho Htilde^-1 (dHtilde/dT) Htilde^-1, with
    // dHtilde/dT = 2(1-2p) T^-2p Q(1) + rho [ -2o (o!)^2 T^(-2o-1) on left rows,
    //              -2o T^(-2o-1) f_o f_o^T on right rows, -2 T^-3 sum_s tau'_s tau'_s^T ]
    double dH[N][N];
    const double cq = 2.0 * (1.0 - 2.0 * P) * iTp[2 * P - 1] * iT;
    for (int j = 0; j < N; ++j)
      for (int k = 0; k < N; ++k) dH[j][k] = cq * cgram(P, j, k);
    for (int o = 1; o < nL; ++o) dH[o][o] += rho * (-2.0 * o) * cfact(o) * cfact(o) * iTp[2 * o] * iT;
    for (int o = 1; o < nR; ++o)
      for (int j = 0; j < N; ++j)
        for (int k = 0; k < N; ++k) dH[j][k] += rho * (-2.0 * o) * iTp[2 * o] * iT * cfall(o, j) * cfall(o, k);
    if (VEL) {
      for (int s = 0; s < M; ++s)
        for (int j = 0; j < N; ++j)
          for (int k = 0; k < N; ++k) dH[j][k] += rho * (-2.0) * iT * iT * iT * cvel(s, j) * cvel(s, k);
    }
    double tmp[N][N];
    for (int r = 0; r < N; ++r)
      for (int c = 0; c < N; ++c) {
        double v = 0.0;
        for (int k = 0; k < N; ++k) v += dH[r][k] * Hi[k][c];
        tmp[r][c] = v;
      }
    for (int r = 0; r < N; ++r)
      for (int c = r; c < N; ++c) {
        double v = 0.0;
        for (int k = 0; k < N; ++k) v += Hi[r][k] * tmp[k][c];
        out.Hd[(int64_t)tri(N, r, c) * ld + i] = (R)(-rho * v);
      }
  }

  // ---- per-segment constants
  out.iT[i] = (R)iT;
  out.flags[i] = (uint8_t)((first ? kFirst : 0) | (last ? kLast : 0));
  out.traj[i] = b;
  out.Tdev[i] = T;
  out.rho_seg[i] = rho;
  const double vmax = (a.vmax != nullptr) ? a.vmax[b] : 1.0;
  out.vmax[i] = (R)vmax;
  const int64_t w0 = i + b, w1 = i + b + 1;  // waypoint rows of the segment's two ends
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int c = 0; c < 3; ++c) {
    if (BOX) { lo[c] = a.box_lo[i * 3 + c]; hi[c] = a.box_hi[i * 3 + c]; }
    out.lo[c * ld + i] = (R)lo[c];
    out.hi[c * ld + i] = (R)hi[c];
  }

  // ---- Init: chord step polynomial in the normalised basis
  double ct[3][N];
  for (int c = 0; c < 3; ++c) {
    const double p0 = a.waypoints[w0 * 3 + c], p1 = a.waypoints[w1 * 3 + c];
#pragma unroll
    for (int j = 0; j < N; ++j) ct[c][j] = (p1 - p0) * cstep(P, j);
    ct[c][0] += p0;
#pragma unroll
    for (int j = 0; j < N; ++j) out.c[(int64_t)(c * N + j) * ld + i] = (R)ct[c][j];
  }
  R* st = out.state;
  for (int c = 0; c < 3; ++c) {
    for (int o = 0; o < S; ++o) {
      double z;
      if (last) z = (o < P) ? end_state(a, P, b, 1, o, c, w1) : 0.0;
      else z = (o == 0) ? a.waypoints[w1 * 3 + c] : 0.0;
      st[(int64_t)(F_ZR + c * S + o) * ld + i] = (R)z;
      st[(int64_t)(F_UL + c * S + o) * ld + i] = (R)0;
      st[(int64_t)(F_UR + c * S + o) * ld + i] = (R)0;
      if (first) out.bcL[((int64_t)b * 3 + c) * S + o] = (R)((o < P) ? end_state(a, P, b, 0, o, c, w0) : 0.0);
    }
  }
  if (BOX) {
    for (int c = 0; c < 3; ++c) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        double pv = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) pv += cpos(s, j) * ct[c][j];
        st[(int64_t)(F_YH + c * M + s) * ld + i] = (R)fmin(0.0, pv - hi[c]);
        st[(int64_t)(F_YL + c * M + s) * ld + i] = (R)fmin(0.0, lo[c] - pv);
      }
    }
  }
  if constexpr (KF > 0) {
    // y = min(0, a_k . p_s - b_k) at each sample position p_s of the chord polynomial
#pragma unroll
    for (int s = 0; s < M; ++s) {
      double pv[3];
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < N; ++j) acc += cpos(s, j) * ct[c][j];
        pv[c] = acc;
      }
      for (int k = 0; k < KF; ++k) {
        double f[4] = {0.0, 0.0, 0.0, 1.0};
        if (k < a.n_faces)
          for (int q = 0; q < 4; ++q) f[q] = a.faces[(i * a.n_faces + k) * 4 + q];
        st[(int64_t)(F_YH + k * M + s) * ld + i] = (R)fmin(0.0, f[0] * pv[0] + f[1] * pv[1] + f[2] * pv[2] - f[3]);
      }
    }
  }
  if constexpr (NUM) {
    for (int s = 0; s < M; ++s) st[(int64_t)(F_G + s) * ld + i] = (R)0;
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < N; ++j) st[(int64_t)(F_G + M + c * N + j) * ld + i] = (R)ct[c][j];
  } else if (VEL) {
#pragma unroll
    for (int s = 0; s < M; ++s) {
      double v[3];
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int j = 1; j < N; ++j) acc += cvel(s, j) * ct[c][j];
        v[c] = acc * iT;
      }
      const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      const double f = fmin(1.0, vmax / sqrt(n2));
      for (int c = 0; c < 3; ++c) st[(int64_t)(F_G + c * M + s) * ld + i] = (R)(f * v[c]);
    }
  }
}

template <typename R>
hipError_t launch_setup(const Variant& v, const SetupArgs& a, const SetupOut<R>& o, hipStream_t st) {
  const int bs = 128;
  const dim3 grid((unsigned)((o.ld + bs - 1) / bs)), block(bs);  // ld >= S: the padding columns too
  if (v.num != 0) {
    if (!v.vel || v.faces || v.s != v.p) return hipErrorInvalidValue;
#define TOP_SETUP_NUM(P_, B_)                                                             \
    if (v.p == P_ && (v.box != 0) == B_) {                                                \
      hipLaunchKernelGGL((setup_kernel<R, P_, P_, B_, true, 0, true>), grid, block, 0, st, a, o); \
      return hipGetLastError();                                                           \
    }
    TOP_SETUP_NUM(3, true) TOP_SETUP_NUM(3, false) TOP_SETUP_NUM(4, true) TOP_SETUP_NUM(4, false)
#undef TOP_SETUP_NUM
    return hipErrorInvalidValue;
  }
  if (v.faces != 0) {
    if (v.faces != kFaces || v.box) return hipErrorInvalidValue;
#define TOP_SETUP_POLY(P_, S_, V_)                                                        \
    if (v.p == P_ && v.s == S_ && (v.vel != 0) == V_) {                                   \
      hipLaunchKernelGGL((setup_kernel<R, P_, S_, false, V_, kFaces>), grid, block, 0, st, a, o); \
      return hipGetLastError();                                                           \
    }
    TOP_SETUP_POLY(3, 3, true) TOP_SETUP_POLY(3, 3, false)
    TOP_SETUP_POLY(3, 4, true) TOP_SETUP_POLY(3, 4, false)
    TOP_SETUP_POLY(4, 4, true) TOP_SETUP_POLY(4, 4, false)
    TOP_SETUP_POLY(4, 5, true) TOP_SETUP_POLY(4, 5, false)
    TOP_SETUP_POLY(3, 5, true) TOP_SETUP_POLY(3, 5, false)
    TOP_SETUP_POLY(4, 7, true) TOP_SETUP_POLY(4, 7, false)
#undef TOP_SETUP_POLY
    return hipErrorInvalidValue;
  }
#define TOP_SETUP_CASE(P_, S_, B_, V_)                                                   \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {            \
    hipLaunchKernelGGL((setup_kernel<R, P_, S_, B_, V_>), grid, block, 0, st, a, o);    \
    return hipGetLastError();                                                          \
  }
#define TOP_SETUP_PS(P_, S_)                                                             \
  TOP_SETUP_CASE(P_, S_, true, true)                                                     \
  TOP_SETUP_CASE(P_, S_, true, false)                                                    \
  TOP_SETUP_CASE(P_, S_, false, true)                                                    \
  TOP_SETUP_CASE(P_, S_, false, false)
  TOP_SETUP_PS(3, 3)
  TOP_SETUP_PS(3, 4)
  TOP_SETUP_PS(4, 4)
  TOP_SETUP_PS(4, 5)
  TOP_SETUP_PS(3, 5)
  TOP_SETUP_PS(4, 7)
#undef TOP_SETUP_PS
#undef TOP_SETUP_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_setup<float>(const Variant&, const SetupArgs&, const SetupOut<float>&, hipStream_t);
template hipError_t launch_setup<double>(const Variant&, const SetupArgs&, const SetupOut<double>&, hipStream_t);

}  // namespace top
