// Last stage of the reverse pass: from the adjoint of the Init state and the
// accumulated parameter adjoints to float64 derivatives of the cost with
// respect to the waypoints and the durations (Init of Algorithm 1, as read in
// setup.hip: chord step polynomial, y = min(0, A^o c - b), g = Proj(A^v c)).
#include "common.h"

namespace top {

template <typename R>
__global__ void fill_kernel(R* p, int64_t n, R v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

template <typename R>
hipError_t launch_fill(R* p, int64_t n, R v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel<R>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
  return hipGetLastError();
}
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);

template <typename R, int P, int S, bool BOX, bool VEL>
__global__ void __launch_bounds__(128) init_adjoint_kernel(InitAdjArgs<R> a) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  constexpr int F_ZR = 0, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_G = 9 * S + (BOX ? 6 * M : 0);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.S) return;
  const int64_t ld = a.ld;
  const int b = a.traj[i];
  const uint8_t fl = a.flags[i];
  const bool first = fl & kFirst, last = fl & kLast;
  const double T = a.durations[i];
  const double iT = 1.0 / T;
  const int64_t w0 = i + b, w1 = i + b + 1;
  double ct[3][N], lc[3][N];
  for (int c = 0; c < 3; ++c) {
    const double p0 = a.waypoints[w0 * 3 + c], p1 = a.waypoints[w1 * 3 + c];
    for (int j = 0; j < N; ++j) { ct[c][j] = (p1 - p0) * cstep(P, j); lc[c][j] = 0.0; }
    ct[c][0] += p0;
  }
  double aiT = 0.0;
  if (BOX) {
    for (int c = 0; c < 3; ++c) {
      const double lo = a.box_lo[i * 3 + c], hi = a.box_hi[i * 3 + c];
      for (int s = 0; s < M; ++s) {
        double pv = 0.0;
        for (int j = 0; j < N; ++j) pv += cpos(s, j) * ct[c][j];
        double w = 0.0;
        if (pv - hi < 0.0) w += (double)a.lam[(int64_t)(F_YH + c * M + s) * ld + i];
        if (lo - pv < 0.0) w -= (double)a.lam[(int64_t)(F_YL + c * M + s) * ld + i];
        for (int j = 0; j < N; ++j) lc[c][j] += w * cpos(s, j);
      }
    }
  }
  if (VEL) {
    const double vmax = a.vmax[b];
    for (int s = 0; s < M; ++s) {
      double dv[3], v[3], lg[3];
      for (int c = 0; c < 3; ++c) {
        double acc = 0.0;
        for (int j = 1; j < N; ++j) acc += cvel(s, j) * ct[c][j];
        dv[c] = acc;
        v[c] = acc * iT;
        lg[c] = (double)a.lam[(int64_t)(F_G + c * M + s) * ld + i];
      }
      const double n2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
      const double q = vmax / sqrt(n2);
      double lv[3];
      if (q < 1.0) {  // outside the ball: Proj = (vmax/|v|) v, Jacobian (vmax/|v|)(I - v v^T/|v|^2)
        const double vl = (v[0] * lg[0] + v[1] * lg[1] + v[2] * lg[2]) / n2;
        for (int c = 0; c < 3; ++c) lv[c] = q * (lg[c] - v[c] * vl);
      } else {
        for (int c = 0; c < 3; ++c) lv[c] = lg[c];
      }
      for (int c = 0; c < 3; ++c) {
        for (int j = 1; j < N; ++j) lc[c][j] += iT * lv[c] * cvel(s, j);
        aiT += lv[c] * dv[c];
      }
    }
  }
  for (int c = 0; c < 3; ++c) {
    double right = 0.0;
    for (int j = 0; j < N; ++j) right += cstep(P, j) * lc[c][j];
    a.dPL[i * 3 + c] = lc[c][0] - right;
    a.dPR[i * 3 + c] = right;
    // the end knot's position is the next waypoint (interior knots, and the trajectory end when its
    // end state is the rest state at that waypoint)
    const bool knot_is_wp = !last || a.bc == nullptr;
    a.dK[i * 3 + c] = knot_is_wp ? (double)a.lam[(int64_t)(F_ZR + c * S) * ld + i] : 0.0;
    a.dK0[i * 3 + c] = (first && a.bc == nullptr) ? (double)a.acc_z0[(int64_t)(c * S) * ld + i] : 0.0;
  }
  if (a.dT != nullptr) a.dT[i] = (double)a.acc_hd[i] + ((double)a.acc_iT[i] + aiT) * (-iT * iT);
}

template <typename R>
hipError_t launch_init_adjoint(const Variant& v, const InitAdjArgs<R>& a, hipStream_t st) {
  const dim3 grid((unsigned)((a.S + 127) / 128)), block(128);
#define TOP_IA_CASE(P_, S_, B_, V_)                                                          \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {               \
    hipLaunchKernelGGL((init_adjoint_kernel<R, P_, S_, B_, V_>), grid, block, 0, st, a);   \
    return hipGetLastError();                                                             \
  }
#define TOP_IA_PS(P_, S_)                                                                    \
  TOP_IA_CASE(P_, S_, true, true)                                                            \
  TOP_IA_CASE(P_, S_, true, false)                                                           \
  TOP_IA_CASE(P_, S_, false, true)                                                           \
  TOP_IA_CASE(P_, S_, false, false)
  TOP_IA_PS(3, 3)
  TOP_IA_PS(3, 4)
  TOP_IA_PS(4, 4)
  TOP_IA_PS(4, 5)
#undef TOP_IA_PS
#undef TOP_IA_CASE
  return hipErrorInvalidValue;
}
template hipError_t launch_init_adjoint<float>(const Variant&, const InitAdjArgs<float>&, hipStream_t);
template hipError_t launch_init_adjoint<double>(const Variant&, const InitAdjArgs<double>&, hipStream_t);

// Each waypoint gathers the contributions of the (up to) two segments that meet there, in a fixed
// order: the segment ending there (its chord end and its end knot), then the one starting there.
__global__ void gather_waypoints_kernel(const double* dPL, const double* dPR, const double* dK,
                                        const double* dK0, const int64_t* off, int B, int64_t rows,
                                        double* dP) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  int lo = 0, hi = B;  // last b with off[b] + b <= r
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (off[mid] + mid <= r) lo = mid; else hi = mid;
  }
  const int b = lo;
  const int64_t q = r - off[b] - b;
  const int64_t n = off[b + 1] - off[b];
  for (int c = 0; c < 3; ++c) {
    double v = 0.0;
    if (q >= 1) {
      const int64_t s = off[b] + q - 1;
      v += dPR[s * 3 + c] + dK[s * 3 + c];
    }
    if (q < n) v += dPL[(off[b] + q) * 3 + c];
    if (q == 0) v += dK0[off[b] * 3 + c];
    dP[r * 3 + c] = v;
  }
}

hipError_t launch_gather_waypoints(const double* dPL, const double* dPR, const double* dK, const double* dK0,
                                   const int64_t* off, int B, int64_t rows, double* dP, hipStream_t st) {
  hipLaunchKernelGGL(gather_waypoints_kernel, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, st, dPL, dPR,
                     dK, dK0, off, B, rows, dP);
  return hipGetLastError();
}

}  // namespace top
