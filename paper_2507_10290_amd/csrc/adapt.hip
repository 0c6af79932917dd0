// Stopping test and adaptive penalty between sweeps (Sec. III-D.3, eqs.
// splitting_tolerance and UpdateRho).
//
// A check follows a sweep launch whose last sweep wrote c~ and the old knots;
// the finalize/reduce kernels have turned them into per-trajectory residual
// norms.  check_kernel then decides per trajectory (float64): stop, or update
// rho.  rescale_kernel applies a change of rho to the folded state and to the
// per-segment solve matrix:
//   * scaled consensus duals: u <- r u with r = rho_old / rho_new;
//   * corridor pairs (box rows or polytope faces): y stands for the slack max(0, -y) and the scaled dual max(0, y),
//     so only a positive y is scaled;
//   * velocity: g stands for the split value Proj(g) and the scaled dual
//     g - Proj(g), so g <- Proj(g) + r (g - Proj(g));
//   * rho * Htilde^-1 (for a polytope, one per rotated axis) is rebuilt in float64 at the new rho.
#include "common.h"
#include "htilde.h"
#include "sweep_impl.h"

namespace top {

__global__ void check_kernel(CheckArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= a.B) return;
  double ratio = 1.0;
  a.fresh[b] = 0;
  if (a.done[b] == 0) {
    a.swept[b] += a.check_every;
    const double rp = a.res[a.B + b], rd = a.res[2 * a.B + b];
    const double t = (double)(a.off[b + 1] - a.off[b]) * a.tol;
    if (a.tol > 0.0 && rp * rp < t * t && rd * rd < t * t) {
      a.done[b] = 1;
      a.stop_at[b] = a.swept[b];
      a.fresh[b] = 1;
      a.lists[atomicAdd(&a.counts[0], 1)] = b;   // list order is irrelevant: entries are independent
    } else if (a.adapt) {
      const double old = a.rho[b];
      double nw = old;
      if (rp > a.mu * rd) nw = old * a.tau_incr;
      else if (rd > a.mu * rp) nw = old / a.tau_decr;
      if (nw != old) {
        ratio = old / nw;
        a.rho[b] = nw;
        a.lists[a.B + atomicAdd(&a.counts[1], 1)] = b;
      }
    }
    if (a.done[b] == 0) a.lists[2 * a.B + atomicAdd(&a.counts[2], 1)] = b;
  }
  a.ratio[b] = ratio;
}

hipError_t launch_check(const CheckArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(check_kernel, dim3((a.B + 255) / 256), dim3(256), 0, st, a);
  return hipGetLastError();
}

__global__ void reset_counts_kernel(int32_t* counts) {
  if (threadIdx.x < 3) counts[threadIdx.x] = 0;
}

__global__ void all_running_kernel(int32_t* lists, int32_t* counts, int B) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) lists[2 * B + b] = b;
  if (b == 0) counts[2] = B;
}

hipError_t launch_all_running(int32_t* lists, int32_t* counts, int B, hipStream_t st) {
  hipLaunchKernelGGL(all_running_kernel, dim3((B + 255) / 256), dim3(256), 0, st, lists, counts, B);
  return hipGetLastError();
}

hipError_t launch_reset_counts(int32_t* counts, hipStream_t st) {
  hipLaunchKernelGGL(reset_counts_kernel, dim3(1), dim3(64), 0, st, counts);
  return hipGetLastError();
}

// Workgroups walk the list of a check (x, grid-stride) and a trajectory's segments in chunks of the
// workgroup size (y); with an empty list every workgroup leaves at once.
constexpr int kListBlocks = 256;

// Over the trajectories that stopped at this check; a lane copies a segment's state column, issuing
// the loads of a batch of rows before their stores, so it waits for memory once per batch rather
// than once per row.
template <typename R>
__global__ void __launch_bounds__(256) freeze_copy_kernel(const R* cur, R* other, const int32_t* list,
                                                          const int32_t* count, const int64_t* off, int nf,
                                                          int64_t ld) {
  constexpr int kBatch = 16;
  const int n = *count;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int b = list[q];
    const int64_t i = off[b] + (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (i >= off[b + 1]) continue;
    for (int f0 = 0; f0 < nf; f0 += kBatch) {
      R v[kBatch];
#pragma unroll
      for (int k = 0; k < kBatch; ++k)
        if (f0 + k < nf) v[k] = cur[(int64_t)(f0 + k) * ld + i];
#pragma unroll
      for (int k = 0; k < kBatch; ++k)
        if (f0 + k < nf) other[(int64_t)(f0 + k) * ld + i] = v[k];
    }
  }
}

hipError_t launch_freeze_copy(const void* cur, void* other, const int32_t* list, const int32_t* count,
                              const int64_t* off, int B, int64_t max_len, int nf, int64_t ld, size_t rsz,
                              hipStream_t st) {
  const dim3 grid((unsigned)std::min(B, kListBlocks), (unsigned)((max_len + 255) / 256)), block(256);
  if (rsz == sizeof(float))
    hipLaunchKernelGGL(freeze_copy_kernel<float>, grid, block, 0, st, (const float*)cur, (float*)other, list, count,
                       off, nf, ld);
  else
    hipLaunchKernelGGL(freeze_copy_kernel<double>, grid, block, 0, st, (const double*)cur, (double*)other, list,
                       count, off, nf, ld);
  return hipGetLastError();
}

// The rescaling of one segment of a trajectory whose rho changed by r = rho_old / rho_new.
template <typename R, int P, int S, bool BOX, bool VEL, int KF>
__device__ void rescale_segment(const RescaleArgs<R>& a, int64_t i, int b, double r) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  constexpr int F_UL = 3 * S, F_YH = 9 * S;
  constexpr int NY = BOX ? 6 * M : KF * M;   // corridor pairs
  constexpr int F_G = 9 * S + NY;
  const int64_t ld = a.ld;
  R* st = a.state;
  const R rr = (R)r;
  for (int f = F_UL; f < F_UL + 6 * S; ++f) st[f * ld + i] *= rr;
  if (NY > 0) {
    for (int f = F_YH; f < F_YH + NY; ++f) {
      const R y = st[f * ld + i];
      if (y > R(0)) st[f * ld + i] = rr * y;
    }
  }
  if (VEL) {
    const R vm = a.vmax[i];
    for (int s = 0; s < M; ++s) {
      R g[3];
      for (int c = 0; c < 3; ++c) g[c] = st[(F_G + c * M + s) * ld + i];
      const R n2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
      const R f = fmin(R(1), vm * inv_sqrt<R>(n2));
      for (int c = 0; c < 3; ++c) {
        const R pr = f * g[c];
        st[(F_G + c * M + s) * ld + i] = pr + rr * (g[c] - pr);
      }
    }
  }
  // rho * Htilde^-1 at the new rho
  const double rho = a.rho[b];
  a.rho_seg[i] = rho;
  const uint8_t fl = a.flags[i];
  const double iT = 1.0 / a.T[i];
  double iTp[2 * N];
  iTp[0] = 1.0;
  for (int o = 1; o < 2 * N; ++o) iTp[o] = iTp[o - 1] * iT;
  double H[N][N], Hi[N][N];
  constexpr int NH = N * (N + 1) / 2;
  for (int ax = 0; ax < (KF > 0 ? 3 : 1); ++ax) {
    const double wpos = KF > 0 ? a.lam[ax * ld + i] : (BOX ? 2.0 : 0.0);
    build_htilde<P, S, VEL>(iTp, iT, rho, (fl & kFirst) != 0, (fl & kLast) != 0, wpos, H);
    spd_inverse<N>(H, Hi);
    for (int rw = 0; rw < N; ++rw)
      for (int c = rw; c < N; ++c) a.Hr[(int64_t)(ax * NH + tri(N, rw, c)) * ld + i] = (R)(rho * Hi[rw][c]);
  }
}

// KF = kFaces: polytope corridor (one y per face and sample, one matrix per rotated axis).  Over the
// trajectories whose rho changed at this check (y = chunk of 128 of a trajectory's segments).
template <typename R, int P, int S, bool BOX, bool VEL, int KF = 0>
__global__ void __launch_bounds__(128) rescale_kernel(RescaleArgs<R> a) {
  const int n = *a.count;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int b = a.list[q];
    const int64_t i = a.off[b] + (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (i < a.off[b + 1]) rescale_segment<R, P, S, BOX, VEL, KF>(a, i, b, a.ratio[b]);
  }
}

template <typename R>
hipError_t launch_rescale(const Variant& v, const RescaleArgs<R>& a, hipStream_t st) {
  const int bs = 128;
  const dim3 grid((unsigned)std::min(a.B, kListBlocks), (unsigned)((a.max_len + bs - 1) / bs)), block(bs);
  if (v.faces != 0) {
    if (v.faces != kFaces || v.box || a.lam == nullptr) return hipErrorInvalidValue;
#define TOP_RESCALE_POLY(P_, S_, V_)                                                        \
    if (v.p == P_ && v.s == S_ && (v.vel != 0) == V_) {                                     \
      hipLaunchKernelGGL((rescale_kernel<R, P_, S_, false, V_, kFaces>), grid, block, 0, st, a); \
      return hipGetLastError();                                                             \
    }
    TOP_RESCALE_POLY(3, 3, true) TOP_RESCALE_POLY(3, 3, false)
    TOP_RESCALE_POLY(3, 4, true) TOP_RESCALE_POLY(3, 4, false)
    TOP_RESCALE_POLY(4, 4, true) TOP_RESCALE_POLY(4, 4, false)
    TOP_RESCALE_POLY(4, 5, true) TOP_RESCALE_POLY(4, 5, false)
    TOP_RESCALE_POLY(3, 5, true) TOP_RESCALE_POLY(3, 5, false)
    TOP_RESCALE_POLY(4, 7, true) TOP_RESCALE_POLY(4, 7, false)
#undef TOP_RESCALE_POLY
    return hipErrorInvalidValue;
  }
#define TOP_RESCALE_CASE(P_, S_, B_, V_)                                                  \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {             \
    hipLaunchKernelGGL((rescale_kernel<R, P_, S_, B_, V_>), grid, block, 0, st, a);      \
    return hipGetLastError();                                                           \
  }
#define TOP_RESCALE_PS(P_, S_)                                                            \
  TOP_RESCALE_CASE(P_, S_, true, true)                                                    \
  TOP_RESCALE_CASE(P_, S_, true, false)                                                   \
  TOP_RESCALE_CASE(P_, S_, false, true)                                                   \
  TOP_RESCALE_CASE(P_, S_, false, false)
  TOP_RESCALE_PS(3, 3)
  TOP_RESCALE_PS(3, 4)
  TOP_RESCALE_PS(4, 4)
  TOP_RESCALE_PS(4, 5)
  TOP_RESCALE_PS(3, 5)
  TOP_RESCALE_PS(4, 7)
#undef TOP_RESCALE_PS
#undef TOP_RESCALE_CASE
  return hipErrorInvalidValue;
}

template hipError_t launch_rescale<float>(const Variant&, const RescaleArgs<float>&, hipStream_t);
template hipError_t launch_rescale<double>(const Variant&, const RescaleArgs<double>&, hipStream_t);

__global__ void conv_report_kernel(const uint8_t* done, const int32_t* stop_at, const double* rho, int B,
                                   int32_t iters_done, int32_t* iters_out, double* rho_out, uint8_t* done_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const bool d = done != nullptr && done[b] != 0;
  if (iters_out != nullptr) iters_out[b] = d ? stop_at[b] : iters_done;
  if (rho_out != nullptr) rho_out[b] = rho[b];
  if (done_out != nullptr) done_out[b] = d ? 1 : 0;
}

hipError_t launch_conv_report(const uint8_t* done, const int32_t* stop_at, const double* rho, int B,
                              int32_t iters_done, int32_t* iters_out, double* rho_out, uint8_t* done_out,
                              hipStream_t st) {
  hipLaunchKernelGGL(conv_report_kernel, dim3((B + 255) / 256), dim3(256), 0, st, done, stop_at, rho, B,
                     iters_done, iters_out, rho_out, done_out);
  return hipGetLastError();
}

}  // namespace top
