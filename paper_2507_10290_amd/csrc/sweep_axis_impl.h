// The sweep with one lane per segment and axis: the form for trajectories longer than a tile.
//
// A trajectory longer than a tile is cut into tiles whose core segments are flanked by `halo`
// copies, and a launch runs at most `halo` sweeps.  With one lane per segment such a launch holds
// one wave per 64 segments, too few to keep every SIMD busy once the halo copies are added (a
// 65,536-segment trajectory fills half the wave slots of the chip, unevenly).  Here a tile of W
// segments runs as 3 W lanes, axis-major (thread a W + l holds axis a of segment l), so each wave
// belongs to one axis: three times the waves, each carrying one third of the per-axis work, with a
// third of the registers.  The arithmetic of every axis is the one-lane form's (axis_update,
// knot_update and vel_factors of sweep_impl.h, in the same order), so both forms give the same bits.
//
// The axes meet only in the velocity projection factor f = min(1, vmax / ||g||) of each sample,
// which needs the split values g of all three axes: every lane puts its updated g into LDS next to
// its knot end states, and after the sweep's one barrier it reads the other two axes' values for the
// next sweep's factors.  Each segment's rho Htilde^-1 is read from LDS by its three lanes.  This form
// has no recording instance and no stopped-trajectory handling (no tape, no residual checks).
#pragma once

#include "sweep_impl.h"

namespace top {

// Largest tile (segments) of the lane-per-axis sweep (axis_max_tile in common.h): 3 W lanes must fit
// one workgroup.
constexpr int kAxisMaxTile = kAxisTileMax;
constexpr int kAxisMaxWaves = kAxisMaxTile / 64;   // waves of one axis

template <typename R, int P, int S, bool BOX, bool VEL>
struct AxisLane {
  static constexpr int N = 2 * P;
  static constexpr int M = kSamples;
  static constexpr int MB = BOX ? M : 1;
  static constexpr int MV = VEL ? M : 1;
  R zL[S], zR[S], uL[S], uR[S], yh[MB], yl[MB], g[MV];
  R iT, iTp[S], lo, hi, vm;
  bool first, last, has_left, has_right, fixpos;
};

// Dynamic LDS: the tile's rho Htilde^-1 [NH][TS], then the split values of the three axes, double
// buffered by sweep parity [2][3][MV][TS], with the row stride TS the instance's largest tile (a
// compile-time stride turns every LDS address into a constant offset from the lane's own).
inline size_t sweep_axis_lds_bytes(int p, bool vel, size_t rsz, int TS) {
  const int n = 2 * p, nh = n * (n + 1) / 2;
  return (size_t)(nh + 2 * 3 * (vel ? kSamples : 1)) * rsz * (size_t)TS;
}

template <typename R, int P, int S, bool BOX, bool VEL, int LB>
__global__ __launch_bounds__(LB) void sweep_axis_kernel(SweepArgs<R> A) {
  using LT = AxisLane<R, P, S, BOX, VEL>;
  constexpr int N = LT::N;
  constexpr int NH = N * (N + 1) / 2;
  constexpr int M = LT::M;
  constexpr int MV = LT::MV;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_G = 9 * S + (BOX ? 6 * M : 0);
  constexpr int TS = LB / 3;   // LDS row stride: the largest tile

  __shared__ R xr_sh[2][3][kAxisMaxWaves][S];   // end states to the right neighbour (wave edges)
  __shared__ R xl_sh[2][3][kAxisMaxWaves][S];   // start states to the left neighbour
  extern __shared__ double axis_lds_raw[];
  R* sh_H = reinterpret_cast<R*>(axis_lds_raw) + threadIdx.x % A.W;   // this lane's column
  R* sh_g = sh_H + NH * TS;

  const int W = A.W;
  const int a = threadIdx.x / W;          // axis of this lane
  const int lane = threadIdx.x - a * W;   // segment lane within the tile
  const int64_t base = (int64_t)blockIdx.x * W;
  const int64_t ld = A.k.ld;
  const int32_t ent = A.lane_seg[base + lane];
  const bool active = ent >= 0;
  const bool core = active && !(ent & kHaloBit);
  const int64_t seg = active ? (int64_t)(ent & kSegMask) : 0;
  const uint8_t fl = active ? A.k.flags[seg] : (uint8_t)(kFirst | kLast);
  const int wl = lane & 63, wid = lane >> 6, nw = W >> 6;
  auto G = [&](int buf, int ax, int s) -> R& { return sh_g[((buf * 3 + ax) * MV + s) * TS]; };

  // the tile's matrices into LDS (the three lanes of a segment share the loads)
  for (int h = a; h < NH; h += 3) sh_H[h * TS] = active ? A.k.Hr[h * ld + seg] : R(0);
  if (__ballot(active) == 0) {            // a wave without segments keeps the barrier count
    __syncthreads();
    for (int it = 0; it < A.iters; ++it) __syncthreads();
    return;
  }

  LT L;
  L.first = fl & kFirst;
  L.last = fl & kLast;
  L.has_left = false;
  L.has_right = false;
  if (active && !L.first && lane > 0) {
    const int32_t e = A.lane_seg[base + lane - 1];
    L.has_left = e >= 0 && (int64_t)(e & kSegMask) == seg - 1;
  }
  if (active && !L.last && lane < W - 1) {
    const int32_t e = A.lane_seg[base + lane + 1];
    L.has_right = e >= 0 && (int64_t)(e & kSegMask) == seg + 1;
  }
  L.fixpos = A.fixpos != 0;
  const int tr = active ? A.k.traj[seg] : 0;
  L.iT = active ? A.k.iT[seg] : R(1);
  L.vm = (VEL && active) ? A.k.vmax[seg] : R(1);
  L.lo = (BOX && active) ? A.k.lo[a * ld + seg] : R(0);
  L.hi = (BOX && active) ? A.k.hi[a * ld + seg] : R(0);
  L.iTp[0] = R(1);
#pragma unroll
  for (int o = 1; o < S; ++o) L.iTp[o] = L.iTp[o - 1] * L.iT;

  // ---- state of this axis, and the split values of all three for the first sweep's factors
  const R* in = A.st_in;
#pragma unroll
  for (int o = 0; o < S; ++o) {
    const int f = a * S + o;
    L.zR[o] = active ? in[(F_ZR + f) * ld + seg] : R(0);
    L.uL[o] = active ? in[(F_UL + f) * ld + seg] : R(0);
    L.uR[o] = active ? in[(F_UR + f) * ld + seg] : R(0);
    L.zL[o] = !active ? R(0)
            : L.first ? A.k.bcL[((int64_t)tr * 3 + a) * S + o]
                      : in[(F_ZR + f) * ld + seg - 1];
  }
#pragma unroll
  for (int s = 0; s < LT::MB; ++s) {
    L.yh[s] = (BOX && active) ? in[(F_YH + a * M + s) * ld + seg] : R(0);
    L.yl[s] = (BOX && active) ? in[(F_YL + a * M + s) * ld + seg] : R(0);
  }
  R gall[3][MV];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int s = 0; s < MV; ++s) gall[b][s] = (VEL && active) ? in[(F_G + b * M + s) * ld + seg] : R(0);
#pragma unroll
  for (int s = 0; s < MV; ++s) L.g[s] = a == 0 ? gall[0][s] : (a == 1 ? gall[1][s] : gall[2][s]);
  __syncthreads();   // the matrices are in LDS

  const auto H = [&](int h) { return sh_H[h * TS]; };
  R cfin[N], zfin[S];
  int buf = 0;
  // One sweep; with FIN (the launch's last sweep when it writes outputs) the local solve and the end
  // knot before its update are kept in cfin / zfin.
  auto sweep = [&](auto fin_tag) {
    constexpr bool FIN = decltype(fin_tag)::value;
    R q[MV], om[MV];
#pragma unroll
    for (int s = 0; s < MV; ++s) {
      if constexpr (VEL) {
        vel_factors(gall[0][s], gall[1][s], gall[2][s], L.vm, L.iT, q[s], om[s]);
      } else {
        q[s] = R(0);
        om[s] = R(0);
      }
    }
    R xL[S], xR[S];
    axis_update<FIN, R, P, S, BOX, VEL>(H, L.iT, L.iTp, L.lo, L.hi, q, om, L.zL, L.zR, L.uL, L.uR, L.yh, L.yl, L.g,
                                        xL, xR, cfin);
    // ---- exchange: knot end states at wave edges, this axis' split values for the other two lanes
    if (wl == 63) {
#pragma unroll
      for (int o = 0; o < S; ++o) xr_sh[buf][a][wid][o] = xR[o];
    }
    if (wl == 0) {
#pragma unroll
      for (int o = 0; o < S; ++o) xl_sh[buf][a][wid][o] = xL[o];
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) G(buf, a, s) = L.g[s];
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R xp = __shfl_up(xR[o], 1);
      R xn = __shfl_down(xL[o], 1);
      if (wl == 0 && wid > 0) xp = xr_sh[buf][a][wid - 1][o];
      if (wl == 63 && wid < nw - 1) xn = xl_sh[buf][a][wid + 1][o];
      knot_update<FIN, P>(o, xL[o], xR[o], xp, xn, L.has_left, L.has_right, L.first, L.last, L.fixpos, L.zL[o],
                          L.zR[o], L.uL[o], L.uR[o], zfin[o]);
    }
    if constexpr (VEL) {
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int s = 0; s < M; ++s) gall[b][s] = G(buf, b, s);
    }
    buf ^= 1;
  };
  const int n_plain = A.final_out ? A.iters - 1 : A.iters;
  for (int it = 0; it < n_plain; ++it) sweep(std::false_type{});
  if (A.final_out && A.iters > 0) sweep(std::true_type{});

  if (core) {
    if (A.final_out && A.iters > 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) A.c_out[(a * N + j) * ld + seg] = cfin[j];
#pragma unroll
      for (int o = 0; o < S; ++o) A.zold_out[(a * S + o) * ld + seg] = zfin[o];
    }
    R* out = A.st_out;
#pragma unroll
    for (int o = 0; o < S; ++o) {
      const int f = a * S + o;
      out[(F_ZR + f) * ld + seg] = L.zR[o];
      out[(F_UL + f) * ld + seg] = L.uL[o];
      out[(F_UR + f) * ld + seg] = L.uR[o];
    }
    if constexpr (BOX) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        out[(F_YH + a * M + s) * ld + seg] = L.yh[s];
        out[(F_YL + a * M + s) * ld + seg] = L.yl[s];
      }
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) out[(F_G + a * M + s) * ld + seg] = L.g[s];
    }
  }
}

// Launch over tiles of W <= LBT segments (3 W threads each); closed form, s in {p, p+1}, no
// recording and no stopped trajectories.
template <typename R, int LBT>
hipError_t dispatch_sweep_axis(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  if (v.num || v.faces || v.s == 2 * v.p - 1 || a.rec != nullptr || a.done != nullptr) return hipErrorInvalidValue;
  if (a.W <= 0 || a.W > LBT || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(3 * a.W);
  const size_t lds = sweep_axis_lds_bytes(v.p, v.vel != 0, sizeof(R), LBT);
#define TOP_AXIS_CASE(P_, S_, B_, V_)                                                             \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {                      \
    auto k_ = sweep_axis_kernel<R, P_, S_, B_, V_, 3 * LBT>;                                     \
    hipError_t e_ = hipFuncSetAttribute((const void*)k_, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e_ != hipSuccess) return e_;                                                             \
    hipLaunchKernelGGL(k_, grid, block, lds, st, a);                                             \
    return hipGetLastError();                                                                    \
  }
#define TOP_AXIS_PS(P_, S_)                                                                        \
  TOP_AXIS_CASE(P_, S_, true, true)                                                                \
  TOP_AXIS_CASE(P_, S_, true, false)                                                               \
  TOP_AXIS_CASE(P_, S_, false, true)                                                               \
  TOP_AXIS_CASE(P_, S_, false, false)
  TOP_AXIS_PS(3, 3)
  TOP_AXIS_PS(3, 4)
  TOP_AXIS_PS(4, 4)
  TOP_AXIS_PS(4, 5)
#undef TOP_AXIS_PS
#undef TOP_AXIS_CASE
  return hipErrorInvalidValue;
}

}  // namespace top
