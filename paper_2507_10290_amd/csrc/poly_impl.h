// Sweep kernel for a general polytope corridor P_i^H = {x : a_k . x <= b_k, k < kFaces} per
// segment (Sec. III-D.1), resident form: same tiles, launch protocol and knot exchange as the box
// kernel of sweep_impl.h.
//
// The corridor rows a_k (x) tau_s couple the three axes.  Their Gram term
// (sum_k a_k a_k^T) (x) (sum_s tau_s tau_s^T) becomes diagonal in the axis index after rotating
// to the eigenvectors U of sum_k a_k a_k^T, and every other term of Htilde is the same for all
// axes, so the local solve splits into one n x n solve per rotated axis (matrices built by setup):
//   r~_a += sum_s tau_s e_{s,a},  e_s = sum_k a_k (b_k - |y_{k,s}|)      [folded slack/dual rows]
//   c~   = U blockdiag_a'(rho Htilde_a'^-1) U^T r~   (U acting on the axis index of each c~_j)
//   y_{k,s} <- a_k . p_s - b_k + max(0, y_{k,s}),  p_s = (tau_s . c~_a)_a
//                                                    [eqs. NonNegativeProject, UpdateV]
// The knot, u and velocity rules are those of the box kernel.
//
// HL: the three rho Htilde_a'^-1 live in the lane's own column of dynamic LDS instead of registers
// (used for the float32 quintic instance, which then fits two waves per SIMD).
#pragma once

#include "sweep_impl.h"

namespace top {

template <typename R, int P, int S, bool VEL>
struct PolyLane {
  static constexpr int N = 2 * P;
  static constexpr int NH = N * (N + 1) / 2;
  static constexpr int M = kSamples;
  static constexpr int MV = VEL ? M : 1;
  static constexpr int KF = kFaces;
  // state
  R zL[3][S], zR[3][S], uL[3][S], uR[3][S], y[KF][M], g[3][MV];
  // constants
  R H[3][NH], U[9], fa[KF][4], iT, iTp[S], vm;
  bool first, last, has_left, has_right, fixpos;
};

// Hs: this lane's LDS column of the matrices (HL), rows TS apart.
template <bool FINAL, bool HL, int TS, typename R, int P, int S, bool VEL>
__device__ __forceinline__ void poly_sweep_once(PolyLane<R, P, S, VEL>& L, const R* Hs,
                                                R (*xr_sh)[3 * S], R (*xl_sh)[3 * S], int wl, int wid, int nw,
                                                R (&cfin)[3][2 * P], R (&zfin)[3][S]) {
  using LT = PolyLane<R, P, S, VEL>;
  constexpr int N = LT::N;
  constexpr int M = LT::M;
  constexpr int MV = LT::MV;
  constexpr int KF = LT::KF;

  R q[MV], om[MV];
#pragma unroll
  for (int s = 0; s < MV; ++s) {
    if constexpr (VEL) {
      const R n2 = L.g[0][s] * L.g[0][s] + L.g[1][s] * L.g[1][s] + L.g[2][s] * L.g[2][s];
      const R f = fmin(R(1), L.vm * inv_sqrt<R>(n2));
      q[s] = (R(2) * f - R(1)) * L.iT;
      om[s] = R(1) - f;
    } else {
      q[s] = R(0);
      om[s] = R(0);
    }
  }

  // ---- r~ of all three axes
  R r[3][N];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int j = 0; j < N; ++j) r[a][j] = R(0);
    static_for<0, S>([&](auto o) {
      const R wl_ = (L.zL[a][o] - L.uL[a][o]) * L.iTp[o];
      constexpr R kf = R(cfact(o));
      r[a][o] += kf * wl_;
      const R wr_ = (L.zR[a][o] - L.uR[a][o]) * L.iTp[o];
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        r[a][j] += k * wr_;
      });
    });
  }
  static_for<0, M>([&](auto s) {
    R e0 = R(0), e1 = R(0), e2 = R(0);
#pragma unroll
    for (int k = 0; k < KF; ++k) {
      const R d = L.fa[k][3] - fabs(L.y[k][s]);
      e0 += L.fa[k][0] * d;
      e1 += L.fa[k][1] * d;
      e2 += L.fa[k][2] * d;
    }
    static_for<0, N>([&](auto j) {
      constexpr R k = R(cpos(s, j));
      r[0][j] += k * e0;
      r[1][j] += k * e1;
      r[2][j] += k * e2;
    });
  });
  if constexpr (VEL) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      static_for<0, M>([&](auto s) {
        const R b = q[s] * L.g[a][s];
        static_for<1, N>([&](auto j) {
          constexpr R k = R(cvel(s, j));
          r[a][j] += k * b;
        });
      });
    }
  }

  // ---- local solve in the rotated frame
  R c[3][N];
  {
    R rr[3][N], cr[3][N];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) rr[ax][j] = L.U[ax] * r[0][j] + L.U[3 + ax] * r[1][j] + L.U[6 + ax] * r[2][j];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      static_for<0, N>([&](auto i) {
        R acc = R(0);
        static_for<0, N>([&](auto j) {
          constexpr int h = tri(N, i, j);
          const R hv = HL ? Hs[(ax * LT::NH + h) * TS] : L.H[ax][h];
          acc += hv * rr[ax][j];
        });
        cr[ax][i] = acc;
      });
    }
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int j = 0; j < N; ++j)
        c[w][j] = L.U[3 * w] * cr[0][j] + L.U[3 * w + 1] * cr[1][j] + L.U[3 * w + 2] * cr[2][j];
  }

  // ---- corridor slack/dual pairs
  static_for<0, M>([&](auto s) {
    R p0 = R(0), p1 = R(0), p2 = R(0);
    static_for<0, N>([&](auto j) {
      constexpr R k = R(cpos(s, j));
      p0 += k * c[0][j];
      p1 += k * c[1][j];
      p2 += k * c[2][j];
    });
#pragma unroll
    for (int k = 0; k < KF; ++k)
      L.y[k][s] = L.fa[k][0] * p0 + L.fa[k][1] * p1 + L.fa[k][2] * p2 - L.fa[k][3] + relu(L.y[k][s]);
  });

  // ---- velocity pairs and end states, per axis
  R xL[3][S], xR[3][S];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if constexpr (VEL) {
      R ci[N];
#pragma unroll
      for (int j = 1; j < N; ++j) ci[j] = c[a][j] * L.iT;
      static_for<0, M>([&](auto s) {
        R vv = R(0);
        static_for<1, N>([&](auto j) {
          constexpr R k = R(cvel(s, j));
          vv += k * ci[j];
        });
        L.g[a][s] = vv + om[s] * L.g[a][s];
      });
    }
    static_for<0, S>([&](auto o) {
      constexpr R kf = R(cfact(o));
      xL[a][o] = kf * c[a][o] * L.iTp[o];
      R acc = R(0);
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        acc += k * c[a][j];
      });
      xR[a][o] = acc * L.iTp[o];
    });
    if constexpr (FINAL) {
#pragma unroll
      for (int j = 0; j < N; ++j) cfin[a][j] = c[a][j];
    }
  }
  knot_exchange_by_order<FINAL, P, S>(L, xL, xR, xr_sh, xl_sh, wl, wid, nw, zfin);
}

template <typename R, int P, int S, bool VEL, int LB, bool HL, int WPE>
__global__ __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(WPE))) void poly_sweep_kernel(SweepArgs<R> A) {
  using LT = PolyLane<R, P, S, VEL>;
  constexpr int N = LT::N;
  constexpr int NH = LT::NH;
  constexpr int M = LT::M;
  constexpr int KF = LT::KF;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_Y = 9 * S;
  constexpr int F_G = F_Y + KF * M;
  constexpr int NF = F_G + (VEL ? 3 * M : 0);

  __shared__ R xr_sh[2][kMaxWaves][3 * S];
  __shared__ R xl_sh[2][kMaxWaves][3 * S];

  const int W = A.W;
  const int lane = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * W;
  const int64_t ld = A.k.ld;
  const int32_t ent = A.lane_seg[base + lane];
  const bool active = ent >= 0;
  const bool core = active && !(ent & kHaloBit);
  const int64_t seg = active ? (int64_t)(ent & kSegMask) : 0;
  const uint8_t fl = active ? A.k.flags[seg] : (uint8_t)(kFirst | kLast);

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

  // ---- per-segment constants
  // matrices in LDS: rows strided by the largest tile LB (a compile-time stride: every LDS address
  // is an immediate offset from the lane's own column)
  extern __shared__ double poly_lds_raw[];
  R* Hs = reinterpret_cast<R*>(poly_lds_raw) + lane;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax)
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const R v = active ? A.k.Hr[(ax * NH + h) * ld + seg] : R(0);
      if constexpr (HL) Hs[(ax * NH + h) * LB] = v;
      else L.H[ax][h] = v;
    }
#pragma unroll
  for (int q = 0; q < 9; ++q) L.U[q] = active ? A.k.U[q * ld + seg] : R(0);
#pragma unroll
  for (int k = 0; k < KF; ++k)
#pragma unroll
    for (int q = 0; q < 4; ++q) L.fa[k][q] = active ? A.k.fa[(k * 4 + q) * ld + seg] : R(0);
  L.iT = active ? A.k.iT[seg] : R(1);
  L.vm = (VEL && active) ? A.k.vmax[seg] : R(1);
  L.iTp[0] = R(1);
#pragma unroll
  for (int o = 1; o < S; ++o) L.iTp[o] = L.iTp[o - 1] * L.iT;

  // ---- state
  const R* in = A.st_in;
  const int tr = active ? A.k.traj[seg] : 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 0; o < S; ++o) {
      const int f = a * S + o;
      L.zR[a][o] = active ? in[(F_ZR + f) * ld + seg] : R(0);
      L.uL[a][o] = active ? in[(F_UL + f) * ld + seg] : R(0);
      L.uR[a][o] = active ? in[(F_UR + f) * ld + seg] : R(0);
      L.zL[a][o] = !active ? R(0)
                 : L.first ? A.k.bcL[((int64_t)tr * 3 + a) * S + o]
                           : in[(F_ZR + f) * ld + seg - 1];
    }
#pragma unroll
    for (int s = 0; s < LT::MV; ++s) L.g[a][s] = (VEL && active) ? in[(F_G + a * M + s) * ld + seg] : R(0);
  }
#pragma unroll
  for (int k = 0; k < KF; ++k)
#pragma unroll
    for (int s = 0; s < M; ++s) L.y[k][s] = active ? in[(F_Y + k * M + s) * ld + seg] : R(0);

  const int wl = lane & 63, wid = lane >> 6, nw = W >> 6;
  // stopped trajectories: both state buffers hold their state; their lanes store nothing
  const bool frozen = active && A.done != nullptr && A.done[tr] != 0;
  if (__ballot(active && !frozen) == 0) {
    for (int it = 0; it < A.iters; ++it) __syncthreads();
    return;
  }
  R cfin[3][N], zfin[3][S];
  const int n_plain = A.final_out ? A.iters - 1 : A.iters;
  int it = 0;
  for (; it < n_plain; ++it)
    poly_sweep_once<false, HL, LB>(L, Hs, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
  if (A.final_out && A.iters > 0) {
    poly_sweep_once<true, HL, LB>(L, Hs, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
    if (core && !frozen) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int j = 0; j < N; ++j) A.c_out[(a * N + j) * ld + seg] = cfin[a][j];
#pragma unroll
        for (int o = 0; o < S; ++o) A.zold_out[(a * S + o) * ld + seg] = zfin[a][o];
      }
    }
  }
  if (core && !frozen) {
    R* out = A.st_out;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        const int f = a * S + o;
        out[(F_ZR + f) * ld + seg] = L.zR[a][o];
        out[(F_UL + f) * ld + seg] = L.uL[a][o];
        out[(F_UR + f) * ld + seg] = L.uR[a][o];
      }
      if constexpr (VEL) {
#pragma unroll
        for (int s = 0; s < M; ++s) out[(F_G + a * M + s) * ld + seg] = L.g[a][s];
      }
    }
#pragma unroll
    for (int k = 0; k < KF; ++k)
#pragma unroll
      for (int s = 0; s < M; ++s) out[(F_Y + k * M + s) * ld + seg] = L.y[k][s];
  }
}

template <typename R>
hipError_t dispatch_poly_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  if (v.faces != kFaces || v.box || a.rec != nullptr) return hipErrorInvalidValue;
  if (a.W <= 0 || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(a.W);
  // float32 quintic: matrices in LDS (252 bytes per lane, 129 KB for a 512-lane tile, within the
  // 160 KB a workgroup may hold), tiles up to 512 lanes, two waves per SIMD; otherwise matrices in
  // registers and tiles up to 256 lanes
  constexpr bool hl3 = std::is_same<R, float>::value;
#define TOP_POLY_CASE(P_, S_, V_)                                                             \
  if (v.p == P_ && v.s == S_ && (v.vel != 0) == V_) {                                       \
    constexpr bool HL_ = hl3 && P_ == 3;                                                    \
    constexpr int NH_ = 2 * P_ * (2 * P_ + 1) / 2;                                          \
    if (a.W > (HL_ ? 512 : 256)) return hipErrorInvalidValue;                               \
    const size_t lds = HL_ ? (size_t)3 * NH_ * 512 * sizeof(R) : 0;                         \
    auto k_ = poly_sweep_kernel<R, P_, S_, V_, HL_ ? 512 : 256, HL_, HL_ ? 2 : 1>;          \
    if (HL_) {                                                                              \
      hipError_t e_ = hipFuncSetAttribute((const void*)k_, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e_ != hipSuccess) return e_;                                                      \
    }                                                                                       \
    hipLaunchKernelGGL(k_, grid, block, lds, st, a);                                        \
    return hipGetLastError();                                                               \
  }
  TOP_POLY_CASE(3, 3, true) TOP_POLY_CASE(3, 3, false)
  TOP_POLY_CASE(3, 4, true) TOP_POLY_CASE(3, 4, false)
  TOP_POLY_CASE(4, 4, true) TOP_POLY_CASE(4, 4, false)
  TOP_POLY_CASE(4, 5, true) TOP_POLY_CASE(4, 5, false)
  TOP_POLY_CASE(3, 5, true) TOP_POLY_CASE(3, 5, false)
  TOP_POLY_CASE(4, 7, true) TOP_POLY_CASE(4, 7, false)
#undef TOP_POLY_CASE
  return hipErrorInvalidValue;
}

// Tiles of W lanes of the instance dispatch_poly_sweep launches for v that the device holds at
// once (0 if the runtime does not say).
template <typename R>
int resident_poly(const Variant& v, int W) {
  if (v.faces != kFaces || v.box || W <= 0 || (W & 63) != 0) return 0;
  constexpr bool hl3 = std::is_same<R, float>::value;
  void* k = nullptr;
  size_t lds = 0;
#define TOP_POLY_RES(P_, S_, V_)                                                              \
  if (k == nullptr && v.p == P_ && v.s == S_ && (v.vel != 0) == V_) {                       \
    constexpr bool HL_ = hl3 && P_ == 3;                                                    \
    constexpr int NH_ = 2 * P_ * (2 * P_ + 1) / 2;                                          \
    if (W > (HL_ ? 512 : 256)) return 0;                                                    \
    lds = HL_ ? (size_t)3 * NH_ * 512 * sizeof(R) : 0;                                      \
    k = reinterpret_cast<void*>(poly_sweep_kernel<R, P_, S_, V_, HL_ ? 512 : 256, HL_, HL_ ? 2 : 1>); \
  }
  TOP_POLY_RES(3, 3, true) TOP_POLY_RES(3, 3, false)
  TOP_POLY_RES(3, 4, true) TOP_POLY_RES(3, 4, false)
  TOP_POLY_RES(4, 4, true) TOP_POLY_RES(4, 4, false)
  TOP_POLY_RES(4, 5, true) TOP_POLY_RES(4, 5, false)
  TOP_POLY_RES(3, 5, true) TOP_POLY_RES(3, 5, false)
  TOP_POLY_RES(4, 7, true) TOP_POLY_RES(4, 7, false)
#undef TOP_POLY_RES
  if (k == nullptr) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (lds > 0 && hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, W, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

}  // namespace top
