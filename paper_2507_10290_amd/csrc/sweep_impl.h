// The fused CADMM sweep kernel (Sec. III-D.1 update rules, one pass of
// Algorithm 1's loop body per sweep), resident form.
//
// Mapping: one segment per lane; a workgroup tile holds up to W consecutive
// segments of one or more trajectories (whole trajectories packed, or a core
// range of one long trajectory plus `halo` copied neighbours on each side).
// The tile loads its segments' state once, runs `iters` sweeps with the state
// in registers, and stores the core segments' state once.  A sweep of a
// segment needs only its own state and, for the knot average, the end states
// of its two neighbours, so the halo copies absorb the one-segment-per-sweep
// spread of information from outside the tile.
//
// Per sweep and segment (normalised-time basis, see common.h), per axis a:
//   r~  = sum_o o! T^-o (zL_o - uL_o) e_o + sum_o T^-o (zR_o - uR_o) f_o
//       + sum_s tau_s (hi + lo - |y^hi_s| + |y^lo_s|)          [box rows, folded slack/dual]
//       + T^-1 sum_s tau'_s (2 Proj(g_s) - g_s)_a              [velocity rows, folded split/dual]
//   c~  = (rho Htilde^-1) r~                                   [eq. QpSubProblem]
//   y^hi_s <- tau_s.c~ - hi + max(0, y^hi_s),  y^lo_s <- lo - tau_s.c~ + max(0, y^lo_s)
//                                                              [eqs. NonNegativeProject, UpdateV]
//   g_s  <- T^-1 tau'_s.c~ + g_s - Proj(g_s)                   [eqs. DynamicProject, UpdateCloseW]
//   xL_o = o! T^-o c~_o, xR_o = T^-o f_o.c~                    [end states, beta~ of eq. UpdateZ]
// then, at each interior knot, z = (xR_i + xL_{i+1}) / 2 on the free orders [eq. UpdateZ] and
// u += x - z on both ends [eq. UpdateU].  The identities behind the folded pairs are
// b - s - v = b - |y| with y = A^o c - b + v, and phi - w = 2 Proj(g) - g with g = A^v c + w.
#pragma once

#include "common.h"

namespace top {

// 1/sqrt(x).  For fp32 the hardware reciprocal square root alone: the library form adds a rescaling
// of denormal inputs (five more instructions).  A denormal x only arises from a velocity split of
// norm below 1e-19, where rsq of the flushed input is +inf and the projection factor min(1, vmax/|g|)
// is 1 either way; for normal x both forms are the same instruction.
template <typename R>
__device__ inline R inv_sqrt(R x);
template <>
__device__ inline float inv_sqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <>
__device__ inline double inv_sqrt<double>(double x) { return 1.0 / sqrt(x); }

// max(0, x).  For fp32 this is one integer max on the bit pattern (non-negative floats order like
// their bits, negative ones have the sign bit set), which avoids the NaN-quieting copy an IEEE
// fmax needs; the result is the same for every finite x.
__device__ __forceinline__ float relu(float x) { return __int_as_float(max(__float_as_int(x), 0)); }
__device__ __forceinline__ double relu(double x) { return fmax(0.0, x); }

template <typename R, int P, int S, bool BOX, bool VEL>
struct Lane {
  static constexpr int N = 2 * P;
  static constexpr int NH = N * (N + 1) / 2;
  static constexpr int M = kSamples;
  static constexpr int MB = BOX ? M : 1;
  static constexpr int MV = VEL ? M : 1;
  // state
  R zL[3][S], zR[3][S], uL[3][S], uR[3][S], yh[3][MB], yl[3][MB], g[3][MV];
  // constants
  R H[NH], iT, iTp[S], lo[3], hi[3], vm;
  bool first, last, has_left, has_right, fixpos;
};

// Knot consensus and the u update after the local solves (eqs. UpdateZ, UpdateU): neighbours
// inside the wave by shuffles, across waves through LDS (one barrier).  LT is any lane type with
// the knot state zL, zR, uL, uR [3][S] and the neighbour flags.
template <bool FINAL, int P, int S, typename LT, typename R>
__device__ __forceinline__ void knot_exchange(LT& L, R (&xL)[3][S], R (&xR)[3][S], R (*xr_sh)[3 * S],
                                              R (*xl_sh)[3 * S], int wl, int wid, int nw, R (&zfin)[3][S]) {
  if (wl == 63) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < S; ++o) xr_sh[wid][a * S + o] = xR[a][o];
  }
  if (wl == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < S; ++o) xl_sh[wid][a * S + o] = xL[a][o];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R xp = __shfl_up(xR[a][o], 1);
      R xn = __shfl_down(xL[a][o], 1);
      if (wl == 0 && wid > 0) xp = xr_sh[wid - 1][a * S + o];
      if (wl == 63 && wid < nw - 1) xn = xl_sh[wid + 1][a * S + o];
      xp = L.has_left ? xp : xL[a][o];
      xn = L.has_right ? xn : xR[a][o];
      if constexpr (FINAL) zfin[a][o] = L.zR[a][o];
      const bool free_o = (o > 0) || !L.fixpos;
      const R zr_new = R(0.5) * (xR[a][o] + xn);
      const R zl_new = R(0.5) * (xp + xL[a][o]);
      L.zR[a][o] = (!L.last && free_o) ? zr_new : L.zR[a][o];
      L.zL[a][o] = (!L.first && free_o) ? zl_new : L.zL[a][o];
      const R du_l = xL[a][o] - L.zL[a][o];
      const R du_r = xR[a][o] - L.zR[a][o];
      L.uL[a][o] += (o < P || !L.first) ? du_l : R(0);
      L.uR[a][o] += (o < P || !L.last) ? du_r : R(0);
    }
  }
}

// One sweep of one lane's segment.  With FINAL the local solve c~ and the end knot before its
// update are returned through cfin / zfin.
template <bool FINAL, typename R, int P, int S, bool BOX, bool VEL>
__device__ __forceinline__ void sweep_once(Lane<R, P, S, BOX, VEL>& L, R (*xr_sh)[3 * S],
                                           R (*xl_sh)[3 * S], int wl, int wid, int nw,
                                           R (&cfin)[3][2 * P], R (&zfin)[3][S]) {
  using LT = Lane<R, P, S, BOX, VEL>;
  constexpr int N = LT::N;
  constexpr int M = LT::M;
  constexpr int MV = LT::MV;

  // velocity projection factors: Proj(g) = f g with f = min(1, vmax / ||g||); per sample, shared by
  // the three axes: q = (2f - 1) / T (right-hand side) and 1 - f (the g update)
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

  R xL[3][S], xR[3][S];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    R r[N];
#pragma unroll
    for (int j = 0; j < N; ++j) r[j] = R(0);
    static_for<0, S>([&](auto o) {
      const R wl_ = (L.zL[a][o] - L.uL[a][o]) * L.iTp[o];
      constexpr R kf = R(cfact(o));
      r[o] += kf * wl_;
      const R wr_ = (L.zR[a][o] - L.uR[a][o]) * L.iTp[o];
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        r[j] += k * wr_;
      });
    });
    if constexpr (BOX) {
      const R hl = L.hi[a] + L.lo[a];
      static_for<0, M>([&](auto s) {
        const R b = hl - fabs(L.yh[a][s]) + fabs(L.yl[a][s]);
        static_for<0, N>([&](auto j) {
          constexpr R k = R(cpos(s, j));
          r[j] += k * b;
        });
      });
    }
    if constexpr (VEL) {
      static_for<0, M>([&](auto s) {
        const R b = q[s] * L.g[a][s];
        static_for<1, N>([&](auto j) {
          constexpr R k = R(cvel(s, j));
          r[j] += k * b;
        });
      });
    }
    R c[N];
    static_for<0, N>([&](auto i) {
      R acc = R(0);
      static_for<0, N>([&](auto j) { acc += L.H[tri(N, i, j)] * r[j]; });
      c[i] = acc;
    });
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        R pv = R(0);
        static_for<0, N>([&](auto j) {
          constexpr R k = R(cpos(s, j));
          pv += k * c[j];
        });
        L.yh[a][s] = pv - L.hi[a] + relu(L.yh[a][s]);
        L.yl[a][s] = L.lo[a] - pv + relu(L.yl[a][s]);
      });
    }
    if constexpr (VEL) {
      R ci[N];                                  // c~ / T: the velocity rows carry 1/T
#pragma unroll
      for (int j = 1; j < N; ++j) ci[j] = c[j] * L.iT;
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
      xL[a][o] = kf * c[o] * L.iTp[o];
      R acc = R(0);
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        acc += k * c[j];
      });
      xR[a][o] = acc * L.iTp[o];
    });
    if constexpr (FINAL) {
#pragma unroll
      for (int j = 0; j < N; ++j) cfin[a][j] = c[j];
    }
  }

  knot_exchange<FINAL, P, S>(L, xL, xR, xr_sh, xl_sh, wl, wid, nw, zfin);
}

// ---- The same arithmetic split by axis, for the lane-per-axis sweep (sweep_axis_impl.h).  Each
// function repeats, statement for statement, the corresponding part of knot_exchange and sweep_once
// above (which keep their own inline form: the one-lane kernel's schedule is tuned around it), so both
// forms compute the same bits; the GPU tests compare them.

// Consensus and dual update of one knot order of one axis (eqs. UpdateZ, UpdateU), given the
// segment's own end states xl / xr and its neighbours' (xp: the left neighbour's end state, xn: the
// right neighbour's start state; ignored without a neighbour).
template <bool FINAL, int P, typename R>
__device__ __forceinline__ void knot_update(int o, R xl, R xr, R xp, R xn, bool has_left, bool has_right,
                                            bool first, bool last, bool fixpos, R& zL, R& zR, R& uL, R& uR,
                                            R& zfin) {
  xp = has_left ? xp : xl;
  xn = has_right ? xn : xr;
  if constexpr (FINAL) zfin = zR;
  const bool free_o = (o > 0) || !fixpos;
  const R zr_new = R(0.5) * (xr + xn);
  const R zl_new = R(0.5) * (xp + xl);
  zR = (!last && free_o) ? zr_new : zR;
  zL = (!first && free_o) ? zl_new : zL;
  const R du_l = xl - zL;
  const R du_r = xr - zR;
  uL += (o < P || !first) ? du_l : R(0);
  uR += (o < P || !last) ? du_r : R(0);
}

// knot_exchange with the per-order update of knot_update (the same arithmetic); the polytope sweep
// uses this form, which schedules better there (10.2 against 11.2 ms for the 8-face batched solve).
template <bool FINAL, int P, int S, typename LT, typename R>
__device__ __forceinline__ void knot_exchange_by_order(LT& L, R (&xL)[3][S], R (&xR)[3][S], R (*xr_sh)[3 * S],
                                                       R (*xl_sh)[3 * S], int wl, int wid, int nw,
                                                       R (&zfin)[3][S]) {
  if (wl == 63) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < S; ++o) xr_sh[wid][a * S + o] = xR[a][o];
  }
  if (wl == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < S; ++o) xl_sh[wid][a * S + o] = xL[a][o];
  }
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R xp = __shfl_up(xR[a][o], 1);
      R xn = __shfl_down(xL[a][o], 1);
      if (wl == 0 && wid > 0) xp = xr_sh[wid - 1][a * S + o];
      if (wl == 63 && wid < nw - 1) xn = xl_sh[wid + 1][a * S + o];
      knot_update<FINAL, P>(o, xL[a][o], xR[a][o], xp, xn, L.has_left, L.has_right, L.first, L.last, L.fixpos,
                            L.zL[a][o], L.zR[a][o], L.uL[a][o], L.uR[a][o], zfin[a][o]);
    }
  }
}

// Velocity projection factors of one sample: Proj(g) = f g with f = min(1, vmax / ||g||); returns
// q = (2f - 1) / T (right-hand side) and om = 1 - f (the g update).
template <typename R>
__device__ __forceinline__ void vel_factors(R g0, R g1, R g2, R vm, R iT, R& q, R& om) {
  const R n2 = g0 * g0 + g1 * g1 + g2 * g2;
  const R f = fmin(R(1), vm * inv_sqrt<R>(n2));
  q = (R(2) * f - R(1)) * iT;
  om = R(1) - f;
}

// The local work of one axis of one segment: the right-hand side r~, the local solve
// c~ = (rho Htilde^-1) r~, the box and velocity pair updates and the end states xL / xR.  H(h) is
// the packed matrix entry h; q / om are the velocity factors of the samples.
template <bool FINAL, typename R, int P, int S, bool BOX, bool VEL, typename HF>
__device__ __forceinline__ void axis_update(const HF& H, R iT, const R (&iTp)[S], R lo, R hi,
                                            const R (&q)[VEL ? kSamples : 1], const R (&om)[VEL ? kSamples : 1],
                                            const R (&zL)[S], const R (&zR)[S], const R (&uL)[S], const R (&uR)[S],
                                            R (&yh)[BOX ? kSamples : 1], R (&yl)[BOX ? kSamples : 1],
                                            R (&g)[VEL ? kSamples : 1], R (&xL)[S], R (&xR)[S], R (&cfin)[2 * P]) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  R r[N];
#pragma unroll
  for (int j = 0; j < N; ++j) r[j] = R(0);
  static_for<0, S>([&](auto o) {
    const R wl_ = (zL[o] - uL[o]) * iTp[o];
    constexpr R kf = R(cfact(o));
    r[o] += kf * wl_;
    const R wr_ = (zR[o] - uR[o]) * iTp[o];
    static_for<o, N>([&](auto j) {
      constexpr R k = R(cfall(o, j));
      r[j] += k * wr_;
    });
  });
  if constexpr (BOX) {
    const R hl = hi + lo;
    static_for<0, M>([&](auto s) {
      const R b = hl - fabs(yh[s]) + fabs(yl[s]);
      static_for<0, N>([&](auto j) {
        constexpr R k = R(cpos(s, j));
        r[j] += k * b;
      });
    });
  }
  if constexpr (VEL) {
    static_for<0, M>([&](auto s) {
      const R b = q[s] * g[s];
      static_for<1, N>([&](auto j) {
        constexpr R k = R(cvel(s, j));
        r[j] += k * b;
      });
    });
  }
  R c[N];
  static_for<0, N>([&](auto i) {
    R acc = R(0);
    static_for<0, N>([&](auto j) { acc += H(tri(N, i, j)) * r[j]; });
    c[i] = acc;
  });
  if constexpr (BOX) {
    static_for<0, M>([&](auto s) {
      R pv = R(0);
      static_for<0, N>([&](auto j) {
        constexpr R k = R(cpos(s, j));
        pv += k * c[j];
      });
      yh[s] = pv - hi + relu(yh[s]);
      yl[s] = lo - pv + relu(yl[s]);
    });
  }
  if constexpr (VEL) {
    R ci[N];                                  // c~ / T: the velocity rows carry 1/T
#pragma unroll
    for (int j = 1; j < N; ++j) ci[j] = c[j] * iT;
    static_for<0, M>([&](auto s) {
      R vv = R(0);
      static_for<1, N>([&](auto j) {
        constexpr R k = R(cvel(s, j));
        vv += k * ci[j];
      });
      g[s] = vv + om[s] * g[s];
    });
  }
  static_for<0, S>([&](auto o) {
    constexpr R kf = R(cfact(o));
    xL[o] = kf * c[o] * iTp[o];
    R acc = R(0);
    static_for<o, N>([&](auto j) {
      constexpr R k = R(cfall(o, j));
      acc += k * c[j];
    });
    xR[o] = acc * iTp[o];
  });
  if constexpr (FINAL) {
#pragma unroll
    for (int j = 0; j < N; ++j) cfin[j] = c[j];
  }
}

// Waves per SIMD the compiler must leave room for.  The float32 septic box + velocity instance
// needs a few VGPRs more than half the file; held to two waves per SIMD, a CU keeps two 256-lane
// tiles resident, which pays when a launch has more tiles than CUs (one long trajectory).
template <typename R, int P, int S, bool BOX, bool VEL, bool REC>
constexpr int sweep_min_waves() {
  return (sizeof(R) == 4 && P == 4 && S == 4 && BOX && VEL && !REC) ? 2 : 1;
}

// REC: the instance used to replay checkpoint blocks for the reverse pass; it also stores the state
// after every sweep but the last (the ordinary instance never stores inside its sweep loop).
template <typename R, int P, int S, bool BOX, bool VEL, int LB, bool REC = false>
__global__ __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<R, P, S, BOX, VEL, REC>())))
void sweep_kernel(SweepArgs<R> A) {
  using LT = Lane<R, P, S, BOX, VEL>;
  constexpr int N = LT::N;
  constexpr int NH = LT::NH;
  constexpr int M = LT::M;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_G = 9 * S + (BOX ? 6 * M : 0);

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

  // A stopped trajectory keeps its state: both state buffers already hold it, so its lanes sweep
  // along (their neighbours belong to the same trajectory, so nothing leaks) and leave c~ and the old
  // knot alone; with store_frozen they also store their input state into the output buffer.
  const int tr = active ? A.k.traj[seg] : 0;
  const bool frozen = active && A.done != nullptr && A.done[tr] != 0;
  if (A.done != nullptr) {
    // Before any state is loaded: a tile with no live segment is done; a wave with none only keeps
    // the workgroup's barrier count (one per sweep).
    if (__syncthreads_or(active && !frozen) == 0) return;
    if (__ballot(active && !frozen) == 0) {
      for (int it = 0; it < A.iters; ++it) __syncthreads();
      return;
    }
  }

  // ---- per-segment constants
#pragma unroll
  for (int h = 0; h < NH; ++h) L.H[h] = active ? A.k.Hr[h * ld + seg] : R(0);
  L.iT = active ? A.k.iT[seg] : R(1);
  L.vm = (VEL && active) ? A.k.vmax[seg] : R(1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    L.lo[a] = (BOX && active) ? A.k.lo[a * ld + seg] : R(0);
    L.hi[a] = (BOX && active) ? A.k.hi[a * ld + seg] : R(0);
  }
  L.iTp[0] = R(1);
#pragma unroll
  for (int o = 1; o < S; ++o) L.iTp[o] = L.iTp[o - 1] * L.iT;

  // ---- state
  const R* in = A.st_in;
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
    for (int s = 0; s < LT::MB; ++s) {
      L.yh[a][s] = (BOX && active) ? in[(F_YH + a * M + s) * ld + seg] : R(0);
      L.yl[a][s] = (BOX && active) ? in[(F_YL + a * M + s) * ld + seg] : R(0);
    }
#pragma unroll
    for (int s = 0; s < LT::MV; ++s) L.g[a][s] = (VEL && active) ? in[(F_G + a * M + s) * ld + seg] : R(0);
  }

  const int wl = lane & 63, wid = lane >> 6, nw = W >> 6;
  auto copy_through = [&]() {
    constexpr int NF = F_G + (VEL ? 3 * M : 0);
#pragma unroll 4
    for (int f = 0; f < NF; ++f) A.st_out[f * ld + seg] = in[f * ld + seg];
  };
  auto store_to = [&](R* out) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        const int f = a * S + o;
        out[(F_ZR + f) * ld + seg] = L.zR[a][o];
        out[(F_UL + f) * ld + seg] = L.uL[a][o];
        out[(F_UR + f) * ld + seg] = L.uR[a][o];
      }
      if constexpr (BOX) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
          out[(F_YH + a * M + s) * ld + seg] = L.yh[a][s];
          out[(F_YL + a * M + s) * ld + seg] = L.yl[a][s];
        }
      }
      if constexpr (VEL) {
#pragma unroll
        for (int s = 0; s < M; ++s) out[(F_G + a * M + s) * ld + seg] = L.g[a][s];
      }
    }
  };
  R cfin[3][N], zfin[3][S];
  const int n_plain = A.final_out ? A.iters - 1 : A.iters;
  int it = 0;
  for (; it < n_plain; ++it) {
    sweep_once<false>(L, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
    if constexpr (REC) {
      if (core && it + 1 < A.iters) store_to(A.rec + (int64_t)(it + 1) * A.rec_slot);
    }
  }
  if (A.final_out && A.iters > 0) {
    sweep_once<true>(L, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
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

  if (core && frozen && A.store_frozen) copy_through();
  if (core && !frozen) store_to(A.st_out);
}

// LB3 / LB4: largest tile (launch bound) for the quintic / septic kernels.  The consensus on all
// orders 0..2p-2 (s = 2p-1) carries more knot state and uses tiles of up to 256 lanes; it has no
// recording instance (no tape).
template <typename R, int LB3, int LB4>
hipError_t dispatch_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  const bool rec = a.rec != nullptr;
  const bool full = v.s == 2 * v.p - 1;
  const int lb = (rec || full) ? 256 : (v.p == 3) ? LB3 : LB4;
  if (rec && full) return hipErrorInvalidValue;
  if (a.W <= 0 || a.W > lb || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(a.W);
#define TOP_SWEEP_CASE(P_, S_, B_, V_, LB_)                                                   \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {                 \
    if (rec) hipLaunchKernelGGL((sweep_kernel<R, P_, S_, B_, V_, 256, true>), grid, block, 0, st, a); \
    else hipLaunchKernelGGL((sweep_kernel<R, P_, S_, B_, V_, LB_>), grid, block, 0, st, a);  \
    return hipGetLastError();                                                               \
  }
#define TOP_SWEEP_PS(P_, S_, LB_)                                                             \
  TOP_SWEEP_CASE(P_, S_, true, true, LB_)                                                     \
  TOP_SWEEP_CASE(P_, S_, true, false, LB_)                                                    \
  TOP_SWEEP_CASE(P_, S_, false, true, LB_)                                                    \
  TOP_SWEEP_CASE(P_, S_, false, false, LB_)
  TOP_SWEEP_PS(3, 3, LB3)
  TOP_SWEEP_PS(3, 4, LB3)
  TOP_SWEEP_PS(4, 4, LB4)
  TOP_SWEEP_PS(4, 5, LB4)
#undef TOP_SWEEP_PS
#undef TOP_SWEEP_CASE
#define TOP_SWEEP_FULL(P_, S_, B_, V_)                                                        \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {                 \
    hipLaunchKernelGGL((sweep_kernel<R, P_, S_, B_, V_, 256>), grid, block, 0, st, a);       \
    return hipGetLastError();                                                               \
  }
  TOP_SWEEP_FULL(3, 5, true, true) TOP_SWEEP_FULL(3, 5, true, false)
  TOP_SWEEP_FULL(3, 5, false, true) TOP_SWEEP_FULL(3, 5, false, false)
  TOP_SWEEP_FULL(4, 7, true, true) TOP_SWEEP_FULL(4, 7, true, false)
  TOP_SWEEP_FULL(4, 7, false, true) TOP_SWEEP_FULL(4, 7, false, false)
#undef TOP_SWEEP_FULL
  return hipErrorInvalidValue;
}

// The (non-recording) kernel instance dispatch_sweep launches for variant v, or nullptr.
template <typename R, int LB3, int LB4>
void* sweep_instance(const Variant& v) {
  if (v.faces || v.num) return nullptr;
  const bool full = v.s == 2 * v.p - 1;
#define TOP_SWEEP_I(P_, S_, B_, V_, LB_)                                                      \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_)                   \
    return reinterpret_cast<void*>(sweep_kernel<R, P_, S_, B_, V_, LB_>);
#define TOP_SWEEP_IPS(P_, S_, LB_)                                                            \
  TOP_SWEEP_I(P_, S_, true, true, LB_) TOP_SWEEP_I(P_, S_, true, false, LB_)                 \
  TOP_SWEEP_I(P_, S_, false, true, LB_) TOP_SWEEP_I(P_, S_, false, false, LB_)
  if (!full) {
    TOP_SWEEP_IPS(3, 3, LB3) TOP_SWEEP_IPS(3, 4, LB3) TOP_SWEEP_IPS(4, 4, LB4) TOP_SWEEP_IPS(4, 5, LB4)
  } else {
    TOP_SWEEP_IPS(3, 5, 256) TOP_SWEEP_IPS(4, 7, 256)
  }
#undef TOP_SWEEP_IPS
#undef TOP_SWEEP_I
  return nullptr;
}

// Tiles of W lanes of that instance the device holds at once (0 if the runtime does not say).
template <typename R, int LB3, int LB4>
int resident_sweep(const Variant& v, int W) {
  void* k = sweep_instance<R, LB3, LB4>(v);
  if (k == nullptr || W <= 0) return 0;
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, W, 0) != hipSuccess) return 0;
  return per_cu * cus;
}

// Largest tile the kernel of this variant accepts.
inline int max_tile_lanes(const Variant& v) {
  return (v.prec == 0 && v.p == 3 && v.s != 2 * v.p - 1) ? 512 : 256;
}

}  // namespace top
