// Reverse-mode derivative of the sweep (the update rules of Sec. III-D.1 as
// computed by sweep_impl.h, folded slack/dual form), resident form.
//
// One launch runs `steps` reverse steps of consecutive forward sweeps.  The
// forward state before each of those sweeps is read from a block buffer that
// a replay of the block has filled; the adjoint state stays in registers,
// one lane per segment and axis.
// Knot adjoints are owned by the segment on the knot's left (as the knot
// values are in the forward state); each reverse step needs two neighbour
// exchanges: the new-knot adjoints before the local work, and the start-knot
// contributions of each segment's local solve after it.
//
// For a forward sweep s -> s' of one segment (per axis a; see sweep_impl.h):
//   u'  = u + m (x - z')             z' = (xR_i + xL_{i+1}) / 2 (free orders) or z (pinned)
//   y'  = A c - b + max(0, y)        g' = T^-1 tau'.c + (1 - f) g,  f = min(1, vmax/||g||)
//   x   = end states of c,           c  = (rho Htilde^-1) r~(z, u, y, g; 1/T)
// the reverse step maps the adjoint of s' to the adjoint of s and adds the
// parameter adjoints of 1/T and of rho Htilde^-1 (contracted with its T-derivative).
#pragma once

#include "common.h"
#include "sweep_impl.h"

namespace top {

template <typename R>
struct AdjArgs {
  SegConsts<R> k;
  const R* Hd;               // [nh][ld] d(rho Htilde^-1)/dT
  const int32_t* lane_seg;
  int W;
  int fixpos;
  const R* blk;              // forward state before sweep t of this launch at blk + t * slot
  const R* blk0;             // or, for t = 0, here when non-null (the block's checkpoint in the tape)
  int64_t slot;
  int steps;
  const R* adj_in;           // adjoint of the state after the last sweep of this launch
  R* adj_out;                // adjoint of the state before the first sweep
  const double* dcost;       // [B] upstream derivative of each trajectory's cost
  int with_cost;             // the last sweep of this launch produced the returned coefficients
  R* acc_iT;                 // [ld] += adjoint of 1/T
  R* acc_hd;                 // [ld] += <adjoint of rho Htilde^-1, its T-derivative>
  R* acc_z0;                 // [3s][ld] += adjoint of the trajectory's start-knot state (first segments)
};

template <typename R>
__device__ __forceinline__ R sgn(R x) { return x > R(0) ? R(1) : (x < R(0) ? R(-1) : R(0)); }

// Lane mapping: one lane per (segment, axis).  A tile of W segments runs as 3W threads, axis-major
// (thread a W + l holds axis a of the tile's segment l), so every wave belongs to one axis and the
// knot exchanges are the same wave shuffles and LDS hand-offs as with one lane per segment, among
// the waves of one axis.  The axes couple only through the velocity ball: each lane reads the three
// axes' split values g to form the projection factor, and the factor's adjoint (a sum over the three
// axes) goes through LDS beside the second knot exchange.  The parameter adjoints are summed over
// the three lanes of a segment, in axis order, at the end.
template <typename R, int P, int S, bool BOX, bool VEL, int LB>
__global__ __launch_bounds__(LB) void adjoint_kernel(AdjArgs<R> A) {
  constexpr int N = 2 * P;
  constexpr int NH = N * (N + 1) / 2;
  constexpr int M = kSamples;
  constexpr int MB = BOX ? M : 1;
  constexpr int MV = VEL ? M : 1;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_G = 9 * S + (BOX ? 6 * M : 0);

  // Wave-boundary values, indexed by the wave's place in its axis group.  E1 and E2 use separate
  // arrays: a wave may write its E2 values while a slower wave still reads E1 values of the same
  // step (no barrier lies between those).
  __shared__ R sh_r[2][3][kMaxAxisWaves][2 * S];   // E1, to the right neighbour: lz, luR
  __shared__ R sh_l[2][3][kMaxAxisWaves][S];       // E1, to the left neighbour: luL
  __shared__ R sh_c[2][3][kMaxAxisWaves][S];       // E2, to the left neighbour: cL
  // Dynamic LDS: the segment's rho Htilde^-1 and its T-derivative [2][NH][W] (read by the three
  // lanes of the segment), the per-axis partial adjoints of the velocity factors [2][3][MV][W], and
  // the per-axis parameter adjoints [3][2][W] of the end.
  extern __shared__ double adj_lds_raw[];
  // rows strided by the instance's largest tile TS (a compile-time stride: every LDS address is an
  // immediate offset from the lane's own column)
  constexpr int TS = LB / 3;
  R* sh_H = reinterpret_cast<R*>(adj_lds_raw) + threadIdx.x % A.W;
  R* sh_f = sh_H + 2 * NH * TS;

  const int W = A.W;
  const int a = threadIdx.x / W;      // axis of this lane
  const int lane = threadIdx.x - a * W;  // segment lane within the tile
  const int64_t base = (int64_t)blockIdx.x * W;
  const int64_t ld = A.k.ld;
  const int32_t ent = A.lane_seg[base + lane];
  const bool active = ent >= 0;
  const bool core = active && !(ent & kHaloBit);
  const int64_t seg = active ? (int64_t)(ent & kSegMask) : 0;
  const uint8_t fl = active ? A.k.flags[seg] : (uint8_t)(kFirst | kLast);
  const bool first = fl & kFirst, last = fl & kLast;
  bool has_left = false, has_right = false;
  if (active && !first && lane > 0) {
    const int32_t e = A.lane_seg[base + lane - 1];
    has_left = e >= 0 && (int64_t)(e & kSegMask) == seg - 1;
  }
  if (active && !last && lane < W - 1) {
    const int32_t e = A.lane_seg[base + lane + 1];
    has_right = e >= 0 && (int64_t)(e & kSegMask) == seg + 1;
  }
  const bool fixpos = A.fixpos != 0;
  const int wl = lane & 63, wid = lane >> 6, nw = W >> 6;
  auto SF = [&](int buf, int ax, int s) -> R& { return sh_f[((buf * 3 + ax) * MV + s) * TS]; };
  auto SA = [&](int ax, int q) -> R& { return sh_f[(2 * 3 * MV + ax * 2 + q) * TS]; };
  if (__ballot(active) == 0) {
    for (int t = 0; t < A.steps; ++t) { __syncthreads(); __syncthreads(); }
    __syncthreads();
    return;
  }

  // the matrices go to LDS once (axis 0 lanes: rho Htilde^-1, axis 1 lanes: its T-derivative); the
  // first step's barrier orders these stores before any read
  const R* Hsrc = a == 0 ? A.k.Hr : A.Hd;
  if (a < 2) {
#pragma unroll
    for (int h = 0; h < NH; ++h) sh_H[(a * NH + h) * TS] = active ? Hsrc[h * ld + seg] : R(0);
  }
  auto H = [&](int h) -> R { return sh_H[h * TS]; };
  auto Hd = [&](int h) -> R { return sh_H[(NH + h) * TS]; };
  const R iT = active ? A.k.iT[seg] : R(1);
  const R vm = (VEL && active) ? A.k.vmax[seg] : R(1);
  const R lo = (BOX && active) ? A.k.lo[a * ld + seg] : R(0);
  const R hi = (BOX && active) ? A.k.hi[a * ld + seg] : R(0);
  R iTp[N];
  iTp[0] = R(1);
#pragma unroll
  for (int o = 1; o < N; ++o) iTp[o] = iTp[o - 1] * iT;
  const int tr = active ? A.k.traj[seg] : 0;
  const R dc = (active && A.with_cost) ? (R)A.dcost[tr] : R(0);
  // the trajectory's start-knot state (the forward start knot of a first segment)
  R zL0[S];
#pragma unroll
  for (int o = 0; o < S; ++o) zL0[o] = (active && first) ? A.k.bcL[((int64_t)tr * 3 + a) * S + o] : R(0);

  // adjoint state of this axis, in registers
  R lz[S], luL[S], luR[S], az0[S], LYH[MB], LYL[MB], LG[MV];
  const R* ai = A.adj_in;
#pragma unroll
  for (int o = 0; o < S; ++o) {
    lz[o] = active ? ai[(F_ZR + a * S + o) * ld + seg] : R(0);
    luL[o] = active ? ai[(F_UL + a * S + o) * ld + seg] : R(0);
    luR[o] = active ? ai[(F_UR + a * S + o) * ld + seg] : R(0);
    az0[o] = R(0);
  }
#pragma unroll
  for (int s = 0; s < MB; ++s) {
    LYH[s] = (BOX && active) ? ai[(F_YH + a * M + s) * ld + seg] : R(0);
    LYL[s] = (BOX && active) ? ai[(F_YL + a * M + s) * ld + seg] : R(0);
  }
#pragma unroll
  for (int s = 0; s < MV; ++s) LG[s] = (VEL && active) ? ai[(F_G + a * M + s) * ld + seg] : R(0);
  R aiT = R(0), ahd = R(0);

  for (int t = A.steps - 1; t >= 0; --t) {
    const R* st = (t == 0 && A.blk0 != nullptr) ? A.blk0 : A.blk + (int64_t)t * A.slot;
    const bool cost_step = A.with_cost && (t == A.steps - 1);
    const int buf = t & 1;

    // ---- forward state before this sweep: this axis' values, and the velocity factors (from all
    // three axes' split values, the same operations on each lane of the segment).  Loaded before
    // the first exchange, whose barrier then hides part of the loads' latency.
    // (every lane loads unconditionally: an idle lane's seg is 0, a valid column, so it computes on
    // finite values that reach no active lane and no output; a first segment reads its own column
    // for the start knot and takes the boundary state instead)
    R zL[S], zR[S], uL[S], uR[S], yh[MB], yl[MB], g[MV];
    const int64_t prev = (active && !first) ? seg - 1 : seg;
#pragma unroll
    for (int o = 0; o < S; ++o) {
      const int fo = a * S + o;
      zR[o] = st[(F_ZR + fo) * ld + seg];
      uL[o] = st[(F_UL + fo) * ld + seg];
      uR[o] = st[(F_UR + fo) * ld + seg];
      const R vzl = st[(F_ZR + fo) * ld + prev];
      zL[o] = first ? zL0[o] : vzl;
    }
#pragma unroll
    for (int s = 0; s < MB; ++s) {
      yh[s] = BOX ? st[(F_YH + a * M + s) * ld + seg] : R(0);
      yl[s] = BOX ? st[(F_YL + a * M + s) * ld + seg] : R(0);
    }
    R gs[3][MV];
#pragma unroll
    for (int s = 0; s < MV; ++s)
#pragma unroll
      for (int b = 0; b < 3; ++b) gs[b][s] = VEL ? st[(F_G + b * M + s) * ld + seg] : R(0);

    // ---- E1: adjoints of the new knot values.  Lam_k = lz(i) - luR(i) - luL(i+1) at an
    // interior knot k between segments i and i+1; both lanes form it with the same operations.
    if (wl == 63) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        sh_r[buf][a][wid][o] = lz[o];
        sh_r[buf][a][wid][S + o] = luR[o];
      }
    }
    if (wl == 0) {
#pragma unroll
      for (int o = 0; o < S; ++o) sh_l[buf][a][wid][o] = luL[o];
    }
    __syncthreads();
    R LamL[S], LamR[S];
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R pz = __shfl_up(lz[o], 1);
      R pu = __shfl_up(luR[o], 1);
      R nu = __shfl_down(luL[o], 1);
      if (wl == 0 && wid > 0) { pz = sh_r[buf][a][wid - 1][o]; pu = sh_r[buf][a][wid - 1][S + o]; }
      if (wl == 63 && wid < nw - 1) nu = sh_l[buf][a][wid + 1][o];
      const bool mR = (o < P) || !last;
      const bool mL = (o < P) || !first;
      LamR[o] = has_right ? (lz[o] - luR[o]) - nu : (lz[o] - (mR ? luR[o] : R(0)));
      LamL[o] = has_left ? (pz - pu) - luL[o] : -(mL ? luL[o] : R(0));
    }

    R f[MV], rs2[MV], lf[MV];
    bool outside[MV];
#pragma unroll
    for (int s = 0; s < MV; ++s) {
      lf[s] = R(0);
      if constexpr (VEL) {
        g[s] = a == 0 ? gs[0][s] : (a == 1 ? gs[1][s] : gs[2][s]);
        const R n2 = gs[0][s] * gs[0][s] + gs[1][s] * gs[1][s] + gs[2][s] * gs[2][s];
        const R q = vm * inv_sqrt<R>(n2);
        outside[s] = q < R(1);
        f[s] = fmin(R(1), q);
        rs2[s] = outside[s] ? R(1) / n2 : R(0);
      } else {
        g[s] = R(0);
        f[s] = R(1);
        rs2[s] = R(0);
        outside[s] = false;
      }
    }

    // ---- recompute r~ and c of this axis exactly as the forward sweep does
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
        const R b = ((R(2) * f[s] - R(1)) * iT) * g[s];
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

    // ---- adjoint of c: through the end states, box rows, velocity rows (and the cost)
    R lc[N];
#pragma unroll
    for (int j = 0; j < N; ++j) lc[j] = R(0);
    static_for<0, S>([&](auto o) {
      const bool mL = (o < P) || !first;
      const bool mR = (o < P) || !last;
      const bool free_o = (o > 0) || !fixpos;
      R lxl = mL ? luL[o] : R(0);
      if (!first && free_o) lxl += R(0.5) * LamL[o];
      R lxr = mR ? luR[o] : R(0);
      if (!last && free_o) lxr += R(0.5) * LamR[o];
      constexpr R kf = R(cfact(o));
      lc[o] += kf * iTp[o] * lxl;
      R fc = R(0);
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        fc += k * c[j];
        lc[j] += k * (iTp[o] * lxr);
      });
      if constexpr (o > 0) {
        aiT += R(o) * iTp[o - 1] * (kf * c[o] * lxl + fc * lxr);
      }
    });
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        const R d = LYH[s] - LYL[s];
        static_for<0, N>([&](auto j) {
          constexpr R k = R(cpos(s, j));
          lc[j] += k * d;
        });
      });
    }
    if constexpr (VEL) {
      static_for<0, M>([&](auto s) {
        R dv = R(0);
        const R t_ = iT * LG[s];
        static_for<1, N>([&](auto j) {
          constexpr R k = R(cvel(s, j));
          dv += k * c[j];
          lc[j] += k * t_;
        });
        aiT += LG[s] * dv;
        lf[s] -= LG[s] * g[s];   // from g' = vv + (1 - f) g
      });
    }
    if (cost_step) {
      // J = T^(1-2p) c^T Q(1) c, summed over the axes
      R q = R(0);
      static_for<P, N>([&](auto j) {
        R qc = R(0);
        static_for<P, N>([&](auto k) {
          constexpr R gq = R(cgram(P, j, k));
          qc += gq * c[k];
        });
        q += qc * c[j];
        lc[j] += R(2) * dc * iTp[2 * P - 1] * qc;
      });
      aiT += dc * R(2 * P - 1) * iTp[2 * P - 2] * q;
    }

    // ---- old-state adjoints of the box and velocity pairs (through max(0, y) and (1 - f) g)
    if constexpr (BOX) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        LYH[s] = yh[s] > R(0) ? LYH[s] : R(0);
        LYL[s] = yl[s] > R(0) ? LYL[s] : R(0);
      }
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) LG[s] = (R(1) - f[s]) * LG[s];
    }

    // ---- through the local solve: lr = (rho Htilde^-1) lc; T-derivative of the matrix
    R lr[N];
    static_for<0, N>([&](auto i) {
      R acc = R(0), hr = R(0);
      static_for<0, N>([&](auto j) {
        acc += H(tri(N, i, j)) * lc[j];
        hr += Hd(tri(N, i, j)) * r[j];
      });
      lr[i] = acc;
      ahd += lc[i] * hr;
    });

    // ---- through r~
    R cL[S], cR[S];
    static_for<0, S>([&](auto o) {
      constexpr R kf = R(cfact(o));
      const R cl = kf * iTp[o] * lr[o];
      cL[o] = cl;
      R fl_ = R(0);
      static_for<o, N>([&](auto j) {
        constexpr R k = R(cfall(o, j));
        fl_ += k * lr[j];
      });
      const R cr = iTp[o] * fl_;
      cR[o] = cr;
      if constexpr (o > 0) {
        aiT += R(o) * iTp[o - 1] * (kf * (zL[o] - uL[o]) * lr[o] + (zR[o] - uR[o]) * fl_);
      }
      luL[o] -= cl;
      luR[o] -= cr;
    });
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        R lb = R(0);
        static_for<0, N>([&](auto j) {
          constexpr R k = R(cpos(s, j));
          lb += k * lr[j];
        });
        LYH[s] -= sgn(yh[s]) * lb;
        LYL[s] += sgn(yl[s]) * lb;
      });
    }
    if constexpr (VEL) {
      static_for<0, M>([&](auto s) {
        R lt = R(0);
        static_for<1, N>([&](auto j) {
          constexpr R k = R(cvel(s, j));
          lt += k * lr[j];
        });
        lf[s] += R(2) * iT * g[s] * lt;
        LG[s] += iT * (R(2) * f[s] - R(1)) * lt;
        aiT += (R(2) * f[s] - R(1)) * g[s] * lt;
      });
    }

    // ---- E2: start-knot contributions cL go to the owner of that knot (left neighbour); the
    // velocity factors' partial adjoints go to the other two lanes of the segment
    if (wl == 0) {
#pragma unroll
      for (int o = 0; o < S; ++o) sh_c[buf][a][wid][o] = cL[o];
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) SF(buf, a, s) = lf[s];
    }
    __syncthreads();
    // ---- through f = min(1, vmax/||g||): outside the ball df/dg = -f g / ||g||^2
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        const R lfs = (SF(buf, 0, s) + SF(buf, 1, s)) + SF(buf, 2, s);
        const R w = outside[s] ? -lfs * f[s] * rs2[s] : R(0);
        LG[s] += w * g[s];
      }
    }
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R nc = __shfl_down(cL[o], 1);
      if (wl == 63 && wid < nw - 1) nc = sh_c[buf][a][wid + 1][o];
      const bool free_o = (o > 0) || !fixpos;
      const bool pinned_r = last || !free_o;
      lz[o] = (pinned_r ? LamR[o] : R(0)) + cR[o] + (has_right ? nc : R(0));
      if (first) az0[o] += cL[o] + LamL[o];
    }
  }

  // parameter adjoints: the three lanes of a segment add theirs in axis order
  SA(a, 0) = aiT;
  SA(a, 1) = ahd;
  __syncthreads();
  if (core) {
    R* ao = A.adj_out;
#pragma unroll
    for (int o = 0; o < S; ++o) {
      ao[(F_ZR + a * S + o) * ld + seg] = lz[o];
      ao[(F_UL + a * S + o) * ld + seg] = luL[o];
      ao[(F_UR + a * S + o) * ld + seg] = luR[o];
      if (first) A.acc_z0[(a * S + o) * ld + seg] += az0[o];
    }
    if constexpr (BOX) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        ao[(F_YH + a * M + s) * ld + seg] = LYH[s];
        ao[(F_YL + a * M + s) * ld + seg] = LYL[s];
      }
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) ao[(F_G + a * M + s) * ld + seg] = LG[s];
    }
    if (a == 0) {
      A.acc_iT[seg] += (SA(0, 0) + SA(1, 0)) + SA(2, 0);
      A.acc_hd[seg] += (SA(0, 1) + SA(1, 1)) + SA(2, 1);
    }
  }
}

// LB: the largest tile (in segments) of the instance; a launch runs 3 W threads.
template <typename R, int LB>
hipError_t dispatch_adjoint(const Variant& v, const AdjArgs<R>& a, int n_tiles, hipStream_t st) {
  if (a.W <= 0 || a.W > LB || (a.W & 63) != 0 || n_tiles <= 0 || a.steps <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(3 * a.W);
  const size_t lds = adjoint_lds_bytes(v, sizeof(R), LB);
#define TOP_ADJ_CASE(P_, S_, B_, V_)                                                              \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {                      \
    hipError_t e_ = hipFuncSetAttribute((const void*)(adjoint_kernel<R, P_, S_, B_, V_, 3 * LB>), \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);    \
    if (e_ != hipSuccess) return e_;                                                             \
    hipLaunchKernelGGL((adjoint_kernel<R, P_, S_, B_, V_, 3 * LB>), grid, block, lds, st, a);      \
    return hipGetLastError();                                                                    \
  }
#define TOP_ADJ_PS(P_, S_)                                                                         \
  TOP_ADJ_CASE(P_, S_, true, true)                                                                 \
  TOP_ADJ_CASE(P_, S_, true, false)                                                                \
  TOP_ADJ_CASE(P_, S_, false, true)                                                                \
  TOP_ADJ_CASE(P_, S_, false, false)
  TOP_ADJ_PS(3, 3)
  TOP_ADJ_PS(3, 4)
  TOP_ADJ_PS(4, 4)
  TOP_ADJ_PS(4, 5)
#undef TOP_ADJ_PS
#undef TOP_ADJ_CASE
  return hipErrorInvalidValue;
}

}  // namespace top
