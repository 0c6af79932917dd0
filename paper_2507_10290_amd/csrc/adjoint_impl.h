// Reverse-mode derivative of the sweep (the update rules of Sec. III-D.1 as
// computed by sweep_impl.h, folded slack/dual form), resident form.
//
// One launch runs `steps` reverse steps of consecutive forward sweeps.  The
// forward state before each of those sweeps is read from a block buffer that
// a replay of the block has filled; the adjoint state stays in registers.
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

  // Wave-boundary values.  E1 and E2 use separate arrays: a wave may write its E2 values while a
  // slower wave still reads E1 values of the same step (no barrier lies between those).
  __shared__ R sh_r[2][kMaxWaves][6 * S];   // E1, to the right neighbour: lz, luR
  __shared__ R sh_l[2][kMaxWaves][3 * S];   // E1, to the left neighbour: luL
  __shared__ R sh_c[2][kMaxWaves][3 * S];   // E2, to the left neighbour: cL

  const int W = A.W;
  const int lane = threadIdx.x;
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
  if (__ballot(active) == 0) {
    for (int t = 0; t < A.steps; ++t) { __syncthreads(); __syncthreads(); }
    return;
  }

  R H[NH], Hd[NH];
#pragma unroll
  for (int h = 0; h < NH; ++h) {
    H[h] = active ? A.k.Hr[h * ld + seg] : R(0);
    Hd[h] = active ? A.Hd[h * ld + seg] : R(0);
  }
  const R iT = active ? A.k.iT[seg] : R(1);
  const R vm = (VEL && active) ? A.k.vmax[seg] : R(1);
  R lo[3], hi[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    lo[a] = (BOX && active) ? A.k.lo[a * ld + seg] : R(0);
    hi[a] = (BOX && active) ? A.k.hi[a * ld + seg] : R(0);
  }
  R iTp[N];
  iTp[0] = R(1);
#pragma unroll
  for (int o = 1; o < N; ++o) iTp[o] = iTp[o - 1] * iT;
  const int tr = active ? A.k.traj[seg] : 0;
  const R dc = (active && A.with_cost) ? (R)A.dcost[tr] : R(0);

  // adjoint state: knot and u adjoints in registers; the box and velocity pair adjoints (9M values)
  // in this lane's own LDS column, which keeps the register set of the kernel small
  extern __shared__ double adj_lds_raw[];
  R* ly = reinterpret_cast<R*>(adj_lds_raw);
  auto LYH = [&](int a, int s) -> R& { return ly[(a * M + s) * W + lane]; };
  auto LYL = [&](int a, int s) -> R& { return ly[(3 * M + a * M + s) * W + lane]; };
  auto LG = [&](int a, int s) -> R& { return ly[((BOX ? 6 * M : 0) + a * M + s) * W + lane]; };
  R lz[3][S], luL[3][S], luR[3][S];
  const R* ai = A.adj_in;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 0; o < S; ++o) {
      lz[a][o] = active ? ai[(F_ZR + a * S + o) * ld + seg] : R(0);
      luL[a][o] = active ? ai[(F_UL + a * S + o) * ld + seg] : R(0);
      luR[a][o] = active ? ai[(F_UR + a * S + o) * ld + seg] : R(0);
    }
    if constexpr (BOX) {
      for (int s = 0; s < M; ++s) {
        LYH(a, s) = active ? ai[(F_YH + a * M + s) * ld + seg] : R(0);
        LYL(a, s) = active ? ai[(F_YL + a * M + s) * ld + seg] : R(0);
      }
    }
    if constexpr (VEL) {
      for (int s = 0; s < M; ++s) LG(a, s) = active ? ai[(F_G + a * M + s) * ld + seg] : R(0);
    }
  }
  R aiT = R(0), ahd = R(0);
  R az0[3][S];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int o = 0; o < S; ++o) az0[a][o] = R(0);

  for (int t = A.steps - 1; t >= 0; --t) {
    const R* st = (t == 0 && A.blk0 != nullptr) ? A.blk0 : A.blk + (int64_t)t * A.slot;
    const bool cost_step = A.with_cost && (t == A.steps - 1);
    const int buf = t & 1;

    // ---- E1: adjoints of the new knot values.  Lam_k = lz(i) - luR(i) - luL(i+1) at an
    // interior knot k between segments i and i+1; both lanes form it with the same operations.
    if (wl == 63) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o < S; ++o) {
          sh_r[buf][wid][a * S + o] = lz[a][o];
          sh_r[buf][wid][3 * S + a * S + o] = luR[a][o];
        }
    }
    if (wl == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o < S; ++o) sh_l[buf][wid][a * S + o] = luL[a][o];
    }
    __syncthreads();
    R LamL[3][S], LamR[3][S];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        R pz = __shfl_up(lz[a][o], 1);
        R pu = __shfl_up(luR[a][o], 1);
        R nu = __shfl_down(luL[a][o], 1);
        if (wl == 0 && wid > 0) { pz = sh_r[buf][wid - 1][a * S + o]; pu = sh_r[buf][wid - 1][3 * S + a * S + o]; }
        if (wl == 63 && wid < nw - 1) nu = sh_l[buf][wid + 1][a * S + o];
        const bool mR = (o < P) || !last;
        const bool mL = (o < P) || !first;
        LamR[a][o] = has_right ? (lz[a][o] - luR[a][o]) - nu : (lz[a][o] - (mR ? luR[a][o] : R(0)));
        LamL[a][o] = has_left ? (pz - pu) - luL[a][o] : -(mL ? luL[a][o] : R(0));
      }
    }

    // ---- forward state before this sweep: only the velocity factors need all three axes up front;
    // each axis' values are read from the block buffer inside the axis loop, which keeps the
    // live register set small (the float64 instance would otherwise spill heavily).
    R f[MV], rs2[MV], lf[MV];
    bool outside[MV];
#pragma unroll
    for (int s = 0; s < MV; ++s) {
      lf[s] = R(0);
      if constexpr (VEL) {
        R gs[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gs[a] = active ? st[(F_G + a * M + s) * ld + seg] : R(0);
        const R n2 = gs[0] * gs[0] + gs[1] * gs[1] + gs[2] * gs[2];
        const R q = vm * inv_sqrt<R>(n2);
        outside[s] = q < R(1);
        f[s] = fmin(R(1), q);
        rs2[s] = outside[s] ? R(1) / n2 : R(0);
      } else {
        f[s] = R(1);
        rs2[s] = R(0);
        outside[s] = false;
      }
    }

    R cL[3][S], cR[3][S];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R zL[S], zR[S], uL[S], uR[S], yh[MB], yl[MB], g[MV];
#pragma unroll
      for (int o = 0; o < S; ++o) {
        const int fo = a * S + o;
        zR[o] = active ? st[(F_ZR + fo) * ld + seg] : R(0);
        uL[o] = active ? st[(F_UL + fo) * ld + seg] : R(0);
        uR[o] = active ? st[(F_UR + fo) * ld + seg] : R(0);
        zL[o] = !active ? R(0)
              : first ? A.k.bcL[((int64_t)tr * 3 + a) * S + o]
                      : st[(F_ZR + fo) * ld + seg - 1];
      }
#pragma unroll
      for (int s = 0; s < MB; ++s) {
        yh[s] = (BOX && active) ? st[(F_YH + a * M + s) * ld + seg] : R(0);
        yl[s] = (BOX && active) ? st[(F_YL + a * M + s) * ld + seg] : R(0);
      }
#pragma unroll
      for (int s = 0; s < MV; ++s) g[s] = (VEL && active) ? st[(F_G + a * M + s) * ld + seg] : R(0);
      // recompute r~ and c of this axis exactly as the forward sweep does
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
        const R hl = hi[a] + lo[a];
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
        static_for<0, N>([&](auto j) { acc += H[tri(N, i, j)] * r[j]; });
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
        R lxl = mL ? luL[a][o] : R(0);
        if (!first && free_o) lxl += R(0.5) * LamL[a][o];
        R lxr = mR ? luR[a][o] : R(0);
        if (!last && free_o) lxr += R(0.5) * LamR[a][o];
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
          const R d = LYH(a, s) - LYL(a, s);
          static_for<0, N>([&](auto j) {
            constexpr R k = R(cpos(s, j));
            lc[j] += k * d;
          });
        });
      }
      if constexpr (VEL) {
        static_for<0, M>([&](auto s) {
          R dv = R(0);
          const R t_ = iT * LG(a, s);
          static_for<1, N>([&](auto j) {
            constexpr R k = R(cvel(s, j));
            dv += k * c[j];
            lc[j] += k * t_;
          });
          aiT += LG(a, s) * dv;
          lf[s] -= LG(a, s) * g[s];   // from g' = vv + (1 - f) g
        });
      }
      if (cost_step) {
        // J = T^(1-2p) c^T Q(1) c
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
          LYH(a, s) = yh[s] > R(0) ? LYH(a, s) : R(0);
          LYL(a, s) = yl[s] > R(0) ? LYL(a, s) : R(0);
        }
      }
      if constexpr (VEL) {
#pragma unroll
        for (int s = 0; s < M; ++s) LG(a, s) = (R(1) - f[s]) * LG(a, s);
      }

      // ---- through the local solve: lr = (rho Htilde^-1) lc; T-derivative of the matrix
      R lr[N];
      static_for<0, N>([&](auto i) {
        R acc = R(0), hr = R(0);
        static_for<0, N>([&](auto j) {
          acc += H[tri(N, i, j)] * lc[j];
          hr += Hd[tri(N, i, j)] * r[j];
        });
        lr[i] = acc;
        ahd += lc[i] * hr;
      });

      // ---- through r~
      static_for<0, S>([&](auto o) {
        constexpr R kf = R(cfact(o));
        const R cl = kf * iTp[o] * lr[o];
        cL[a][o] = cl;
        R fl_ = R(0);
        static_for<o, N>([&](auto j) {
          constexpr R k = R(cfall(o, j));
          fl_ += k * lr[j];
        });
        const R cr = iTp[o] * fl_;
        cR[a][o] = cr;
        if constexpr (o > 0) {
          aiT += R(o) * iTp[o - 1] * (kf * (zL[o] - uL[o]) * lr[o] + (zR[o] - uR[o]) * fl_);
        }
        luL[a][o] -= cl;
        luR[a][o] -= cr;
      });
      if constexpr (BOX) {
        static_for<0, M>([&](auto s) {
          R lb = R(0);
          static_for<0, N>([&](auto j) {
            constexpr R k = R(cpos(s, j));
            lb += k * lr[j];
          });
          LYH(a, s) -= sgn(yh[s]) * lb;
          LYL(a, s) += sgn(yl[s]) * lb;
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
          LG(a, s) += iT * (R(2) * f[s] - R(1)) * lt;
          aiT += (R(2) * f[s] - R(1)) * g[s] * lt;
        });
      }
    }
    // ---- through f = min(1, vmax/||g||): outside the ball df/dg = -f g / ||g||^2
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        const R w = outside[s] ? -lf[s] * f[s] * rs2[s] : R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a) LG(a, s) += w * (active ? st[(F_G + a * M + s) * ld + seg] : R(0));
      }
    }

    // ---- E2: start-knot contributions cL go to the owner of that knot (left neighbour)
    if (wl == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int o = 0; o < S; ++o) sh_c[buf][wid][a * S + o] = cL[a][o];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        R nc = __shfl_down(cL[a][o], 1);
        if (wl == 63 && wid < nw - 1) nc = sh_c[buf][wid + 1][a * S + o];
        const bool free_o = (o > 0) || !fixpos;
        const bool pinned_r = last || !free_o;
        lz[a][o] = (pinned_r ? LamR[a][o] : R(0)) + cR[a][o] + (has_right ? nc : R(0));
        if (first) az0[a][o] += cL[a][o] + LamL[a][o];
      }
    }
  }

  if (core) {
    R* ao = A.adj_out;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int o = 0; o < S; ++o) {
        ao[(F_ZR + a * S + o) * ld + seg] = lz[a][o];
        ao[(F_UL + a * S + o) * ld + seg] = luL[a][o];
        ao[(F_UR + a * S + o) * ld + seg] = luR[a][o];
        if (first) A.acc_z0[(a * S + o) * ld + seg] += az0[a][o];
      }
      if constexpr (BOX) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
          ao[(F_YH + a * M + s) * ld + seg] = LYH(a, s);
          ao[(F_YL + a * M + s) * ld + seg] = LYL(a, s);
        }
      }
      if constexpr (VEL) {
#pragma unroll
        for (int s = 0; s < M; ++s) ao[(F_G + a * M + s) * ld + seg] = LG(a, s);
      }
    }
    A.acc_iT[seg] += aiT;
    A.acc_hd[seg] += ahd;
  }
}

template <typename R, int LB3, int LB4>
hipError_t dispatch_adjoint(const Variant& v, const AdjArgs<R>& a, int n_tiles, hipStream_t st) {
  const int lb = (v.p == 3) ? LB3 : LB4;
  if (a.W <= 0 || a.W > lb || (a.W & 63) != 0 || n_tiles <= 0 || a.steps <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(a.W);
  const size_t lds = adjoint_lds_bytes(v, sizeof(R), a.W);
#define TOP_ADJ_CASE(P_, S_, B_, V_, LB_)                                                     \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_) {                 \
    hipError_t e_ = hipFuncSetAttribute((const void*)(adjoint_kernel<R, P_, S_, B_, V_, LB_>), \
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e_ != hipSuccess) return e_;                                                        \
    hipLaunchKernelGGL((adjoint_kernel<R, P_, S_, B_, V_, LB_>), grid, block, lds, st, a);   \
    return hipGetLastError();                                                               \
  }
#define TOP_ADJ_PS(P_, S_, LB_)                                                               \
  TOP_ADJ_CASE(P_, S_, true, true, LB_)                                                       \
  TOP_ADJ_CASE(P_, S_, true, false, LB_)                                                      \
  TOP_ADJ_CASE(P_, S_, false, true, LB_)                                                      \
  TOP_ADJ_CASE(P_, S_, false, false, LB_)
  TOP_ADJ_PS(3, 3, LB3)
  TOP_ADJ_PS(3, 4, LB3)
  TOP_ADJ_PS(4, 4, LB4)
  TOP_ADJ_PS(4, 5, LB4)
#undef TOP_ADJ_PS
#undef TOP_ADJ_CASE
  return hipErrorInvalidValue;
}

}  // namespace top
