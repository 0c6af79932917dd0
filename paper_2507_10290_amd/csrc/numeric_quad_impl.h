// NumericSolve sweep with four lanes per segment: lane 4 l + a holds axis a of the tile's segment l
// (a = 0, 1, 2) and lane 4 l + 3 is a spare that carries zeros.  The local update is the one of
// numeric_impl.h (Sec. III-C.3, eq. general_constraint_aug, minimised by L-BFGS with a backtracking
// Armijo search), split by axis: the cost, the consensus rows and the box rows of the augmented
// Lagrangian are sums of per-axis terms, and only the velocity bound couples the axes, through |v_s|
// at each sample.  Every sum over the 18 (or 24) unknowns -- the value of L, the dot products of the
// two-loop recursion, the line-search slope, s^T y and y^T y -- is a per-lane partial sum reduced
// over the quad with two DPP exchanges, which leaves the same bits on all four lanes, so the quad's
// lanes take every branch of the line search and the history update together.  Each lane keeps its
// axis' slice of the L-BFGS history in registers: no LDS beyond the knot exchange, and a third of
// the registers of the one-lane kernel, which at 64-segment tiles held one wave per SIMD.
//
// The knot exchange is the lane-per-axis one (knot_update per order): the neighbour segments' end
// states come from lanes 4 away, or through LDS at wave edges (16 segments per wave).
#pragma once

#include "numeric_impl.h"

namespace top {

// Largest tile (segments) of this form, 4 W threads per workgroup: 128 in float32 (two waves per
// SIMD), 64 in float64 (one wave per SIMD, whose doubled registers then need no spills).
constexpr int kNumQuadMaxWaves = 4 * kNumQuadTileMax / 64;

// x summed over the four lanes of its quad (every lane of the quad must be active).  The butterfly
// adds (x0 + x1) + (x2 + x3) on every lane, so all four hold the same bits.
__device__ __forceinline__ float quad_sum(float x) {
  const float y = x + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
  return y + __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, y), 0x4E, 0xF, 0xF, false));
}
__device__ __forceinline__ double quad_swap(double x, int ctrl_is_b1) {
  const long long b = __builtin_bit_cast(long long, x);
  int lo = (int)(b & 0xFFFFFFFFll), hi = (int)(b >> 32);
  if (ctrl_is_b1) {
    lo = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else {
    lo = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  }
  return __builtin_bit_cast(double, ((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double quad_sum(double x) {
  const double y = x + quad_swap(x, 1);
  return y + quad_swap(y, 0);
}

template <typename R, int P, int S, bool BOX>
struct NumQuadLane {
  static constexpr int N = 2 * P;
  static constexpr int M = kSamples;
  static constexpr int MB = BOX ? M : 1;
  // state of this lane's axis, and the segment's multipliers (the same on the quad's lanes)
  R zL[S], zR[S], uL[S], uR[S], yh[MB], yl[MB], w[M], cw[N];
  // constants
  R iT, iTp[N], Tp[N], qs, rho, vm, lo, hi;
  bool first, last, has_left, has_right, fixpos;
};

// h of the velocity bound at one sample from this lane's velocity component v, and dh/dv for it.
template <int VN, typename R>
__device__ __forceinline__ R quad_vel_excess(R v, R vm, R& dh) {
  if constexpr (VN == 2) {
    dh = R(2) * v;
    return quad_sum(v * v) - vm * vm;
  } else {
    static_assert(VN == 4, "the velocity bound is the 2- or the 4-norm");
    const R v2 = v * v;
    const R n4 = sqrt(sqrt(quad_sum(v2 * v2)));
    const R i3 = n4 > R(0) ? R(1) / (n4 * n4 * n4) : R(0);
    dh = v * v2 * i3;
    return n4 - vm;
  }
}

// L at the monomial coefficients (this lane's axis: x), the same value on the quad's lanes, and
// this axis' part of dL/dx when GRAD.
template <bool GRAD, int VN, typename R, int P, int S, bool BOX>
__device__ __forceinline__ R quad_objective(const NumQuadLane<R, P, S, BOX>& L, const R (&x)[2 * P], R (&gx)[2 * P]) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  R ct[N], gt[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    ct[j] = x[j] * L.Tp[j];
    gt[j] = R(0);
  }
  R val = R(0);
  const R hr = R(0.5) * L.rho;
  // cost T^(1-2p) c~^T Q(1) c~
  static_for<P, N>([&](auto j) {
    R qc = R(0);
    static_for<P, N>([&](auto k) { qc += R(cgram(P, j, k)) * ct[k]; });
    val += L.qs * ct[j] * qc;
    if constexpr (GRAD) gt[j] += R(2) * L.qs * qc;
  });
  // consensus rows: left o! T^-o c~_o, right T^-o f_o . c~, against z - u
  static_for<0, S>([&](auto o) {
    constexpr R kf = R(cfact(o));
    if (o < P || !L.first) {
      const R rl = kf * L.iTp[o] * ct[o] - (L.zL[o] - L.uL[o]);
      val += hr * rl * rl;
      if constexpr (GRAD) gt[o] += L.rho * rl * kf * L.iTp[o];
    }
    if (o < P || !L.last) {
      R xr = R(0);
      static_for<o, N>([&](auto j) { xr += R(cfall(o, j)) * ct[j]; });
      const R rr = L.iTp[o] * xr - (L.zR[o] - L.uR[o]);
      val += hr * rr * rr;
      if constexpr (GRAD) {
        const R t = L.rho * rr * L.iTp[o];
        static_for<o, N>([&](auto j) { gt[j] += t * R(cfall(o, j)); });
      }
    }
  });
  // box rows against b - |y|
  if constexpr (BOX) {
    static_for<0, M>([&](auto s) {
      R pv = R(0);
      static_for<0, N>([&](auto j) { pv += R(cpos(s, j)) * ct[j]; });
      const R ru = pv - L.hi + fabs(L.yh[s]);
      const R rl = L.lo - pv + fabs(L.yl[s]);
      val += hr * (ru * ru + rl * rl);
      if constexpr (GRAD) {
        const R t = L.rho * (ru - rl);
        static_for<0, N>([&](auto j) { gt[j] += t * R(cpos(s, j)); });
      }
    });
  }
  R f = quad_sum(val);
  // velocity: rho/2 (g_s + w_s)^2, g_s = max{0, h_s}^2
  static_for<0, M>([&](auto s) {
    R acc = R(0);
    static_for<1, N>([&](auto j) { acc += R(cvel(s, j)) * ct[j]; });
    R dh;
    const R h = quad_vel_excess<VN>(acc * L.iT, L.vm, dh);
    const R hp = h > R(0) ? h : R(0);
    const R e = hp * hp + L.w[s];
    f += hr * e * e;
    if constexpr (GRAD) {
      const R ta = L.rho * e * R(2) * hp * L.iT * dh;
      static_for<1, N>([&](auto j) { gt[j] += ta * R(cvel(s, j)); });
    }
  });
  if constexpr (GRAD) {
#pragma unroll
    for (int j = 0; j < N; ++j) gx[j] = gt[j] * L.Tp[j];
  }
  return f;
}

template <typename R, int N>
__device__ __forceinline__ R quad_dot(const R (&a)[N], const R (&b)[N]) {
  R s = R(0);
#pragma unroll
  for (int j = 0; j < N; ++j) s += a[j] * b[j];
  return quad_sum(s);
}

// Local update: `inner` L-BFGS iterations on L from the segment's previous c; returns this axis' c~.
// The history is kept newest last (slot m - 1) and shifted down when a pair is added, so that every
// slot index is a compile-time constant and the history stays in registers.
template <int VN, typename R, int P, int S, bool BOX>
__device__ __forceinline__ void quad_local_solve(const NumQuadLane<R, P, S, BOX>& L, int inner, R (&ct)[2 * P]) {
  constexpr int N = 2 * P;
  constexpr int m = kLbfgsMem;
  R Sh[m][N] = {}, Yh[m][N] = {}, Rh[m] = {};
  R x[N], g[N];
#pragma unroll
  for (int j = 0; j < N; ++j) x[j] = L.cw[j] * L.iTp[j];
  R f = quad_objective<true, VN>(L, x, g);
  int count = 0;
  R gamma = R(1);
  for (int it = 0; it < inner; ++it) {
    // two-loop recursion: d = -H g, over the count newest pairs (pair i back from the newest in
    // slot m - 1 - i)
    R q[N], alpha[m];
#pragma unroll
    for (int j = 0; j < N; ++j) q[j] = g[j];
#pragma unroll
    for (int i = 0; i < m; ++i) {
      alpha[i] = R(0);
      if (i < count) {
        const int k = m - 1 - i;
        R p = R(0);
#pragma unroll
        for (int j = 0; j < N; ++j) p += Sh[k][j] * q[j];
        const R ai = Rh[k] * quad_sum(p);
        alpha[i] = ai;
#pragma unroll
        for (int j = 0; j < N; ++j) q[j] -= ai * Yh[k][j];
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) q[j] *= gamma;
#pragma unroll
    for (int i = m - 1; i >= 0; --i) {
      if (i < count) {
        const int k = m - 1 - i;
        R p = R(0);
#pragma unroll
        for (int j = 0; j < N; ++j) p += Yh[k][j] * q[j];
        const R bi = Rh[k] * quad_sum(p);
#pragma unroll
        for (int j = 0; j < N; ++j) q[j] += Sh[k][j] * (alpha[i] - bi);
      }
    }
    R d[N];
#pragma unroll
    for (int j = 0; j < N; ++j) d[j] = -q[j];
    const R slope = quad_dot(g, d);
    // backtracking line search (quads that have accepted only wait for the others)
    R step = R(0), al = R(1);
    bool acc = false;
    for (int t = 0; t < kLsTrials; ++t) {
      if (!acc) {
        R xt[N], dummy[N];
#pragma unroll
        for (int j = 0; j < N; ++j) xt[j] = x[j] + al * d[j];
        const R ft = quad_objective<false, VN>(L, xt, dummy);
        if (ft <= f + R(1e-4) * al * slope) {
          step = al;
          acc = true;
        }
      }
      al *= R(0.5);
      if (__all(acc)) break;
    }
    if (step > R(0)) {
      R xn[N], gn[N];
#pragma unroll
      for (int j = 0; j < N; ++j) xn[j] = x[j] + step * d[j];
      const R fn = quad_objective<true, VN>(L, xn, gn);
      R sy = R(0), yy = R(0);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const R sv = xn[j] - x[j], yv = gn[j] - g[j];
        sy += sv * yv;
        yy += yv * yv;
      }
      sy = quad_sum(sy);
      yy = quad_sum(yy);
      if (sy > R(0)) {
#pragma unroll
        for (int k = 0; k + 1 < m; ++k) {
#pragma unroll
          for (int j = 0; j < N; ++j) {
            Sh[k][j] = Sh[k + 1][j];
            Yh[k][j] = Yh[k + 1][j];
          }
          Rh[k] = Rh[k + 1];
        }
#pragma unroll
        for (int j = 0; j < N; ++j) {
          Sh[m - 1][j] = xn[j] - x[j];
          Yh[m - 1][j] = gn[j] - g[j];
        }
        Rh[m - 1] = R(1) / sy;
        count = count < m ? count + 1 : m;
        gamma = sy / yy;
      }
#pragma unroll
      for (int j = 0; j < N; ++j) {
        x[j] = xn[j];
        g[j] = gn[j];
      }
      f = fn;
    }
  }
#pragma unroll
  for (int j = 0; j < N; ++j) ct[j] = x[j] * L.Tp[j];
}

// Waves per SIMD the compiler must leave room for: three for the float32 quintic Euclidean-ball
// instances (168 registers, a few spills outside the L-BFGS loop; 7.4 against 8.0 ms on the 256
// batched trajectories at two waves, 8.9 ms at four), the register count's own otherwise.
template <typename R, int P, int VN>
constexpr int num_quad_min_waves() {
  return (sizeof(R) == 4 && P == 3 && VN == 2) ? 3 : 1;
}

template <typename R, int P, int S, bool BOX, int VN, int LB>
__global__ __launch_bounds__(LB) __attribute__((amdgpu_waves_per_eu(num_quad_min_waves<R, P, VN>())))
void numeric_quad_kernel(SweepArgs<R> A) {
  using LT = NumQuadLane<R, P, S, BOX>;
  constexpr int N = LT::N;
  constexpr int M = LT::M;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_W = 9 * S + (BOX ? 6 * M : 0);
  constexpr int F_C = F_W + M;

  __shared__ R xr_sh[2][kNumQuadMaxWaves][4][S];   // end states to the right neighbour (wave edges)
  __shared__ R xl_sh[2][kNumQuadMaxWaves][4][S];   // start states to the left neighbour

  const int W = A.W;
  const int a = threadIdx.x & 3;           // axis of this lane (3: the spare)
  const int lane = threadIdx.x >> 2;       // segment lane within the tile
  const int64_t base = (int64_t)blockIdx.x * W;
  const int64_t ld = A.k.ld;
  const int32_t ent = A.lane_seg[base + lane];
  const bool active = ent >= 0;            // the quad has a segment
  const bool axl = active && a < 3;        // ... and this lane one of its axes
  const bool core = axl && !(ent & kHaloBit);
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

  // ---- per-segment constants (an idle quad gets a harmless unit segment)
  L.iT = active ? A.k.iT[seg] : R(1);
  const R T = R(1) / L.iT;
  L.iTp[0] = R(1);
  L.Tp[0] = R(1);
#pragma unroll
  for (int j = 1; j < N; ++j) {
    L.iTp[j] = L.iTp[j - 1] * L.iT;
    L.Tp[j] = L.Tp[j - 1] * T;
  }
  L.qs = L.iTp[2 * P - 1];
  L.rho = active ? (R)A.k.rho[seg] : R(1);
  L.vm = active ? A.k.vmax[seg] : R(1);
  L.lo = (BOX && axl) ? A.k.lo[a * ld + seg] : R(0);
  L.hi = (BOX && axl) ? A.k.hi[a * ld + seg] : R(0);

  // ---- state of this axis (zeros on the spare lane), and the segment's multipliers
  const R* in = A.st_in;
  const int tr = active ? A.k.traj[seg] : 0;
#pragma unroll
  for (int o = 0; o < S; ++o) {
    const int f = a * S + o;
    L.zR[o] = axl ? in[(F_ZR + f) * ld + seg] : R(0);
    L.uL[o] = axl ? in[(F_UL + f) * ld + seg] : R(0);
    L.uR[o] = axl ? in[(F_UR + f) * ld + seg] : R(0);
    L.zL[o] = !axl ? R(0) : L.first ? A.k.bcL[((int64_t)tr * 3 + a) * S + o] : in[(F_ZR + f) * ld + seg - 1];
  }
#pragma unroll
  for (int s = 0; s < LT::MB; ++s) {
    L.yh[s] = (BOX && axl) ? in[(F_YH + a * M + s) * ld + seg] : R(0);
    L.yl[s] = (BOX && axl) ? in[(F_YL + a * M + s) * ld + seg] : R(0);
  }
#pragma unroll
  for (int j = 0; j < N; ++j) L.cw[j] = axl ? in[(F_C + a * N + j) * ld + seg] : R(0);
#pragma unroll
  for (int s = 0; s < M; ++s) L.w[s] = active ? in[(F_W + s) * ld + seg] : R(0);

  const int wl = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (4 * W) >> 6;
  if (__ballot(active) == 0) {   // a wave without segments keeps the barrier count
    for (int it = 0; it < A.iters; ++it) __syncthreads();
    return;
  }
  R cfin[N], zfin[S];
  auto sweep = [&](auto fin_tag, int buf) {
    constexpr bool FIN = decltype(fin_tag)::value;
    R c[N];
    quad_local_solve<VN>(L, A.inner, c);
    // multipliers of g_s = 0
    static_for<0, M>([&](auto s) {
      R acc = R(0);
      static_for<1, N>([&](auto j) { acc += R(cvel(s, j)) * c[j]; });
      R dh;
      const R h = quad_vel_excess<VN>(acc * L.iT, L.vm, dh);
      const R hp = h > R(0) ? h : R(0);
      L.w[s] += hp * hp;
    });
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        R pv = R(0);
        static_for<0, N>([&](auto j) { pv += R(cpos(s, j)) * c[j]; });
        L.yh[s] = pv - L.hi + relu(L.yh[s]);
        L.yl[s] = L.lo - pv + relu(L.yl[s]);
      });
    }
    R xL[S], xR[S];
    static_for<0, S>([&](auto o) {
      constexpr R kf = R(cfact(o));
      xL[o] = kf * c[o] * L.iTp[o];
      R acc = R(0);
      static_for<o, N>([&](auto j) { acc += R(cfall(o, j)) * c[j]; });
      xR[o] = acc * L.iTp[o];
    });
#pragma unroll
    for (int j = 0; j < N; ++j) {
      L.cw[j] = c[j];
      if constexpr (FIN) cfin[j] = c[j];
    }
    // ---- knot exchange: the neighbour segments' quads are 4 lanes away, or across a wave edge
    if (wl >= 60) {
#pragma unroll
      for (int o = 0; o < S; ++o) xr_sh[buf][wid][a][o] = xR[o];
    }
    if (wl < 4) {
#pragma unroll
      for (int o = 0; o < S; ++o) xl_sh[buf][wid][a][o] = xL[o];
    }
    __syncthreads();
#pragma unroll
    for (int o = 0; o < S; ++o) {
      R xp = __shfl_up(xR[o], 4);
      R xn = __shfl_down(xL[o], 4);
      if (wl < 4 && wid > 0) xp = xr_sh[buf][wid - 1][a][o];
      if (wl >= 60 && wid < nw - 1) xn = xl_sh[buf][wid + 1][a][o];
      knot_update<FIN, P>(o, xL[o], xR[o], xp, xn, L.has_left, L.has_right, L.first, L.last, L.fixpos, L.zL[o],
                          L.zR[o], L.uL[o], L.uR[o], zfin[o]);
    }
  };
  const int n_plain = A.final_out ? A.iters - 1 : A.iters;
  int it = 0;
  for (; it < n_plain; ++it) sweep(std::false_type{}, it & 1);
  if (A.final_out && A.iters > 0) {
    sweep(std::true_type{}, it & 1);
    if (core) {
#pragma unroll
      for (int j = 0; j < N; ++j) A.c_out[(a * N + j) * ld + seg] = cfin[j];
#pragma unroll
      for (int o = 0; o < S; ++o) A.zold_out[(a * S + o) * ld + seg] = zfin[o];
    }
  }
  if (core) {
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
#pragma unroll
    for (int j = 0; j < N; ++j) out[(F_C + a * N + j) * ld + seg] = L.cw[j];
    if (a == 0) {
#pragma unroll
      for (int s = 0; s < M; ++s) out[(F_W + s) * ld + seg] = L.w[s];
    }
  }
}

template <typename R>
hipError_t dispatch_numeric_quad(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  if (!v.num || !v.vel || v.faces || v.s != v.p || a.rec != nullptr || a.done != nullptr || a.inner < 0)
    return hipErrorInvalidValue;
  constexpr int kMax = num_quad_max_tile(sizeof(R) == 4 ? 0 : 1);
  if (a.W <= 0 || a.W > kMax || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(4 * a.W);
#define TOP_NUMQ_CASE(P_, B_, VN_)                                                          \
  if (v.p == P_ && (v.box != 0) == B_ && v.vn == VN_) {                                   \
    hipLaunchKernelGGL((numeric_quad_kernel<R, P_, P_, B_, VN_, 4 * kMax>), grid, block, 0, st, a); \
    return hipGetLastError();                                                             \
  }
  TOP_NUMQ_CASE(3, true, 2) TOP_NUMQ_CASE(3, false, 2)
  TOP_NUMQ_CASE(4, true, 2) TOP_NUMQ_CASE(4, false, 2)
  TOP_NUMQ_CASE(3, true, 4) TOP_NUMQ_CASE(3, false, 4)
  TOP_NUMQ_CASE(4, true, 4) TOP_NUMQ_CASE(4, false, 4)
#undef TOP_NUMQ_CASE
  return hipErrorInvalidValue;
}

}  // namespace top
