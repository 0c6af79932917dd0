// NumericSolve sweep (Sec. III-C.3, general inequality constraints; the NumericSolve branch of
// Algorithm 1), resident form: same tiles, launch protocol and knot exchange as the closed-form
// kernel of sweep_impl.h.
//
// The velocity bound is a general convex inequality h_s(c) <= 0 turned into the equality
// g_s = max{0, h_s}^2 = 0 (eq. componentwise maximum) with a scaled multiplier w_s, where h_s is
// |v_s|^2 - vmax^2 (VN = 2, the Euclidean ball of Sec. III-C.2) or ||v_s||_4 - vmax (VN = 4, the l4
// ball, which has no closed-form projection); the box rows keep their folded slack/dual pairs.  The local update minimises the segment's augmented
// Lagrangian (eq. general_constraint_aug, scaled form)
//   L(c) = c^T Q~ c + rho/2 |M~ c - z~ + u|^2 + rho/2 |A^o c - (b - |y|)|^2 + rho/2 sum_s (g_s + w_s)^2
// by `inner` L-BFGS iterations (two-loop recursion, memory kLbfgsMem, H0 = gamma I with gamma =
// s^T y / y^T y of the newest pair, pairs with s^T y <= 0 dropped) from the previous c, with a
// backtracking Armijo search from step 1 (c1 = 1e-4, halving, at most kLsTrials steps; no move if
// none is accepted).  L-BFGS runs in the monomial coefficients c_j = c~_j / T^j, the variables the
// method is stated in (it is not invariant to rescaling them); L and its gradient are evaluated in
// the normalised basis and mapped by dL/dc_j = T^j dL/dc~_j.  The history lives in the lane's own
// column of dynamic LDS.  After the local solve: w_s += g_s(c), then the box pairs, the knots and u
// exactly as in the closed form.
#pragma once

#include "sweep_impl.h"

namespace top {

constexpr int kLbfgsMem = 5;
constexpr int kLsTrials = 20;

template <typename R, int P, int S, bool BOX>
struct NumLane {
  static constexpr int N = 2 * P;
  static constexpr int M = kSamples;
  static constexpr int MB = BOX ? M : 1;
  // state
  R zL[3][S], zR[3][S], uL[3][S], uR[3][S], yh[3][MB], yl[3][MB], w[M], cw[3][N];
  // constants
  R iT, iTp[N], Tp[N], qs, rho, vm, lo[3], hi[3];
  bool first, last, has_left, has_right, fixpos;
};

// h of the velocity bound at one sample and dh/dv.
template <int VN, typename R>
__device__ __forceinline__ R vel_excess(const R (&v)[3], R vm, R (&dh)[3]) {
  if constexpr (VN == 2) {
#pragma unroll
    for (int a = 0; a < 3; ++a) dh[a] = R(2) * v[a];
    return v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - vm * vm;
  } else {
    static_assert(VN == 4, "the velocity bound is the 2- or the 4-norm");
    R v2[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) v2[a] = v[a] * v[a];
    const R n4 = sqrt(sqrt(v2[0] * v2[0] + v2[1] * v2[1] + v2[2] * v2[2]));
    const R i3 = n4 > R(0) ? R(1) / (n4 * n4 * n4) : R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) dh[a] = v[a] * v2[a] * i3;
    return n4 - vm;
  }
}

// L at the monomial coefficients x (and dL/dx when GRAD).
template <bool GRAD, int VN, typename R, int P, int S, bool BOX>
__device__ __forceinline__ R num_objective(const NumLane<R, P, S, BOX>& L, const R (&x)[3][2 * P],
                                           R (&gx)[3][2 * P]) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  R ct[3][N], gt[3][N];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      ct[a][j] = x[a][j] * L.Tp[j];
      gt[a][j] = R(0);
    }
  R val = R(0);
  const R hr = R(0.5) * L.rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // cost T^(1-2p) c~^T Q(1) c~
    static_for<P, N>([&](auto j) {
      R qc = R(0);
      static_for<P, N>([&](auto k) { qc += R(cgram(P, j, k)) * ct[a][k]; });
      val += L.qs * ct[a][j] * qc;
      if constexpr (GRAD) gt[a][j] += R(2) * L.qs * qc;
    });
    // consensus rows: left o! T^-o c~_o, right T^-o f_o . c~, against z - u
    static_for<0, S>([&](auto o) {
      constexpr R kf = R(cfact(o));
      if (o < P || !L.first) {
        const R rl = kf * L.iTp[o] * ct[a][o] - (L.zL[a][o] - L.uL[a][o]);
        val += hr * rl * rl;
        if constexpr (GRAD) gt[a][o] += L.rho * rl * kf * L.iTp[o];
      }
      if (o < P || !L.last) {
        R xr = R(0);
        static_for<o, N>([&](auto j) { xr += R(cfall(o, j)) * ct[a][j]; });
        const R rr = L.iTp[o] * xr - (L.zR[a][o] - L.uR[a][o]);
        val += hr * rr * rr;
        if constexpr (GRAD) {
          const R t = L.rho * rr * L.iTp[o];
          static_for<o, N>([&](auto j) { gt[a][j] += t * R(cfall(o, j)); });
        }
      }
    });
    // box rows against b - |y|
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        R pv = R(0);
        static_for<0, N>([&](auto j) { pv += R(cpos(s, j)) * ct[a][j]; });
        const R ru = pv - L.hi[a] + fabs(L.yh[a][s]);
        const R rl = L.lo[a] - pv + fabs(L.yl[a][s]);
        val += hr * (ru * ru + rl * rl);
        if constexpr (GRAD) {
          const R t = L.rho * (ru - rl);
          static_for<0, N>([&](auto j) { gt[a][j] += t * R(cpos(s, j)); });
        }
      });
    }
  }
  // velocity: rho/2 (g_s + w_s)^2, g_s = max{0, h_s}^2
  static_for<0, M>([&](auto s) {
    R v[3], dh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R acc = R(0);
      static_for<1, N>([&](auto j) { acc += R(cvel(s, j)) * ct[a][j]; });
      v[a] = acc * L.iT;
    }
    const R h = vel_excess<VN>(v, L.vm, dh);
    const R hp = h > R(0) ? h : R(0);
    const R e = hp * hp + L.w[s];
    val += hr * e * e;
    if constexpr (GRAD) {
      const R t = L.rho * e * R(2) * hp * L.iT;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const R ta = t * dh[a];
        static_for<1, N>([&](auto j) { gt[a][j] += ta * R(cvel(s, j)); });
      }
    }
  });
  if constexpr (GRAD) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < N; ++j) gx[a][j] = gt[a][j] * L.Tp[j];
  }
  return val;
}

template <typename R, int N>
__device__ __forceinline__ R dot3(const R (&a)[3][N], const R (&b)[3][N]) {
  R s = R(0);
#pragma unroll
  for (int q = 0; q < 3; ++q)
#pragma unroll
    for (int j = 0; j < N; ++j) s += a[q][j] * b[q][j];
  return s;
}

// Local update: `inner` L-BFGS iterations on L from the lane's previous c; returns c~ in ct.
// hist: this lane's LDS column, element (k) at hist[k * W + lane].
template <int VN, typename R, int P, int S, bool BOX>
__device__ __forceinline__ void num_local_solve(const NumLane<R, P, S, BOX>& L, int inner, R* hist, int W, int lane,
                                                R (&ct)[3][2 * P]) {
  constexpr int N = 2 * P;
  constexpr int NV = 3 * N;
  constexpr int m = kLbfgsMem;
  auto Sh = [&](int slot, int a, int j) -> R& { return hist[((slot * 2 + 0) * NV + a * N + j) * W + lane]; };
  auto Yh = [&](int slot, int a, int j) -> R& { return hist[((slot * 2 + 1) * NV + a * N + j) * W + lane]; };
  auto Rh = [&](int slot) -> R& { return hist[(2 * m * NV + slot) * W + lane]; };

  R x[3][N], g[3][N];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < N; ++j) x[a][j] = L.cw[a][j] * L.iTp[j];
  R f = num_objective<true, VN>(L, x, g);
  int head = m - 1, count = 0;
  R gamma = R(1);
  for (int it = 0; it < inner; ++it) {
    // two-loop recursion: d = -H g
    R q[3][N], alpha[m];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < N; ++j) q[a][j] = g[a][j];
#pragma unroll
    for (int i = 0; i < m; ++i) {
      alpha[i] = R(0);
      if (i < count) {
        const int slot = (head - i + m) % m;
        R sq = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) sq += Sh(slot, a, j) * q[a][j];
        const R ai = Rh(slot) * sq;
        alpha[i] = ai;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) q[a][j] -= ai * Yh(slot, a, j);
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < N; ++j) q[a][j] *= gamma;
#pragma unroll
    for (int i = m - 1; i >= 0; --i) {
      if (i < count) {
        const int slot = (head - i + m) % m;
        R yr = R(0);
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) yr += Yh(slot, a, j) * q[a][j];
        const R bi = Rh(slot) * yr;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) q[a][j] += Sh(slot, a, j) * (alpha[i] - bi);
      }
    }
    R d[3][N];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int j = 0; j < N; ++j) d[a][j] = -q[a][j];
    const R slope = dot3(g, d);
    // backtracking line search (lanes that have accepted only wait for the others)
    R step = R(0), al = R(1);
    bool acc = false;
    for (int t = 0; t < kLsTrials; ++t) {
      if (!acc) {
        R xt[3][N], dummy[3][N];
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) xt[a][j] = x[a][j] + al * d[a][j];
        const R ft = num_objective<false, VN>(L, xt, dummy);
        if (ft <= f + R(1e-4) * al * slope) {
          step = al;
          acc = true;
        }
      }
      al *= R(0.5);
      if (__all(acc)) break;
    }
    if (step > R(0)) {
      R xn[3][N], gn[3][N];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < N; ++j) xn[a][j] = x[a][j] + step * d[a][j];
      const R fn = num_objective<true, VN>(L, xn, gn);
      R sy = R(0), yy = R(0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const R sv = xn[a][j] - x[a][j], yv = gn[a][j] - g[a][j];
          sy += sv * yv;
          yy += yv * yv;
        }
      if (sy > R(0)) {
        head = (head + 1) % m;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int j = 0; j < N; ++j) {
            Sh(head, a, j) = xn[a][j] - x[a][j];
            Yh(head, a, j) = gn[a][j] - g[a][j];
          }
        Rh(head) = R(1) / sy;
        count = count < m ? count + 1 : m;
        gamma = sy / yy;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int j = 0; j < N; ++j) {
          x[a][j] = xn[a][j];
          g[a][j] = gn[a][j];
        }
      f = fn;
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int j = 0; j < N; ++j) ct[a][j] = x[a][j] * L.Tp[j];
}

template <bool FINAL, int VN, typename R, int P, int S, bool BOX>
__device__ __forceinline__ void num_sweep_once(NumLane<R, P, S, BOX>& L, int inner, R* hist, int W, int lane,
                                               R (*xr_sh)[3 * S], R (*xl_sh)[3 * S], int wl, int wid, int nw,
                                               R (&cfin)[3][2 * P], R (&zfin)[3][S]) {
  constexpr int N = 2 * P;
  constexpr int M = kSamples;
  R c[3][N];
  num_local_solve<VN>(L, inner, hist, W, lane, c);
  // multipliers of g_s = 0
  static_for<0, M>([&](auto s) {
    R v[3], dh[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      R acc = R(0);
      static_for<1, N>([&](auto j) { acc += R(cvel(s, j)) * c[a][j]; });
      v[a] = acc * L.iT;
    }
    const R h = vel_excess<VN>(v, L.vm, dh);
    const R hp = h > R(0) ? h : R(0);
    L.w[s] += hp * hp;
  });
  R xL[3][S], xR[3][S];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if constexpr (BOX) {
      static_for<0, M>([&](auto s) {
        R pv = R(0);
        static_for<0, N>([&](auto j) { pv += R(cpos(s, j)) * c[a][j]; });
        L.yh[a][s] = pv - L.hi[a] + relu(L.yh[a][s]);
        L.yl[a][s] = L.lo[a] - pv + relu(L.yl[a][s]);
      });
    }
    static_for<0, S>([&](auto o) {
      constexpr R kf = R(cfact(o));
      xL[a][o] = kf * c[a][o] * L.iTp[o];
      R acc = R(0);
      static_for<o, N>([&](auto j) { acc += R(cfall(o, j)) * c[a][j]; });
      xR[a][o] = acc * L.iTp[o];
    });
#pragma unroll
    for (int j = 0; j < N; ++j) {
      L.cw[a][j] = c[a][j];
      if constexpr (FINAL) cfin[a][j] = c[a][j];
    }
  }
  knot_exchange<FINAL, P, S>(L, xL, xR, xr_sh, xl_sh, wl, wid, nw, zfin);
}

// Dynamic LDS of the NumericSolve kernel: the L-BFGS history of every lane.
inline size_t numeric_lds_bytes(int p, size_t rsz, int W) {
  return (size_t)(2 * kLbfgsMem * 3 * 2 * p + kLbfgsMem) * rsz * (size_t)W;
}

template <typename R, int P, int S, bool BOX, int VN, int LB>
__global__ __launch_bounds__(LB) void numeric_sweep_kernel(SweepArgs<R> A) {
  using LT = NumLane<R, P, S, BOX>;
  constexpr int N = LT::N;
  constexpr int M = LT::M;
  constexpr int F_ZR = 0, F_UL = 3 * S, F_UR = 6 * S, F_YH = 9 * S;
  constexpr int F_YL = F_YH + (BOX ? 3 * M : 0);
  constexpr int F_W = 9 * S + (BOX ? 6 * M : 0);
  constexpr int F_C = F_W + M;

  __shared__ R xr_sh[2][kMaxWaves][3 * S];
  __shared__ R xl_sh[2][kMaxWaves][3 * S];
  extern __shared__ double num_lds_raw[];
  R* hist = reinterpret_cast<R*>(num_lds_raw);

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

  // ---- per-segment constants (an idle lane gets a harmless unit segment)
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
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    L.lo[a] = (BOX && active) ? A.k.lo[a * ld + seg] : R(0);
    L.hi[a] = (BOX && active) ? A.k.hi[a * ld + seg] : R(0);
  }

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
    for (int s = 0; s < LT::MB; ++s) {
      L.yh[a][s] = (BOX && active) ? in[(F_YH + a * M + s) * ld + seg] : R(0);
      L.yl[a][s] = (BOX && active) ? in[(F_YL + a * M + s) * ld + seg] : R(0);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) L.cw[a][j] = active ? in[(F_C + a * N + j) * ld + seg] : R(0);
  }
#pragma unroll
  for (int s = 0; s < M; ++s) L.w[s] = active ? in[(F_W + s) * ld + seg] : R(0);

  const int wl = lane & 63, wid = lane >> 6, nw = W >> 6;
  if (__ballot(active) == 0) {
    for (int it = 0; it < A.iters; ++it) __syncthreads();
    return;
  }
  R cfin[3][N], zfin[3][S];
  const int n_plain = A.final_out ? A.iters - 1 : A.iters;
  int it = 0;
  for (; it < n_plain; ++it)
    num_sweep_once<false, VN>(L, A.inner, hist, W, lane, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
  if (A.final_out && A.iters > 0) {
    num_sweep_once<true, VN>(L, A.inner, hist, W, lane, xr_sh[it & 1], xl_sh[it & 1], wl, wid, nw, cfin, zfin);
    if (core) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int j = 0; j < N; ++j) A.c_out[(a * N + j) * ld + seg] = cfin[a][j];
#pragma unroll
        for (int o = 0; o < S; ++o) A.zold_out[(a * S + o) * ld + seg] = zfin[a][o];
      }
    }
  }
  if (core) {
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
      if constexpr (BOX) {
#pragma unroll
        for (int s = 0; s < M; ++s) {
          out[(F_YH + a * M + s) * ld + seg] = L.yh[a][s];
          out[(F_YL + a * M + s) * ld + seg] = L.yl[a][s];
        }
      }
#pragma unroll
      for (int j = 0; j < N; ++j) out[(F_C + a * N + j) * ld + seg] = L.cw[a][j];
    }
#pragma unroll
    for (int s = 0; s < M; ++s) out[(F_W + s) * ld + seg] = L.w[s];
  }
}

template <typename R>
hipError_t dispatch_numeric_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  if (!v.num || !v.vel || v.faces || v.s != v.p || a.rec != nullptr || a.done != nullptr || a.inner < 0)
    return hipErrorInvalidValue;
  if (a.W <= 0 || a.W > 64 || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(a.W);
  const size_t lds = numeric_lds_bytes(v.p, sizeof(R), a.W);
#define TOP_NUM_CASE(P_, B_, VN_)                                                             \
  if (v.p == P_ && (v.box != 0) == B_ && v.vn == VN_) {                                     \
    auto k_ = numeric_sweep_kernel<R, P_, P_, B_, VN_, 64>;                                 \
    hipError_t e_ = hipFuncSetAttribute((const void*)k_, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
    if (e_ != hipSuccess) return e_;                                                        \
    hipLaunchKernelGGL(k_, grid, block, lds, st, a);                                        \
    return hipGetLastError();                                                               \
  }
  TOP_NUM_CASE(3, true, 2) TOP_NUM_CASE(3, false, 2)
  TOP_NUM_CASE(4, true, 2) TOP_NUM_CASE(4, false, 2)
  TOP_NUM_CASE(3, true, 4) TOP_NUM_CASE(3, false, 4)
  TOP_NUM_CASE(4, true, 4) TOP_NUM_CASE(4, false, 4)
#undef TOP_NUM_CASE
  return hipErrorInvalidValue;
}

}  // namespace top
