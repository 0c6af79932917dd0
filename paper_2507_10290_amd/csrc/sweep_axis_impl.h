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
//
// Chained launches.  Run as one launch per `halo` sweeps, every launch reloads and stores the whole
// state of every tile, a fixed cost of about six sweeps' time for a 320-segment tile.  A chained
// launch (SweepArgs::chain_halo > 0, cooperative, so that every tile is resident) runs all the
// sweeps of the call in epochs of at most `halo` sweeps.  At the end of an epoch each wave holding
// core segments a neighbour copies (the `halo` segments next to each core edge, one more on the
// right for the start knot of the neighbour's outermost copy) stores them into the other state
// buffer and counts itself in the tile's flag, one 32-bit count per edge; each wave holding halo
// copies waits until the edges it copies from have been counted by all of their waves for this
// epoch, and reloads its copies.  The halo copies then hold exactly what a fresh launch would load,
// and the core segments keep their registers, so the results are the same bits as one launch per
// epoch.  No tile-wide barrier is added: the sweep's own barrier keeps a tile's waves together.
//
// Ordering of the exchange.  The published values and the counts are written and read only with
// device-scope atomic accesses (relaxed), which the L2 caches of the chip's dies do not hold
// incoherently.  A writer wave waits for its stores to complete before one of its lanes adds to the
// count; a reader wave's polling lane sees the count before the wave issues its loads.  So every
// value is complete before it is counted and read only after the count is seen: the order a release
// and an acquire would give, without their write-back and invalidation of the whole L2 (which cost
// more than the launch they replace).  A buffer is written again two epochs later, after both
// neighbours have counted the epoch in between, which they do only after their sweeps have used
// every value they loaded from it.
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

// x, hidden from the optimiser: address arithmetic built on it is redone at every use instead of
// being hoisted out of the epoch loop into registers held across every sweep.
__device__ __forceinline__ int64_t opaque(int64_t x) {
  asm volatile("" : "+v"(x));
  return x;
}

// s_waitcnt operand that waits for every outstanding vector memory access (vmcnt 0) and for
// nothing else (expcnt 7, lgkmcnt 15: their maxima, in the GFX9 encoding).
constexpr int kWaitStores = 0x0F70;

// Wait until the 32-bit count at bit `shift` of a tile's flag reaches `count`; false if the poll
// bound ran out.  The polls are device-scope atomic loads; every load of the values the count
// guards comes after them.
__device__ inline bool chain_wait(const unsigned long long* flag, int shift, unsigned long long count, int spin) {
  for (int i = 0; i < spin; ++i) {
    const unsigned long long f = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (((f >> shift) & 0xFFFFFFFFull) >= count) return true;
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
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
  // axis of this lane, the same for every lane of a wave (W is a multiple of 64): taken as a scalar,
  // every state field's offset is one scalar for the wave
  const int a = __builtin_amdgcn_readfirstlane(threadIdx.x / W);
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

  // epochs: one, or ceil(iters / chain_halo) in a chained launch (chain: neighbour tiles and the
  // core lane range)
  const int ep_len = A.chain_halo > 0 ? A.chain_halo : A.iters;
  const int n_ep = A.chain_halo > 0 ? (A.iters + ep_len - 1) / ep_len : 1;
  int dep_l = -1, dep_r = -1, core_lo = 0, core_hi = W;
  if (A.chain_halo > 0) {
    const int32_t* c = A.chain + 4 * (int64_t)blockIdx.x;
    dep_l = c[0];
    dep_r = c[1];
    core_lo = c[2];
    core_hi = c[3];
  }

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
  R gall[3][MV];
#pragma unroll
  for (int o = 0; o < S; ++o) L.zL[o] = (active && L.first) ? A.k.bcL[((int64_t)tr * 3 + a) * S + o] : R(0);
  // (a trajectory's first segment keeps its start knot, which no sweep changes)
  auto get = [](const R* p, auto dev) -> R {
    if constexpr (decltype(dev)::value) return __hip_atomic_load(const_cast<R*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else return *p;
  };
  auto load = [&](const R* in0, auto dev) {
    const R* in = in0 + opaque(seg);
#pragma unroll
    for (int o = 0; o < S; ++o) {
      const int f = a * S + o;
      L.zR[o] = active ? get(&in[(F_ZR + f) * ld], dev) : R(0);
      L.uL[o] = active ? get(&in[(F_UL + f) * ld], dev) : R(0);
      L.uR[o] = active ? get(&in[(F_UR + f) * ld], dev) : R(0);
      if (active && !L.first) L.zL[o] = get(&in[(F_ZR + f) * ld - 1], dev);
    }
#pragma unroll
    for (int s = 0; s < LT::MB; ++s) {
      L.yh[s] = (BOX && active) ? get(&in[(F_YH + a * M + s) * ld], dev) : R(0);
      L.yl[s] = (BOX && active) ? get(&in[(F_YL + a * M + s) * ld], dev) : R(0);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int s = 0; s < MV; ++s) gall[b][s] = (VEL && active) ? get(&in[(F_G + b * M + s) * ld], dev) : R(0);
    // (the own axis' values loaded again rather than picked out of gall by axis: a pick by the
    // lane's axis index can turn gall into an indexed array in scratch memory)
#pragma unroll
    for (int s = 0; s < MV; ++s) L.g[s] = (VEL && active) ? get(&in[(F_G + a * M + s) * ld], dev) : R(0);
  };
  // this axis' state fields of the segment; DEV: as device-coherent accesses (the exchange between
  // the tiles of a chained launch)
  auto put = [](R* p, R x, auto dev) {
    if constexpr (decltype(dev)::value) __hip_atomic_store(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else *p = x;
  };
  auto store = [&](R* out0, auto dev) {
    R* out = out0 + opaque(seg);
#pragma unroll
    for (int o = 0; o < S; ++o) {
      const int f = a * S + o;
      put(&out[(F_ZR + f) * ld], L.zR[o], dev);
      put(&out[(F_UL + f) * ld], L.uL[o], dev);
      put(&out[(F_UR + f) * ld], L.uR[o], dev);
    }
    if constexpr (BOX) {
#pragma unroll
      for (int s = 0; s < M; ++s) {
        put(&out[(F_YH + a * M + s) * ld], L.yh[s], dev);
        put(&out[(F_YL + a * M + s) * ld], L.yl[s], dev);
      }
    }
    if constexpr (VEL) {
#pragma unroll
      for (int s = 0; s < M; ++s) put(&out[(F_G + a * M + s) * ld], L.g[s], dev);
    }
  };
  // epoch e reads buffer e % 2 (0: st_in) and writes the other
  R* const buf0 = const_cast<R*>(A.st_in);
  R* const buf1 = A.st_out;
  auto bufs = [&](int q) { return (q & 1) ? buf1 : buf0; };
  load(buf0, std::false_type{});
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
  // Chained epochs, wave by wave (no tile barrier at an epoch boundary): a wave holding core lanes a
  // neighbour copies stores them and adds one to the tile's count for that edge (low half of its
  // flag: left edge, high half: right edge); a wave holding halo copies waits until the count of
  // every edge it copies from has reached the epoch times the number of waves that export that edge,
  // then reloads.  The other waves go straight on; the sweep's barrier holds them.
  const int h = A.chain_halo;
  const bool exp_l = core && dep_l >= 0 && lane < core_lo + h;
  const bool exp_r = core && dep_r >= 0 && lane >= core_hi - h - 1;
  const bool cp_l = active && !core && lane < core_lo;
  const bool cp_r = active && !core && lane >= core_hi;
  const unsigned long long add = (__ballot(exp_l) != 0 ? 1ull : 0ull) + (__ballot(exp_r) != 0 ? 1ull << 32 : 0ull);
  const bool wait_l = __ballot(cp_l) != 0, wait_r = __ballot(cp_r) != 0;
  // waves (three axes) holding the lanes [lo, hi) of an axis
  auto waves_over = [](int lo, int hi) { return hi > lo ? 3 * (((hi - 1) >> 6) - (lo >> 6) + 1) : 0; };
  unsigned long long need_l = 0, need_r = 0, need_own = 0;   // per epoch
  if (h > 0) {
    if (wait_l) {   // dep_l's right edge
      const int lo2 = A.chain[4 * (int64_t)dep_l + 2], hi2 = A.chain[4 * (int64_t)dep_l + 3];
      need_l = waves_over(max(lo2, hi2 - h - 1), hi2);
    }
    if (wait_r) {   // dep_r's left edge, and this tile's right edge (the start knot of the first copy)
      const int lo2 = A.chain[4 * (int64_t)dep_r + 2], hi2 = A.chain[4 * (int64_t)dep_r + 3];
      need_r = waves_over(lo2, min(hi2, lo2 + h));
      need_own = waves_over(max(core_lo, core_hi - h - 1), core_hi);
    }
  }
  int left = A.iters;
  for (int e = 0; e < n_ep; ++e) {
    if (e > 0 && (wait_l || wait_r)) {
      // the neighbours' core edges of the last epoch are in bufs(e) once their counts show it
      if (wl == 0) {
        const unsigned long long E = (unsigned long long)e;
        bool ok = true;
        if (wait_l) ok = chain_wait(A.chain_flag + dep_l, 32, E * need_l, A.chain_spin);
        if (ok && wait_r) ok = chain_wait(A.chain_flag + dep_r, 0, E * need_r, A.chain_spin);
        if (ok && wait_r) ok = chain_wait(A.chain_flag + blockIdx.x, 32, E * need_own, A.chain_spin);
        if (!ok) atomicOr(A.chain_err, 1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");   // no load moves above the polls
      if (cp_l || cp_r) load(bufs(e), std::true_type{});
    }
    const int n = e + 1 < n_ep ? ep_len : left;
    // the call's last sweep (with its outputs) runs after the loop
    const int n_plain = e + 1 == n_ep && A.final_out && n > 0 ? n - 1 : n;
    for (int it = 0; it < n_plain; ++it) sweep(std::false_type{});
    left -= n;
    if (e + 1 < n_ep && add != 0) {
      // publish the core segments the neighbours copy: the chain_halo next to each core edge that
      // has a neighbour, and on the right one more (the start knot of the neighbour's outermost
      // copy is that segment's end knot)
      if (exp_l || exp_r) store(bufs(e + 1), std::true_type{});
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");   // no store moves below the count
      __builtin_amdgcn_s_waitcnt(kWaitStores);   // this wave's exchange stores are complete
      if (wl == 0) __hip_atomic_fetch_add(A.chain_flag + blockIdx.x, add, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }

  if (A.final_out && A.iters > 0) sweep(std::true_type{});

  if (core) {
    if (A.final_out && A.iters > 0) {
#pragma unroll
      for (int j = 0; j < N; ++j) A.c_out[(a * N + j) * ld + seg] = cfin[j];
#pragma unroll
      for (int o = 0; o < S; ++o) A.zold_out[(a * S + o) * ld + seg] = zfin[o];
    }
    store(bufs(n_ep), std::false_type{});
  }
}

// The kernel instance of variant v, or nullptr.
template <typename R, int LBT>
void* sweep_axis_instance(const Variant& v) {
  if (v.num || v.faces || v.s == 2 * v.p - 1) return nullptr;
#define TOP_AXIS_CASE(P_, S_, B_, V_)                                                             \
  if (v.p == P_ && v.s == S_ && (v.box != 0) == B_ && (v.vel != 0) == V_)                        \
    return reinterpret_cast<void*>(sweep_axis_kernel<R, P_, S_, B_, V_, 3 * LBT>);
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
  return nullptr;
}

// Launch over tiles of W <= LBT segments (3 W threads each); closed form, s in {p, p+1}, no
// recording and no stopped trajectories.  A chained launch (a.chain_halo > 0) is cooperative: the
// runtime refuses it unless every tile can be resident at once.
template <typename R, int LBT>
hipError_t dispatch_sweep_axis(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st) {
  if (a.rec != nullptr || a.done != nullptr) return hipErrorInvalidValue;
  if (a.W <= 0 || a.W > LBT || (a.W & 63) != 0 || n_tiles <= 0) return hipErrorInvalidValue;
  if (a.chain_halo > 0 && (a.chain == nullptr || a.chain_flag == nullptr || a.chain_err == nullptr))
    return hipErrorInvalidValue;
  void* k = sweep_axis_instance<R, LBT>(v);
  if (k == nullptr) return hipErrorInvalidValue;
  dim3 grid(n_tiles), block(3 * a.W);
  const size_t lds = sweep_axis_lds_bytes(v.p, v.vel != 0, sizeof(R), LBT);
  hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  SweepArgs<R> arg = a;
  void* params[] = {&arg};
  if (a.chain_halo > 0) return hipLaunchCooperativeKernel(k, grid, block, params, (unsigned)lds, st);
  return hipLaunchKernel(k, grid, block, params, lds, st);
}

// Tiles of W segments that the device holds at once, 0 without cooperative launches.
template <typename R, int LBT>
int resident_sweep_axis(const Variant& v, int W) {
  void* k = sweep_axis_instance<R, LBT>(v);
  if (k == nullptr || W <= 0 || W > LBT) return 0;
  int dev = 0, coop = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || coop == 0) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  const size_t lds = sweep_axis_lds_bytes(v.p, v.vel != 0, sizeof(R), LBT);
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 3 * W, lds) != hipSuccess) return 0;
  return per_cu * cus;
}

}  // namespace top
