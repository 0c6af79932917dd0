// Shared definitions of the CADMM sweep library: constants of the
// normalised-time basis, the state layout, and launcher declarations.
//
// Basis.  A segment of duration T is stored as c~_j = c_j T^j, so that
// sigma(tau T) = sum_j c~_j tau^j for tau in [0, 1].  In this basis the
// constraint sample rows of Sec. III-D.1 (positions beta(t_s) and velocities
// beta'(t_s) at t_s = tau_s T, tau_s = s/(M+1)) become the T-independent
// vectors tau_s^j and (1/T) j tau_s^(j-1), the boundary rows of M(T) become
// T^-o times fixed integer vectors, and the cost Gram matrix becomes
// T^(1-2p) Q(1).  All fixed vectors are compile-time constants below.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

namespace top {

// Compile-time loop: f(std::integral_constant<int, i>) for i = Begin..End-1, so that every index
// (and every table value derived from it) is a constant expression.
template <int Begin, int End, typename F>
__host__ __device__ __forceinline__ void static_for(F&& f) {
  if constexpr (Begin < End) {
    f(std::integral_constant<int, Begin>{});
    static_for<Begin + 1, End>(f);
  }
}

constexpr int kSamples = 8;      // M, constraint samples per segment
constexpr int kFaces = 8;        // faces of a general polytope corridor (fewer are padded with inert faces)
constexpr int kMaxWaves = 16;    // 1024-lane workgroups at most
constexpr int32_t kHaloBit = 1 << 30;
constexpr size_t kScratchLimit = 8192;  // per-lane stack limit the library sets; no kernel may exceed it
constexpr int32_t kSegMask = kHaloBit - 1;
// Polls of a neighbour's epoch flag before a chained launch gives up on it (a poll is a memory
// round trip plus a short sleep, so roughly a second in all; an epoch takes tens of microseconds).
// The environment variable TOP_CHAIN_SPIN, read when a handle is created, can lower it (a test of
// the give-up path sets 0).
constexpr int kChainSpin = 1 << 20;

enum : uint8_t { kFirst = 1, kLast = 2 };

// The helpers below are loops, not recursion, so that a call left to run time needs no stack.
__host__ __device__ constexpr double cfact(int o) {
  double r = 1.0;
  for (int k = 2; k <= o; ++k) r *= k;
  return r;
}
// j! / (j - o)!: factor of the o-th derivative on t^j
__host__ __device__ constexpr double cfall(int o, int j) {
  if (j < o) return 0.0;
  double r = 1.0;
  for (int k = j - o + 1; k <= j; ++k) r *= k;
  return r;
}
__host__ __device__ constexpr double cpow(double x, int e) {
  double r = 1.0;
  for (int k = 0; k < e; ++k) r *= x;
  return r;
}
// sample instant tau_s = (s+1)/(M+1), s = 0..M-1
__host__ __device__ constexpr double ctau(int s) { return double(s + 1) / double(kSamples + 1); }
// position row of sample s, coefficient j: tau_s^j
__host__ __device__ constexpr double cpos(int s, int j) { return cpow(ctau(s), j); }
// velocity row of sample s (before the 1/T factor): j tau_s^(j-1)
__host__ __device__ constexpr double cvel(int s, int j) { return j == 0 ? 0.0 : j * cpow(ctau(s), j - 1); }
// Q(1) entry for cost order p: [j!/(j-p)!][k!/(k-p)!] / (j+k-2p+1), zero below order p
__host__ __device__ constexpr double cgram(int p, int j, int k) {
  return (j < p || k < p) ? 0.0 : cfall(p, j) * cfall(p, k) / double(j + k - 2 * p + 1);
}
// Coefficients of the rest-to-rest unit step of degree 2p-1 in tau (derivatives 1..p-1 vanish at
// both ends): 10 t^3 - 15 t^4 + 6 t^5 for p = 3 and 35 t^4 - 84 t^5 + 70 t^6 - 20 t^7 for p = 4.
__host__ __device__ constexpr double cstep(int p, int j) {
  return p == 3 ? (j == 3 ? 10.0 : j == 4 ? -15.0 : j == 5 ? 6.0 : 0.0)
                : (j == 4 ? 35.0 : j == 5 ? -84.0 : j == 6 ? 70.0 : j == 7 ? -20.0 : 0.0);
}
// packed upper-triangle index of a symmetric n x n matrix
__host__ __device__ constexpr int tri(int n, int i, int j) {
  return i <= j ? i * n - i * (i - 1) / 2 + (j - i) : j * n - j * (j - 1) / 2 + (i - j);
}

// Field offsets of the per-segment iterate state (structure of arrays, one row of ld values per
// field).  z holds the segment's end knot; its start knot is the previous segment's end knot, or
// the trajectory's start state.  y packs each corridor slack/dual pair (box: upper and lower row
// per axis and sample; polytope: one row per face and sample), g each velocity split/dual pair.
struct Layout {
  int p, s, box, vel;
  int faces = 0;             // kFaces for a polytope corridor, else 0
  int num = 0;               // NumericSolve: velocity multipliers w [M] and the last c~ [3n] instead of g
  __host__ __device__ int n() const { return 2 * p; }
  __host__ __device__ int nh() const { return n() * (n() + 1) / 2; }
  __host__ __device__ int zR() const { return 0; }
  __host__ __device__ int uL() const { return 3 * s; }
  __host__ __device__ int uR() const { return 6 * s; }
  __host__ __device__ int yh() const { return 9 * s; }
  __host__ __device__ int yl() const { return 9 * s + (box ? 3 * kSamples : 0); }
  __host__ __device__ int g() const { return 9 * s + (box ? 6 * kSamples : faces * kSamples); }
  __host__ __device__ int nf() const { return g() + (num ? kSamples + 3 * n() : (vel ? 3 * kSamples : 0)); }
  // rho * Htilde^-1 rows: one matrix, or one per rotated axis for a polytope
  __host__ __device__ int nhr() const { return faces ? 3 * nh() : nh(); }
};

// Read-only per-segment constants, all [.][ld] structure of arrays in the iterate precision.
template <typename R>
struct SegConsts {
  const R* Hr;          // [nh] packed rho * Htilde^-1 (symmetric); polytope: [3][nh], one per rotated axis
  const R* iT;          // 1/T
  const R* lo;          // [3] corridor
  const R* hi;          // [3]
  const R* U;           // polytope: [9] rotation to the axes of sum_k a_k a_k^T, U[3 q + a'] = U_{q a'}
  const R* fa;          // polytope: [kFaces][4] faces a_x, a_y, a_z, b
  const double* rho;    // [S] rho of the segment's trajectory (NumericSolve)
  const R* vmax;        // velocity bound of the segment's trajectory
  const uint8_t* flags; // kFirst | kLast
  const int32_t* traj;  // trajectory of the segment
  const R* bcL;         // [B][3][s] start-knot state of each trajectory
  int64_t ld;
};

template <typename R>
struct SweepArgs {
  SegConsts<R> k;
  const int32_t* lane_seg;  // [n_tiles * W] segment of each lane, | kHaloBit for halo copies, -1 idle
  int W;
  const R* st_in;
  R* st_out;
  int iters;                // sweeps in this launch
  int fixpos;
  int final_out;            // write c~ and the end knot before its last update, at the last sweep
  R* c_out;                 // [3n][ld]
  R* zold_out;              // [3s][ld]
  const uint8_t* done;      // [B] nonzero: the trajectory has stopped; both state buffers hold its final
                            // state and its lanes neither load nor store; or null
  int inner;                // NumericSolve: L-BFGS iterations per local solve
  int store_frozen;         // 1: lanes of stopped trajectories in waves with live lanes store their (unchanged)
                            // state, for an output buffer that does not hold it yet (tuning probes)
  R* rec;                   // recording launches (reverse-pass replay): the state after sweep i of the
  int64_t rec_slot;         // launch, i < iters - 1, goes to rec + (i + 1) * rec_slot; else null
  // Chained launch (lane-per-axis sweep): `iters` sweeps in epochs of chain_halo sweeps inside one
  // cooperative launch.  Between epochs every tile publishes the core segments its neighbours copy
  // into their halos (to the other state buffer) and reloads its own halo copies once its two
  // neighbours have published; 0 runs one epoch (the ordinary launch).
  int chain_halo;
  const int32_t* chain;            // [n_tiles][4]: left / right source tile of the halo (-1: none),
                                   // first core lane, one past the last core lane
  unsigned long long* chain_flag;  // [n_tiles] waves' exports per tile (left edge low, right high), zero at launch
  int* chain_err;                  // set to 1 when a wait for a neighbour gave up
  int chain_spin;                  // polls of a neighbour's flag before giving up (kChainSpin)
};

struct Variant {
  int prec;  // 0 fp32, 1 fp64
  int p, s, box, vel;
  int faces = 0;  // kFaces: general polytope corridor (box is then 0)
  int num = 0;    // 1: NumericSolve local update (L-BFGS) instead of the closed form
  int vn = 2;     // norm of the velocity bound: 2 (Euclidean ball) or 4 (l4 ball, NumericSolve only)
};

template <typename R>
hipError_t launch_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st);
// Tiles of W lanes of that sweep (one lane per segment) the device holds at once, or 0.
template <typename R>
int sweep_resident(const Variant& v, int W);
// the same sweep with one lane per segment and axis (3 W threads per tile of W <= axis_max_tile
// segments; closed form with s < 2p - 1, no recording, no stopped trajectories).  Float32 tiles go
// to 320 segments (960 lanes at four waves per SIMD, 128 VGPRs); float64 ones to 128, so that the
// doubled registers need no spills.
constexpr int kAxisTileMax = 320;
inline int axis_max_tile(int prec) { return prec == 0 ? kAxisTileMax : 128; }
template <typename R>
hipError_t launch_sweep_axis(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st);
// Workgroups of the lane-per-axis sweep for W-segment tiles that the device holds at once (the
// bound of a chained launch), or 0 when the device has no cooperative launch.
template <typename R>
int sweep_axis_resident(const Variant& v, int W);
// zero n unsigned 64-bit words (the epoch flags of a chained launch)
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st);
// the same launch for a general polytope corridor (v.faces = kFaces)
template <typename R>
hipError_t launch_poly_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st);
// Tiles of W lanes of that sweep the device holds at once, or 0.
template <typename R>
int poly_resident(const Variant& v, int W);
// the same launch with the NumericSolve local update (v.num = 1)
template <typename R>
hipError_t launch_numeric_sweep(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st);
// ... with four lanes per segment (three axes and a spare; 4 W threads per tile of W <=
// num_quad_max_tile segments)
constexpr int kNumQuadTileMax = 128;
constexpr int num_quad_max_tile(int prec) { return prec == 0 ? kNumQuadTileMax : 64; }
template <typename R>
hipError_t launch_numeric_quad(const Variant& v, const SweepArgs<R>& a, int n_tiles, hipStream_t st);

// One-time setup (precompute + Init), float64 arithmetic, output in R.
struct SetupArgs {
  const double* waypoints;   // [S+B][3]
  const double* durations;   // [S]
  const double* bc;          // [B][2][p][3] or null
  const double* box_lo;      // [S][3] or null
  const double* box_hi;
  const double* faces;       // [S][n_faces][4] polytope a_x, a_y, a_z, b, or null
  int n_faces;
  const double* vmax;        // [B] or null
  const double* rho;         // [B]
  const int64_t* seg_off;    // [B+1] device copy
  int B;
  int64_t S;
  int fixpos;
};

template <typename R>
struct SetupOut {
  R* Hr; R* iT; R* lo; R* hi; R* vmax; uint8_t* flags; int32_t* traj; R* bcL;
  R* state; R* c; int64_t ld;
  double* Tdev;              // [S] float64 copy of T (finalize)
  double* rho_seg;           // [S] float64 rho of the segment's trajectory (finalize)
  R* Hd;                     // [nh][ld] d(rho Htilde^-1)/dT, or null when no tape is kept
  R* U;                      // polytope: [9][ld] rotation
  R* fa;                     // polytope: [kFaces * 4][ld] faces (padded)
  double* lam;               // polytope: [3][ld] eigenvalues of sum_k a_k a_k^T
  R* state1;                 // the second state buffer (its padding columns are zeroed too), or null
  int nf;                    // state rows
};

template <typename R>
hipError_t launch_setup(const Variant& v, const SetupArgs& a, const SetupOut<R>& o, hipStream_t st);

hipError_t launch_validate(const SetupArgs& a, int p, int* bad, hipStream_t st);

// Finalize: per-segment float64 partials (cost, primal gap^2, dual^2) and monomial coefficients.
template <typename R>
struct FinalArgs {
  const R* c;           // [3n][ld]
  const R* state;       // current state [nf][ld]
  const R* zold;        // [3s][ld]
  const R* bcL;
  const double* T;      // [S]
  const double* rho;    // [S]
  const uint8_t* flags;
  const int32_t* traj;
  int64_t S, ld;
  double* part;         // [3][S] cost, rp^2, rd^2
  double* coeffs;       // [S][3][n] or null
  int* nonfinite;
  int with_res;
  const uint8_t* done;  // [B] or null: segments of stopped trajectories keep their partials (skipped)
  const int64_t* off;   // [B + 1] segment offsets (used with done: a trajectory-major grid)
  int B;
  int64_t max_len;      // segments of the longest trajectory
  const int32_t* live;        // with done: the trajectories still running (the last check's list)
  const int32_t* live_count;  // and their number
};

template <typename R>
hipError_t launch_finalize(const Variant& v, const FinalArgs<R>& a, hipStream_t st);

// Monomial coefficients c_{a,j} = c~_{a,j} / T^j in float64, [S][3][2p], from c~ [3*2p][ld].
template <typename R>
hipError_t launch_coeffs(int p, const R* c, const double* T, int64_t S, int64_t ld, double* out, hipStream_t st);

// Per-trajectory sums of the per-segment partials part[3][S] in a fixed order: out[0][b] = cost,
// out[1][b] = ||r_p||, out[2][b] = ||r_d|| (square roots taken).  Each trajectory is cut into chunks of
// kReduceChunk segments (chunk j of trajectory b covers segments off[b] + j*kReduceChunk onwards); one
// workgroup sums a chunk, then one lane per trajectory adds its chunk sums in order.  The order depends
// only on the segment offsets, not on the sweep's tiling.
constexpr int kReduceChunk = 4096;
struct ReduceArgs {
  const double* part;        // [3][S]
  int64_t S;
  const int64_t* off;        // [B + 1] segment offsets
  int B;
  const int32_t* chunk_traj; // [n_chunks] trajectory of each chunk (chunks of a trajectory are consecutive)
  const int32_t* chunk_off;  // [B + 1] first chunk of each trajectory
  int n_chunks;
  double* chunk_sum;         // [3][n_chunks] scratch
  double* out;               // [3][B]
  const uint8_t* done;       // [B] or null: stopped trajectories keep their sums (skipped)
};
hipError_t launch_reduce(const ReduceArgs& a, hipStream_t st);

hipError_t launch_copy_rows(const double* src, double* dst, int B, hipStream_t st);

// ---- residual checks and the adaptive penalty (Sec. III-D.3)
struct CheckArgs {
  const double* res;      // [3][B] cost, ||r_p||, ||r_d|| of the sweep just finished
  const int64_t* off;     // [B+1] segment offsets
  int B;
  int check_every;
  int adapt;
  double tol, mu, tau_incr, tau_decr;
  uint8_t* done;          // [B] set once the stopping test passes
  uint8_t* fresh;         // [B] 1 for the trajectories that stopped at this check, else 0
  int32_t* swept;         // [B] sweeps counted at the checks while the trajectory runs
  int32_t* stop_at;       // [B] sweeps applied when it stopped
  double* rho;            // [B] current penalty
  double* ratio;          // [B] rho_old / rho_new at this check, 1 when unchanged
  int32_t* lists;         // [3][B] the trajectories that stopped / whose rho changed at this check /
                          // that still run after it
  int32_t* counts;        // [3] their numbers (zeroed before the check)
};
hipError_t launch_check(const CheckArgs& a, hipStream_t st);
// Zero the three list lengths of a check (a one-lane kernel, so that a captured graph holds no memset).
hipError_t launch_reset_counts(int32_t* counts, hipStream_t st);
// The list of running trajectories before the first check: every trajectory.
hipError_t launch_all_running(int32_t* lists, int32_t* counts, int B, hipStream_t st);
// Copy the state of the trajectories that just stopped into the other ping-pong buffer (nf fields of
// rsz bytes per segment), so that later sweeps can leave them alone.
// list / count: the trajectories that stopped at this check (check_kernel's first list); off [B + 1]
// the segment offsets, max_len the longest trajectory's segment count.
hipError_t launch_freeze_copy(const void* cur, void* other, const int32_t* list, const int32_t* count,
                              const int64_t* off, int B, int64_t max_len, int nf, int64_t ld, size_t rsz,
                              hipStream_t st);

template <typename R>
struct RescaleArgs {
  const double* lam;      // polytope: [3][ld] eigenvalues of sum_k a_k a_k^T
  R* state;               // [nf][ld] current state, rescaled in place
  R* Hr;                  // [nh][ld] rho * Htilde^-1, refactored in place
  double* rho_seg;        // [S]
  const double* ratio;    // [B]
  const double* rho;      // [B]
  const double* T;        // [S]
  const uint8_t* flags;
  const int32_t* traj;
  const R* vmax;
  int64_t S, ld;
  const int64_t* off;     // [B + 1] segment offsets (trajectory-major grid)
  int B;
  int64_t max_len;        // segments of the longest trajectory
  const int32_t* list;    // the trajectories whose rho changed at this check
  const int32_t* count;   // their number
};
template <typename R>
hipError_t launch_rescale(const Variant& v, const RescaleArgs<R>& a, hipStream_t st);

// top_convergence outputs; done/stop_at may be null (no checks), then every trajectory has all sweeps.
hipError_t launch_conv_report(const uint8_t* done, const int32_t* stop_at, const double* rho, int B,
                              int32_t iters_done, int32_t* iters_out, double* rho_out, uint8_t* done_out,
                              hipStream_t st);

// ---- reverse pass
template <typename R>
struct AdjArgs;
template <typename R>
hipError_t launch_adjoint(const Variant& v, const AdjArgs<R>& a, int n_tiles, hipStream_t st);

template <typename R>
hipError_t launch_fill(R* p, int64_t n, R v, hipStream_t st);

// The adjoint kernel runs a tile of W segments as 3 W lanes (one per segment and axis), so an axis
// has at most kMaxAxisWaves waves.  Its largest tile: 128 segments in float32 (384 lanes, two waves
// per SIMD), 64 in float64 (192 lanes, one wave per SIMD).
constexpr int kMaxAxisWaves = 4;
inline int adjoint_max_tile(int prec) { return prec == 0 ? 128 : 64; }
// Dynamic LDS of the adjoint kernel: each segment's rho Htilde^-1 and its T-derivative, the per-axis
// partial adjoints of the velocity factors (double buffered), then the per-axis parameter adjoints
// summed at the end; rows of W values (the kernel strides them by its largest tile).
inline size_t adjoint_lds_bytes(const Variant& v, size_t rsz, int W) {
  const int n = 2 * v.p, nh = n * (n + 1) / 2;
  const int nf = 2 * nh + 2 * 3 * (v.vel ? kSamples : 1) + 6;
  return (size_t)nf * rsz * (size_t)W;
}
// Static LDS of the adjoint kernel (wave-boundary exchange buffers), an upper bound.
constexpr size_t kAdjointStaticLds = 2 * 3 * kMaxAxisWaves * 4 * 5 * sizeof(double);

template <typename R>
struct InitAdjArgs {
  const double* waypoints;
  const double* durations;
  const double* box_lo;
  const double* box_hi;
  const double* vmax;
  const double* bc;          // null: rest end states at the end waypoints
  const int32_t* traj;
  const uint8_t* flags;
  int64_t S, ld;
  const R* lam;              // adjoint of the Init state [nf][ld]
  const R* acc_iT;
  const R* acc_hd;
  const R* acc_z0;           // [3s][ld]
  double* dPL;               // [S][3] per segment: its start waypoint
  double* dPR;               // [S][3] its end waypoint
  double* dK;                // [S][3] its end knot's position
  double* dK0;               // [S][3] the trajectory start knot's position (first segments)
  double* dT;                // [S] or null
};

template <typename R>
hipError_t launch_init_adjoint(const Variant& v, const InitAdjArgs<R>& a, hipStream_t st);

hipError_t launch_gather_waypoints(const double* dPL, const double* dPR, const double* dK, const double* dK0,
                                   const int64_t* off, int B, int64_t rows, double* dP, hipStream_t st);

}  // namespace top
