/*
 * top.h -- C ABI of the MI355X consensus-ADMM (CADMM) trajectory sweep.
 *
 * The library solves, for a batch of independent trajectories, the
 * piecewise-polynomial minimum-effort problem of the TOP paper (arXiv
 * 2507.10290): Sec. III-A states the problem (cost int sigma^(p)T sigma^(p),
 * end states sigma_0 / sigma_N, continuity between segments), Sec. III-B
 * turns it into a consensus problem over knot states z with scaled duals u,
 * Sec. III-C adds the corridor (linear inequalities with slack s and dual v)
 * and the velocity ball (quadratic inequality with split phi and dual w), and
 * Sec. III-D.1 gives the per-segment closed-form update rules (eqs.
 * QpSubProblem, UpdateZ, UpdateU, NonNegativeProject, UpdateV,
 * DynamicProject, UpdateCloseW).  Each call of top_iterate runs k passes of
 * Algorithm 1's loop body with fixed rho over every segment of every
 * trajectory.
 *
 * Conventions
 *   - Trajectories are given in CSR form: trajectory b owns segments
 *     seg_offsets[b] .. seg_offsets[b+1]-1 (S = seg_offsets[B] in total) and
 *     the S+B waypoint rows seg_offsets[b]+b .. seg_offsets[b+1]+b.
 *   - Arrays marked [dev] are device pointers, valid on the stream passed to
 *     top_create; arrays marked [host] are host pointers.  All [dev] inputs
 *     are float64 whatever the iterate precision.
 *   - Inputs are read only by work that top_create queues on its stream; the
 *     library keeps its own copies (in the iterate precision, or float64 where
 *     noted).  The inputs must stay allocated and unchanged until the stream
 *     has run that work (work queued on the same stream afterwards is ordered
 *     after it).  The caller owns every output buffer.
 *   - Device memory.  The per-problem state (Algorithm 1's iterates, the
 *     per-segment factors, the tape) lives in one workspace that the caller
 *     allocates (top_workspace_bytes gives its size) and passes to
 *     top_create; such a handle makes no device allocation of its own.  The
 *     caller keeps the workspace allocated, and uses it for nothing else,
 *     until the handle has been destroyed and the handle's stream has run the
 *     work queued before that (an allocation made on that stream by a
 *     stream-ordered allocator, such as PyTorch's, satisfies this when it is
 *     released after top_destroy).  Read-only tables that depend only on the
 *     trajectory lengths (device copies of the offsets, the reduction chunk
 *     table, the tile lane map) are built once per shape and device and kept
 *     in a library cache shared by every handle of that shape.  A NULL
 *     workspace makes the library take the state from its own pool instead
 *     (hipMalloc; blocks are kept for reuse by later handles).
 *   - Every call that launches work is asynchronous on the handle's stream:
 *     outputs are ready once that stream has been synchronised.
 *   - A handle is not thread-safe; use one handle per host thread.  It belongs
 *     to the device that was current at top_create (its stream's device):
 *     make that device current for every later call on it.
 *   - Errors: every call returns a top_status.  Argument errors are reported
 *     before any work is queued and leave the handle unchanged.  A non-finite
 *     iterate is flagged on the device and reported by top_sync_status.
 *     top_last_error() gives a thread-local message for the last failure.
 */
#ifndef TOP_H_
#define TOP_H_

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct top_problem top_problem;

typedef enum top_status {
  TOP_OK = 0,
  TOP_E_INVALID = -1,      /* an argument is null, out of range or not finite          */
  TOP_E_WORKSPACE = -2,    /* the workspace given to top_create is too small            */
  TOP_E_HIP = -3,          /* a HIP runtime call failed                                 */
  TOP_E_STATE = -4,        /* the call is not valid in the handle's current state       */
  TOP_E_NONFINITE = -5,    /* an iterate became NaN or infinite                         */
  TOP_E_UNSUPPORTED = -6,  /* the option combination is not implemented                */
  TOP_E_NOMEM = -7         /* a host or device allocation failed                        */
} top_status;

enum { TOP_FP32 = 0, TOP_FP64 = 1 };

/* Problem and execution options (host struct, copied by top_create). */
typedef struct top_options {
  int32_t order;             /* p: 3 = minimum jerk (quintic), 4 = minimum snap (septic) (Sec. III-A) */
  int32_t n_cont;            /* s: derivative orders 0..s-1 shared at interior knots, s in {p, p+1,
                                2p-1} (2p-1 is the consensus on every order 0..2p-2, without a tape);
                                0 selects s = p (Sec. III-B, eq. Consensus_problem)                   */
  int32_t fix_interior;      /* 1: interior knot positions are pinned to the waypoints;
                                0: they are averaged like the other orders (Sec. III-D.2)              */
  int32_t n_samples;         /* M: constraint samples per segment at t_j = j T/(M+1), j = 1..M;
                                only 8 is built (0 selects 8) (Sec. III-D.1)                          */
  int32_t precision;         /* TOP_FP32 or TOP_FP64 iterates; the per-segment factorisation and all
                                reductions are float64 in both                                       */
  int32_t checkpoint_every;  /* m > 0 records the state every m sweeps so top_backward can run;
                                0 records nothing                                                     */
  int32_t max_taped_iters;   /* sweeps the tape can hold when checkpoint_every > 0                    */
  int32_t tile_lanes;        /* segments per workgroup tile, a multiple of 64 from 64 up to the
                                variant's maximum (TOP_E_INVALID above it).  One lane per segment:
                                512 for float32 order 3 (closed form with n_cont < 2p-1, or a
                                polytope corridor), 64 for NumericSolve, 256 otherwise; with a tape
                                128 (float32) or 64 (float64), the adjoint's tiles.  One lane per
                                segment and axis (lane_form 3): 320 (float32) or 128 (float64);
                                NumericSolve's four lanes per segment: 128 (float32) or 64
                                (float64).  0 picks the maximum (64 for NumericSolve's four-lane
                                form), or the tuned value after top_tune                             */
  int32_t halo;              /* sweeps per launch for trajectories longer than a tile (their halo
                                width); 0 picks the default.  With a tape it must be >= 2: the
                                reverse pass runs halo - 1 steps per launch                           */
  int32_t use_graph;         /* 1: a top_iterate(k) launch sequence asked for again (same k, buffer
                                and check phase) is captured once and replayed as a hipGraph      */
  /* Stopping test and adaptive penalty (Sec. III-D.3, eqs. splitting_tolerance and UpdateRho).
     Residuals are formed every check_every sweeps, counted from Init; at each such check a
     trajectory of N segments whose ||r_p||^2 and ||r_d||^2 are both below (N tol)^2 stops (its
     coefficients, cost and residuals stay those of that sweep; later sweeps leave it unchanged),
     and otherwise, with adapt_rho, its rho is multiplied by tau_incr when ||r_p|| > mu ||r_d||
     or divided by tau_decr when ||r_d|| > mu ||r_p||, the scaled duals being multiplied by
     rho_old / rho_new.  Not available together with a tape, nor for trajectories of more than
     65535 * 128 segments (TOP_E_UNSUPPORTED).                                                     */
  int32_t check_every;       /* sweeps between checks; 0 disables checks (fixed rho, no stopping)    */
  int32_t adapt_rho;         /* 1: apply the penalty rule at every check                             */
  double tol;                /* E of the stopping test; <= 0 never stops (the paper uses 0.05)        */
  double mu;                 /* residual ratio that triggers a change (> 1; the paper uses 10)        */
  double tau_incr;           /* growth factor (> 1; the paper uses 1.1)                               */
  double tau_decr;           /* shrink factor (> 1; the paper uses 1.1)                               */
  /* Local update (Alg. 1): 0 = ClosedFormSolve; 1 = NumericSolve (Sec. III-C.3): the velocity bound
     as the general inequality g_s = max{0, |v_s|^2 - vmax^2}^2 = 0 with scaled multipliers, each
     segment's augmented Lagrangian minimised by lbfgs_iters L-BFGS iterations (memory 5, Armijo
     backtracking) from its previous c.  NumericSolve needs vmax, s = p and a box or no corridor,
     and takes no tape and no residual checks.                                                     */
  int32_t local_solve;
  int32_t lbfgs_iters;       /* L-BFGS iterations per local solve (>= 0; default 10)                 */
  int32_t vel_norm;          /* the speed bound at the samples: 2 (or 0): the Euclidean ball |v| <= vmax
                                (Sec. III-C.2); 4: the l4 ball (v_x^4 + v_y^4 + v_z^4)^(1/4) <= vmax, a
                                convex bound with no closed-form projection, NumericSolve only
                                (TOP_E_UNSUPPORTED otherwise), as h = ||v||_4 - vmax in g = max{0,h}^2 */
  int32_t lane_form;         /* lanes per segment of the sweep: 1, or 3 (one per axis: three times the
                                waves, for trajectories longer than a tile; tiles of at most 320
                                segments; n_cont < 2p-1, no polytope, no tape, no checks,
                                TOP_E_UNSUPPORTED otherwise; with NumericSolve four lanes, the three
                                axes and a spare, whose L-BFGS sums are reduced across the four);
                                0 picks 3 where allowed and either the local update is NumericSolve,
                                or some trajectory is longer than the largest one-lane tile, or, in
                                FP32 with no tile_lanes given, one lane per segment would make fewer
                                waves than half the device's SIMDs; else 1 (or the tuned form after
                                top_tune)                                                           */
  int32_t chain;             /* 0: where the plan has halo tiles and the device can hold all of them at
                                once, one top_iterate call runs all its sweeps in one cooperative
                                launch (lane_form 3 only): between epochs of halo sweeps each tile
                                publishes the core segments its neighbours copy and waits for theirs,
                                instead of ending the launch (the same results, bit for bit, without
                                one state reload per epoch); such calls are not captured into the
                                handle's graphs, and while the caller captures the stream the call
                                takes one launch per epoch instead.  1: one launch per epoch.         */
} top_options;

/* Fill *opt with the defaults: p = 3, s = p, pinned interior, M = 8, FP32, no tape, graph on,
   no checks (check_every = 0), and the paper's rule constants tol = 0.05, mu = 10,
   tau_incr = tau_decr = 1.1 for when checks are switched on; closed-form local update, Euclidean
   speed bound. */
void top_default_options(top_options* opt);

/* Bytes of workspace a problem of n_traj trajectories and n_seg_total segments needs, for
 * top_create with these options (NULL: the defaults) when a corridor, a velocity bound and end
 * states are all given (less is needed without them; top_create checks the exact amount).  The
 * workspace holds everything Algorithm 1 keeps per problem: the per-segment factors of eq.
 * QpSubProblem, the iterate (c, z, u and the slack/dual pairs of Sec. III-C) in two buffers, the
 * residual and cost partials of Sec. III-D.3, and with checkpoint_every > 0 the tape and the
 * reverse pass's buffers.  Host-only: no device call.  Returns 0 for invalid arguments
 * (top_last_error says why). */
size_t top_workspace_bytes(int32_t n_traj, int64_t n_seg_total, const top_options* opt);

/* The same for top_create_polytope with n_faces faces per segment (the faces and the per-axis
 * factors of the rotated solve take the place of the box). */
size_t top_workspace_bytes_polytope(int32_t n_traj, int64_t n_seg_total, int32_t n_faces,
                                    const top_options* opt);

/* Create a problem and run Init (Algorithm 1) on `stream`.
 *   n_traj       B >= 1
 *   seg_offsets  [host] int64 [B+1], seg_offsets[0] = 0, strictly increasing (every trajectory
 *                has at least one segment)
 *   waypoints    [dev] [S+B][3] path points P (Alg. 1 input)
 *   durations    [dev] [S] segment durations T_i > 0 (Sec. III-A)
 *   bc           [dev] [B][2][p][3] end states sigma_0, sigma_N (position and derivatives up to
 *                p-1, eq. start_points_constraints), or NULL for rest at the end waypoints.  The
 *                position rows must equal the end waypoints when fix_interior is set.
 *   box_lo/hi    [dev] [S][3] axis-aligned corridor per segment (the K = 6 polytope of
 *                Sec. III-D.1), or both NULL for no corridor; lo < hi
 *   vmax         [dev] [B] velocity-norm bound per trajectory (Sec. III-C.2), > 0, or NULL
 *   rho          [dev] [B] penalty per trajectory, > 0
 *   opt          [host] options, NULL for the defaults
 *   workspace    [dev] caller-owned device memory for the problem's state, workspace_bytes long
 *                (any alignment; at most top_workspace_bytes(...) is used), or NULL with
 *                workspace_bytes = 0 for the library's own pool.  TOP_E_WORKSPACE, before any
 *                device work, when workspace_bytes is below what this problem needs.
 *   stream       HIP stream all work of this handle is queued on (0 = the null stream)
 *   out          receives the handle; set to NULL on failure
 * Blocks once, to validate the device inputs. */
top_status top_create(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                      const double* durations, const double* bc, const double* box_lo,
                      const double* box_hi, const double* vmax, const double* rho,
                      const top_options* opt, void* workspace, size_t workspace_bytes,
                      hipStream_t stream, top_problem** out);

/* top_create with a general convex polytope corridor per segment instead of a box: the
 * H-representation P_i^H = {x : a_k . x <= b_k} of Sec. III-D.1, imposed at the M samples
 * (M * n_faces rows per segment, eq. linear_inequality).
 *   n_faces  K in [1, 8] faces per segment (segments with fewer faces pad with a = 0, b = 1)
 *   faces    [dev] float64 [S][K][4]: a_x, a_y, a_z, b of each face, finite
 * The other arguments are those of top_create.  The axes are coupled through sum_k a_k a_k^T; the
 * library solves per segment in the frame of its eigenvectors.  Not available with a tape
 * (checkpoint_every > 0): TOP_E_UNSUPPORTED. */
top_status top_create_polytope(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                               const double* durations, const double* bc, int32_t n_faces, const double* faces,
                               const double* vmax, const double* rho, const top_options* opt,
                               void* workspace, size_t workspace_bytes, hipStream_t stream,
                               top_problem** out);

/* Queue k >= 0 more sweeps, each one ADMM iteration of Sec. III-D.1 (eqs. QpSubProblem,
 * DynamicProject, UpdateCloseW, UpdateZ, NonNegativeProject, UpdateV, UpdateU), with the residuals of
 * Sec. III-D.3 and eq. UpdateRho at the checks when check_every > 0.
 * Trajectories that passed the stopping test are left unchanged.  Asynchronous. */
top_status top_iterate(top_problem* h, int32_t k);

/* Like top_iterate(h, k) with k >= 1, launched directly (no graph), then blocks and stores in *ms
 * [host] the device time from the first to the last sweep launch (outputs excluded), measured
 * with HIP events on the handle's stream.  For benchmarking. */
top_status top_time_sweeps(top_problem* h, int32_t k, float* ms);

/* [dev] float64 [B] outputs: ||r_p|| and ||r_d|| of the last sweep (eqs. splitting_primal_residual
 * and splitting_dual_residual, the dual residual read per segment as rho M~(T_i)^T (z~^{k+1}-z~^k)).
 * Either pointer may be NULL.  TOP_E_STATE before the first sweep. */
top_status top_residuals(const top_problem* h, double* r_primal, double* r_dual);

/* [dev] float64 [B]: the objective sum_i c_i^T Q~(T_i) c_i of the last local solves (Sec. III-D.1). */
top_status top_cost(const top_problem* h, double* cost);

/* [dev] float64 [S][3][2p]: the last local solves c_i (the output C of Algorithm 1), monomial
 * coefficients in ascending powers of the segment-local time; after 0 sweeps, the Init guess. */
top_status top_coeffs(const top_problem* h, double* coeffs);

/* Reverse-mode derivative of sum_b dcost[b] * J_b (J from top_cost after all sweeps so far) with
 * respect to the waypoints and durations, through Init and every sweep; corridor, vmax, rho and bc
 * are held constant.  Needs checkpoint_every > 0 and at most max_taped_iters sweeps so far.
 *   dcost       [dev] float64 [B]
 *   dwaypoints  [dev] float64 [S+B][3] (overwritten), or NULL
 *   ddurations  [dev] float64 [S] (overwritten), or NULL
 * TOP_E_STATE without a tape or after too many sweeps.  The block replays run on a second stream of
 * the device (default priority, created on first use and shared by all handles), joined back into
 * the handle's stream before any reverse step that needs them; the call is asynchronous on the
 * handle's stream like the others. */
top_status top_backward(top_problem* h, const double* dcost, double* dwaypoints, double* ddurations);

/* Time the candidate tile shapes on this problem (k_probe sweeps each, on scratch state, leaving the
 * iterate untouched), keep the fastest and remember it for problems of the same shape class.
 * Blocks.  A tile shape given explicitly in the options is not overridden.  A candidate that would
 * run as a chained launch (see top_options.chain) is timed as one, on a copy of the iterate in a
 * state-sized block taken from the library's pool for the call (also for a handle on a caller's
 * workspace) and kept in the pool afterwards; TOP_E_NOMEM if it cannot be had. */
top_status top_tune(top_problem* h, int32_t k_probe);

/* Per-trajectory outcome of the checks (Sec. III-D.3), written on the handle's stream:
 *   iters  [dev] int32 [B]: sweeps applied to each trajectory (where it stopped, else all so far)
 *   rho    [dev] float64 [B]: its current penalty (the input rho when adapt_rho is off)
 *   done   [dev] uint8 [B]: 1 if it passed the stopping test
 * Any pointer may be NULL.  Without checks every trajectory reports all sweeps, its input rho
 * and 0. */
top_status top_convergence(const top_problem* h, int32_t* iters, double* rho, uint8_t* done);

/* Block on the stream; TOP_E_NONFINITE if any sweep so far produced a non-finite value;
 * TOP_E_HIP if a tile of a chained launch gave up waiting for a neighbour (about a second: the
 * device did not run all tiles at once after all; the iterate is then wrong). */
top_status top_sync_status(top_problem* h);

/* Copy of the iterate state (checkpoint and resume), in the iterate precision (float or double),
 * structure of arrays: n_fields rows of ld elements (top_plan_info), row f, segment i at f * ld + i;
 * columns S..ld-1 are padding (zero unless a set state put other values there; never read).
 * Rows, with s = n_cont, M = 8, n = 2p, per axis a = 0..2 and order o < s, sample j < M:
 *   z_R  (end knot of the segment, orders 0..s-1)      rows a*s + o
 *   u_L, u_R (scaled consensus duals, start / end knot)  rows 3s + a*s + o, 6s + a*s + o
 *   box: y_hi, y_lo folded corridor pairs               rows 9s + a*M + j, 9s + 3M + a*M + j
 *   polytope: y of face k                                rows 9s + k*M + j
 *   closed form with vmax: g (folded velocity pair)      rows C + a*M + j
 *   NumericSolve: w_j, then the last c~ (c~_k = c_k T^k) rows C + j, C + M + a*n + k
 * where C = 9s plus the corridor rows.  A folded pair y stands for the slack max(0, -y) and the
 * scaled dual max(0, y); g for the split value Proj(g) and the scaled dual g - Proj(g).
 *   state  [dev] n_fields * ld elements (written by top_get_state, read by top_set_state)
 * top_set_state replaces the iterate (the next sweep starts from it); cost, residuals and
 * coefficients keep describing the last sweep until another one runs.  Both are queued on the
 * handle's stream. */
top_status top_get_state(const top_problem* h, void* state);
top_status top_set_state(top_problem* h, const void* state);

/* Execution plan actually in use (host struct). */
typedef struct top_plan_info {
  int32_t tile_lanes;        /* segments per workgroup tile (3x as many lanes with lane_form 3) */
  int32_t n_tiles;           /* workgroups per launch                                       */
  int32_t halo;              /* sweeps per launch when some trajectory is split, else 0     */
  int32_t n_traj;
  int64_t n_seg;
  int64_t used_lanes;        /* lanes holding a segment, halo copies included               */
  int32_t precision;
  int32_t order;
  int32_t n_cont;
  int32_t iters_done;        /* sweeps run since top_create                                 */
  int32_t n_fields;          /* rows of the iterate state (see top_get_state)               */
  int64_t ld;                /* elements per state row, n_seg rounded up to a multiple of 64 */
  int32_t lane_form;         /* lanes per segment of the sweep launches: 1 or 3                */
  int32_t chained;           /* 1: an iterate call of more than halo sweeps runs as one chained
                                launch (see top_options.chain)                                  */
  int32_t tail_tiles;        /* tiles of the tail launch that follows each sweep launch (0: none):
                                when nothing is split and the tiles would leave a last round of
                                the device holding only a few of them, those tiles' trajectories
                                run there instead, one lane per segment and axis where that form
                                takes the variant and options, else in the plan's own form on
                                tiles of at most half the width; not with a tape, residual
                                checks or NumericSolve                                          */
  int32_t tail_tile_lanes;   /* segments per tail tile                                          */
} top_plan_info;

top_status top_get_plan(const top_problem* h, top_plan_info* info);

/* Host only (touches no device; for callers that inspect or check the tiling): the tile plan
 * top_create builds for these trajectory lengths at a given tile width, halo and tail, the batching of
 * the per-segment solves of one sweep (Sec. III-D.1, Alg. 1: the segments' local updates of an
 * iteration are independent of each other) into workgroup tiles.
 *   n_traj, seg_offsets  as top_create
 *   tile_lanes   segments per tile, a multiple of 64 in [64, 512]
 *   halo         1 <= halo < tile_lanes / 2: segment copies on each side a split trajectory's tile
 *                keeps, and the sweeps per launch
 *   tiles_per_round  tiles the device holds at once (top_create asks the runtime), or 0 for no tail
 *   tail_tile_lanes  widest tail tile, a multiple of 64 in [64, 320] (ignored when
 *                tiles_per_round is 0).  When no trajectory is split and the tiles would leave a
 *                last round of k <= tiles_per_round / 8 tiles, the trajectories of the k tiles whose
 *                longest trajectory is shortest (then the least filled) are repacked, first-fit
 *                decreasing, into tail tiles as wide as that longest trajectory rounded up to 64
 *                (none if that exceeds tail_tile_lanes), for a second launch (top_create runs it
 *                with one lane per segment and axis where that form takes the variant)
 *   lanes        [host] int32 [n_tiles][tile_lanes] then [tail_tiles][tail_tile_lanes], or NULL: per
 *                lane its segment (global index), | TOP_HALO_BIT for a halo copy, -1 for an idle
 *                lane.  Trajectories of at most tile_lanes segments share tiles, packed first-fit
 *                in decreasing length; longer ones run over consecutive tiles whose core segments
 *                partition the trajectory
 *   chain        [host] int32 [n_tiles][4], or NULL: per tile the left and right tile holding its halo
 *                copies in their cores (-1 none) and its core lane range [lo, hi); the plan chains
 *                (info->chained = 1) only when every halo copy, and the start knot of its segment,
 *                is in a neighbour's published edge (within halo of a core edge, one more on the
 *                right), else the table is empty
 *   lanes_cap, chain_cap  entries the caller's arrays hold (n_tiles * tile_lanes + tail_tiles *
 *                tail_tile_lanes and 4 * n_tiles suffice; call once with NULL arrays and read info
 *                to size them)
 *   info         [host] tile_lanes, n_tiles (main launch), halo (0 if no trajectory is split),
 *                n_traj, n_seg, used_lanes (both launches), chained, tail_tiles and
 *                tail_tile_lanes; the other fields are 0
 * TOP_E_INVALID for bad offsets or sizes, or arrays smaller than the plan (nothing written to
 * them then). */
#define TOP_HALO_BIT (1 << 30)
top_status top_plan_tiles(int32_t n_traj, const int64_t* seg_offsets, int32_t tile_lanes, int32_t halo,
                          int32_t tiles_per_round, int32_t tail_tile_lanes, int32_t* lanes, int64_t lanes_cap,
                          int32_t* chain, int64_t chain_cap, top_plan_info* info);

/* Release the handle; NULL is a no-op.  Handles that captured graphs wait for their stream first;
 * others return at once.  A handle on a caller's workspace leaves the workspace
 * to the caller (see the device-memory convention above).  A handle on the library's pool returns
 * its buffers there without waiting for the work still queued on its stream: a later handle on the
 * same stream reuses them in stream order, one on another stream first waits (on the device) for
 * that work. */
void top_destroy(top_problem* h);

/* Free the device memory the library keeps for reuse: pool blocks no handle holds, and cached shape
 * tables and lane maps no handle uses.  Blocks until the device has finished the work that last
 * used them.  Handles stay valid. */
void top_trim(void);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): one whole solve -- top_create, top_iterate(k), then
 * top_residuals, top_cost and top_coeffs into the given buffers -- whose device memory (the problem's
 * state, its shape tables and tile lane map) is a fixed array of TOP_STATIC_SCRATCH_BYTES compiled into
 * the library, one copy per device, held until the process ends.  The call makes no hipMalloc or
 * other device allocation, no pinned host allocation and no graph.
 *   arguments    as top_create (box corridor or none; no workspace) and top_iterate; k >= 0
 *   coeffs       [dev] float64 [S][3][2p], or NULL
 *   cost         [dev] float64 [B], or NULL
 *   r_primal/r_dual  [dev] float64 [B], or NULL (both NULL when k = 0: TOP_E_STATE otherwise)
 * Options: a tape (checkpoint_every > 0) is TOP_E_UNSUPPORTED; use_graph and chain are ignored (no
 * graph, one launch per epoch).  A problem whose buffers exceed the scratch returns TOP_E_WORKSPACE
 * before any device work (about 2.0 KB per segment in float64, 1.05 KB in float32, for quintic box +
 * velocity: some 8,000 or 15,000 segments).
 * Blocks until the outputs are written and returns TOP_E_NONFINITE like top_sync_status.  Every
 * call on a device shares that device's copy of the array (one per process), which keeps what the
 * last call left; a call writes everything it reads first.  Calls that overlapped on one device
 * would race on the array: the library serialises them with a per-device lock, and each call waits
 * for its own work before it returns. */
#define TOP_STATIC_SCRATCH_BYTES (16u << 20)
top_status top_solve_static(int32_t n_traj, const int64_t* seg_offsets, const double* waypoints,
                            const double* durations, const double* bc, const double* box_lo,
                            const double* box_hi, const double* vmax, const double* rho,
                            const top_options* opt, int32_t k, double* coeffs, double* cost,
                            double* r_primal, double* r_dual, hipStream_t stream);

/* Thread-local text of the last error reported by this library on the calling thread. */
const char* top_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TOP_H_ */
