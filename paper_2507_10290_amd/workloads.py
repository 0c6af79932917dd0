"""Seeded synthetic workloads for the consensus-ADMM trajectory sweep.

This module only draws random inputs; it holds none of the method's
arithmetic, so both the GPU library and the CPU oracle can take their inputs
from it.

The paper's own inputs (RRT* paths through a forest, FIRI corridors, a sampled
parametric curve; Sec. III-D and Sec. IV) are not available.  These generators
stand in for them with the same structure:

* a path P of N+1 waypoints in R^3 (Alg. 1 input) drawn as a random walk with
  step lengths U[lo, hi] metres and uniformly random unit directions;
* per-segment durations T_i > 0 (Sec. III-A): either step / 2 m/s or drawn
  U[0.3, 1.5] s independently of the step;
* an axis-aligned box corridor per segment (the K = 6 half-space polytope of
  Sec. III-D), built around the segment's chord: per axis
  lo = min(P_{i-1}, P_i) - h, hi = max(P_{i-1}, P_i) + h, h ~ U[0.3, 1.0];
* or, instead of the box, a general convex polytope per segment (the
  H-representation P_i^H = {x : a_k . x <= b_k, k = 1..K} of Sec. III-D.1):
  the six faces of a randomly rotated box around the chord plus K - 6 random
  cuts, each offset h ~ U[0.3, 1.0] beyond the farther chord end, so both
  waypoints lie strictly inside and consecutive polytopes overlap;
* a velocity-norm bound v_max (the quadratic constraint of Sec. III-C.2);
* a penalty rho per trajectory.

Batched workloads concatenate trajectories in CSR form: trajectory b owns
segments seg_offsets[b] .. seg_offsets[b+1]-1 and waypoint rows
seg_offsets[b] + b .. seg_offsets[b+1] + b (N_b + 1 points).

Draw order inside one trajectory (fixed, so every consumer sees the same
numbers): step lengths (N), directions (N x 3 normals), independent durations
(N, only when requested), box half-widths (N x 3, only when boxes are on);
for polytopes, per segment in order: a 3 x 3 normal matrix (rotation by QR),
(K - 6) x 3 normals of the extra cuts, K offsets.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Workload:
    """One batch of trajectories, all arrays float64 on the host."""

    name: str
    order: int                      # p: 3 = minimum jerk, 4 = minimum snap
    n_cont: int                     # s: orders 0..s-1 shared at interior knots
    n_samples: int                  # M: constraint sample points per segment
    fix_interior: bool              # interior waypoint positions pinned
    seg_offsets: np.ndarray         # int64 [B+1]
    waypoints: np.ndarray           # [S+B, 3]
    durations: np.ndarray           # [S]
    box_lo: Optional[np.ndarray]    # [S, 3] or None
    box_hi: Optional[np.ndarray]    # [S, 3] or None
    vmax: Optional[np.ndarray]      # [B] or None
    rho: np.ndarray                 # [B]
    iters: int                      # fixed iteration count K of the workload
    precision: str = "fp64"         # iterate precision the workload is quoted in
    bc: Optional[np.ndarray] = None  # [B, 2, p, 3] end states, None = rest-to-rest
    notes: str = ""
    faces: Optional[np.ndarray] = None  # [S, K, 4] polytope corridor a . x <= b (rows a_x, a_y, a_z, b)

    @property
    def n_traj(self) -> int:
        return int(self.seg_offsets.shape[0] - 1)

    @property
    def n_seg(self) -> int:
        return int(self.seg_offsets[-1])

    def traj_lengths(self) -> np.ndarray:
        return np.diff(self.seg_offsets)

    def subset(self, trajs: Sequence[int], name: Optional[str] = None) -> "Workload":
        """The same inputs restricted to the listed trajectories (in that order)."""
        offs = [0]
        wp, du, lo, hi, fc = [], [], [], [], []
        for b in trajs:
            s0, s1 = int(self.seg_offsets[b]), int(self.seg_offsets[b + 1])
            offs.append(offs[-1] + (s1 - s0))
            wp.append(self.waypoints[s0 + b: s1 + b + 1])
            du.append(self.durations[s0:s1])
            if self.box_lo is not None:
                lo.append(self.box_lo[s0:s1])
                hi.append(self.box_hi[s0:s1])
            if self.faces is not None:
                fc.append(self.faces[s0:s1])
        idx = np.asarray(list(trajs), dtype=np.int64)
        return Workload(
            name=name or f"{self.name}[subset]",
            order=self.order, n_cont=self.n_cont, n_samples=self.n_samples,
            fix_interior=self.fix_interior,
            seg_offsets=np.asarray(offs, dtype=np.int64),
            waypoints=np.concatenate(wp, 0), durations=np.concatenate(du, 0),
            box_lo=np.concatenate(lo, 0) if lo else None,
            box_hi=np.concatenate(hi, 0) if hi else None,
            vmax=None if self.vmax is None else self.vmax[idx].copy(),
            rho=self.rho[idx].copy(), iters=self.iters, precision=self.precision,
            bc=None if self.bc is None else self.bc[idx].copy(), notes=self.notes,
            faces=np.concatenate(fc, 0) if fc else None)

    def window(self, traj: int, seg_lo: int, seg_hi: int, name: Optional[str] = None) -> "Workload":
        """Segments seg_lo..seg_hi-1 (local indices) of one trajectory as a trajectory of its own.

        Its end knots become rest end states at the window's first and last
        waypoints.  After K sweeps, a segment more than K segments away from
        both window ends has exactly the same iterate as in the full
        trajectory, because one sweep couples a segment only to its two
        neighbours.
        """
        s0 = int(self.seg_offsets[traj])
        a, b = s0 + seg_lo, s0 + seg_hi
        return Workload(
            name=name or f"{self.name}[t{traj}:{seg_lo}:{seg_hi}]",
            order=self.order, n_cont=self.n_cont, n_samples=self.n_samples,
            fix_interior=self.fix_interior,
            seg_offsets=np.asarray([0, seg_hi - seg_lo], dtype=np.int64),
            waypoints=self.waypoints[a + traj: b + traj + 1].copy(),
            durations=self.durations[a:b].copy(),
            box_lo=None if self.box_lo is None else self.box_lo[a:b].copy(),
            box_hi=None if self.box_hi is None else self.box_hi[a:b].copy(),
            vmax=None if self.vmax is None else self.vmax[[traj]].copy(),
            rho=self.rho[[traj]].copy(), iters=self.iters, precision=self.precision,
            bc=None, notes="light-cone window",
            faces=None if self.faces is None else self.faces[a:b].copy())


def _unit_dirs(rng: np.random.Generator, n: int) -> np.ndarray:
    d = rng.standard_normal((n, 3))
    nrm = np.linalg.norm(d, axis=1, keepdims=True)
    nrm[nrm == 0.0] = 1.0
    return d / nrm


def _one_walk(rng: np.random.Generator, n: int, step: Sequence[float],
              dur: Optional[Sequence[float]], speed: float, box: bool):
    L = rng.uniform(step[0], step[1], n)
    dirs = _unit_dirs(rng, n)
    P = np.zeros((n + 1, 3))
    P[1:] = np.cumsum(L[:, None] * dirs, axis=0)
    if dur is None:
        T = L / speed
    else:
        T = rng.uniform(dur[0], dur[1], n)
    lo = hi = None
    if box:
        h = rng.uniform(0.3, 1.0, (n, 3))
        lo = np.minimum(P[:-1], P[1:]) - h
        hi = np.maximum(P[:-1], P[1:]) + h
    return P, T, lo, hi


def _polytopes(rng: np.random.Generator, P: np.ndarray, K: int) -> np.ndarray:
    """[N, K, 4] half-spaces around each chord P[i] -> P[i+1]: a rotated box plus K - 6 cuts."""
    n = P.shape[0] - 1
    out = np.zeros((n, K, 4))
    for i in range(n):
        Rm, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        normals = [Rm[:, a] for a in range(3)] + [-Rm[:, a] for a in range(3)]
        normals += list(_unit_dirs(rng, K - 6))
        h = rng.uniform(0.3, 1.0, K)
        for k, a in enumerate(normals):
            out[i, k, :3] = a
            out[i, k, 3] = max(a @ P[i], a @ P[i + 1]) + h[k]
    return out


def random_walk_batch(name: str, lengths: Sequence[int], seeds: Sequence, *, order: int = 3,
                      n_cont: int = 0, n_samples: int = 8, step=(1.0, 3.0), dur=None,
                      speed: float = 2.0, box: bool = True, vmax: Optional[float] = 3.0,
                      rho=1.0, iters: int = 200, precision: str = "fp32",
                      fix_interior: bool = True, faces: int = 0) -> Workload:
    """A batch of independent random-walk trajectories, one seed per trajectory.

    faces = K >= 6 replaces the box corridor by a K-face polytope per segment."""
    lengths = [int(n) for n in lengths]
    if any(n < 1 for n in lengths):
        raise ValueError("every trajectory needs at least one segment")
    if faces and faces < 6:
        raise ValueError("a polytope corridor needs at least 6 faces")
    if faces:
        box = False
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lengths)
    wp, du, lo, hi, fc = [], [], [], [], []
    for n, sd in zip(lengths, seeds):
        rng = np.random.Generator(np.random.PCG64(sd))
        P, T, l, h = _one_walk(rng, n, step, dur, speed, box)
        wp.append(P)
        du.append(T)
        if box:
            lo.append(l)
            hi.append(h)
        if faces:
            fc.append(_polytopes(rng, P, faces))
    B = len(lengths)
    rho_arr = np.broadcast_to(np.asarray(rho, dtype=np.float64), (B,)).copy()
    return Workload(
        name=name, order=order, n_cont=n_cont or order, n_samples=n_samples,
        fix_interior=fix_interior, seg_offsets=offs,
        waypoints=np.concatenate(wp, 0), durations=np.concatenate(du, 0),
        box_lo=np.concatenate(lo, 0) if box else None,
        box_hi=np.concatenate(hi, 0) if box else None,
        vmax=None if vmax is None else np.full(B, float(vmax)),
        rho=rho_arr, iters=iters, precision=precision,
        faces=np.concatenate(fc, 0) if faces else None)


# ---------------------------------------------------------------------------
# The five benchmark workloads.  Sizes and distributions are the ones the
# benchmark definitions fix; the seeds are 0..4.
# ---------------------------------------------------------------------------

CONFIG_NAMES = {
    0: "plain-N8-quintic-fp64-unconstrained",
    1: "single-N1024-quintic-box-vel",
    2: "single-N65536-septic-box-vel",
    3: "batched-B4096-quintic-box-vel",
    4: "grad-B256xN128-quintic-box-vel",
    5: "batched-B4096-quintic-poly8-vel",
}


def make_config(i: int, *, scale: Optional[float] = None, n_traj: Optional[int] = None) -> Workload:
    """Benchmark workload i (0..4).

    ``scale`` shrinks single-trajectory segment counts (configs 1, 2) and
    ``n_traj`` takes the first trajectories of the batched ones (configs 3, 4);
    both are for tests that need the same distributions at smaller sizes.
    """
    if i == 0:
        return random_walk_batch(CONFIG_NAMES[0], [8], [0], order=3, box=False, vmax=None,
                                 rho=1.0, iters=200, precision="fp64")
    if i == 1:
        n = 1024 if scale is None else max(2, int(1024 * scale))
        return random_walk_batch(CONFIG_NAMES[1], [n], [1], order=3, rho=1.0, iters=500,
                                 precision="fp32")
    if i == 2:
        n = 65536 if scale is None else max(2, int(65536 * scale))
        return random_walk_batch(CONFIG_NAMES[2], [n], [2], order=4, step=(0.5, 2.0),
                                 dur=(0.3, 1.5), rho=1.0, iters=300, precision="fp32")
    if i == 3:
        parent = np.random.Generator(np.random.PCG64(3))
        B = 4096
        lengths = parent.integers(8, 512, size=B, endpoint=True)
        rhos = parent.choice(np.array([0.5, 1.0, 2.0]), size=B)
        seeds = np.random.SeedSequence(3).spawn(B)
        if n_traj is not None:
            lengths, rhos, seeds = lengths[:n_traj], rhos[:n_traj], seeds[:n_traj]
        return random_walk_batch(CONFIG_NAMES[3], lengths, seeds, order=3, rho=rhos,
                                 iters=200, precision="fp32")
    if i == 4:
        B = 256 if n_traj is None else n_traj
        seeds = np.random.SeedSequence(4).spawn(256)[:B]
        return random_walk_batch(CONFIG_NAMES[4], [128] * B, seeds, order=3, rho=1.0,
                                 iters=100, precision="fp32")
    if i == 5:
        # the batched workload with 8-face polytope corridors instead of boxes (general corridor form)
        parent = np.random.Generator(np.random.PCG64(3))
        B = 4096
        lengths = parent.integers(8, 512, size=B, endpoint=True)
        rhos = parent.choice(np.array([0.5, 1.0, 2.0]), size=B)
        seeds = np.random.SeedSequence(5).spawn(B)
        if n_traj is not None:
            lengths, rhos, seeds = lengths[:n_traj], rhos[:n_traj], seeds[:n_traj]
        return random_walk_batch(CONFIG_NAMES[5], lengths, seeds, order=3, rho=rhos, iters=200,
                                 precision="fp32", faces=8)
    raise ValueError(f"no workload {i}")


# ---------------------------------------------------------------------------
# Segment-count scaling study (Sec. IV): points sampled from a parametric curve.
# ---------------------------------------------------------------------------

CURVE_PERIOD = 2.0 * np.pi


def curve(theta: np.ndarray, order: int = 0) -> np.ndarray:
    """A smooth closed 3-D curve (a trefoil knot) and its derivatives w.r.t. theta: [len(theta), 3]."""
    th = np.asarray(theta, dtype=np.float64)
    # x = sin t + 2 sin 2t, y = cos t - 2 cos 2t, z = -sin 3t; each term a sin/cos with a known derivative
    terms = [(0, 1.0, 1, "s"), (0, 2.0, 2, "s"), (1, 1.0, 1, "c"), (1, -2.0, 2, "c"), (2, -1.0, 3, "s")]
    out = np.zeros(th.shape + (3,))
    for ax, amp, f, kind in terms:
        # d^o/dt^o sin(f t) = f^o sin(f t + o pi/2); cos(f t) = sin(f t + pi/2)
        phase = (np.pi / 2 if kind == "c" else 0.0) + order * np.pi / 2
        out[..., ax] += amp * f ** order * np.sin(f * th + phase)
    return out


def curve_workload(n_seg: int, *, order: int = 3, total_time: float = 20.0, rho: float = 1.0,
                   iters: int = 1000, precision: str = "fp32", n_turns: float = 1.0) -> Workload:
    """N + 1 points sampled uniformly in the curve parameter, uniform durations, pinned interior
    points, end states from the curve's own derivatives (time t = theta * total_time / span), no
    corridor and no velocity bound: the trajectory must pass through the sampled points."""
    span = CURVE_PERIOD * n_turns
    theta = np.linspace(0.0, span, n_seg + 1)
    P = curve(theta)
    T = np.full(n_seg, total_time / n_seg)
    dth = span / total_time                     # d theta / dt
    bc = np.zeros((1, 2, order, 3))
    for side, th in ((0, theta[0]), (1, theta[-1])):
        for o in range(order):
            bc[0, side, o] = curve(np.array([th]), o)[0] * dth ** o
    return Workload(name=f"curve-N{n_seg}", order=order, n_cont=order, n_samples=8, fix_interior=True,
                    seg_offsets=np.array([0, n_seg], dtype=np.int64), waypoints=P, durations=T,
                    box_lo=None, box_hi=None, vmax=None, rho=np.array([float(rho)]), iters=iters,
                    precision=precision, bc=bc, notes=f"trefoil, {n_turns} turn(s) in {total_time} s")


def config_summary(w: Workload) -> dict:
    L = w.traj_lengths()
    return {"workload": w.name, "n_traj": w.n_traj, "n_seg": w.n_seg,
            "seg_per_traj": [int(L.min()), int(L.max())], "order": w.order,
            "n_cont": w.n_cont, "n_samples": w.n_samples, "iters": w.iters,
            "box": w.box_lo is not None, "vmax": None if w.vmax is None else float(w.vmax[0]),
            "precision": w.precision}
