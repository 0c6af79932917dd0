"""Algorithm 1 (TOP) with the closed-form local update, in the paper's variables.

Sources (Sec. III of the paper):
* consensus reformulation and the scaled-dual CADMM iteration: Sec. III-B,
  eqs. ``Consensus_problem``, ``Consensus_augmented_Lagrangian_problem``,
  ``Consensus_update``;
* corridor as linear inequalities with slack s and dual v: Sec. III-C.1
  (slack update) and the per-segment polytope P_i^H of Sec. III-D.1, either
  an axis-aligned box (lo, hi) or general half-spaces a_k . x <= b_k, each
  imposed at the M sample instants (M K rows);
* velocity ball as a quadratic inequality with split variable phi and dual w:
  Sec. III-C.2 (closed-form projection);
* the per-segment closed-form update rules: Sec. III-D.1, eqs.
  ``QpSubProblem``, ``UpdateZ``, ``UpdateU``, ``NonNegativeProject``,
  ``UpdateV``, ``DynamicProject``, ``UpdateCloseW``;
* stopping residuals: Sec. III-D.3, eqs. ``splitting_primal_residual`` and
  ``splitting_dual_residual``.

One iteration is the scaled-form ADMM pass those equations define: minimise
each segment's augmented Lagrangian over c (with the velocity split's
projection and dual step right after it, since they need only the new c),
then the knot averages, the residuals of the new iterate, the corridor slacks,
and the dual steps that use the new c, z and slacks.

Readings taken where the paper is silent or inconsistent (each is listed with
its justification in the design notes of the repository):
* the right-hand side of ``QpSubProblem`` carries the factor rho, as setting
  the gradient of the segment's augmented Lagrangian to zero gives;
* consensus is on derivative orders 0..s-1 at interior knots (s = p by
  default); end knots constrain orders 0..p-1 and are never updated;
* interior knot positions are pinned to the waypoints when
  ``fix_interior`` (the paper's own variant leaves them free and averages
  them; both are supported);
* constraint samples sit at t_j = j T / (M+1), j = 1..M;
* Init: each segment starts on its chord as the rest-to-rest step polynomial,
  z^0 holds the waypoint positions with zero higher derivatives, all scaled
  duals start at zero, s^0 = max(0, b - A^o c^0), phi^0 = Proj(A^v c^0);
* rho is fixed per trajectory here; the stopping test and the adaptive-rho
  rule are applied around this iteration by ``adaptive``.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from .polynomial import DT, beta, boundary_map, cost_gram, knot_map, kron_axes, smoothstep_coeffs

M_AXES = 3


@dataclass
class Problem:
    """A batch of independent trajectories in the paper's matrices (float64, CPU)."""

    p: int
    s: int
    d: int
    n_samples: int
    fix_interior: bool
    seg_offsets: np.ndarray
    traj: torch.Tensor       # [S] trajectory index of each segment
    first: torch.Tensor      # [S] bool, first segment of its trajectory
    last: torch.Tensor       # [S] bool, last segment of its trajectory
    knot_l: torch.Tensor     # [S] knot index of the segment's start
    knot_r: torch.Tensor     # [S] knot index of the segment's end
    P: torch.Tensor          # [S+B, 3] path points (knots)
    T: torch.Tensor          # [S] durations
    lo: Optional[torch.Tensor]
    hi: Optional[torch.Tensor]
    vmax: Optional[torch.Tensor]   # [B]
    rho: torch.Tensor              # [B]
    bc: Optional[torch.Tensor]     # [B, 2, p, 3]
    faces: Optional[torch.Tensor] = None   # [S, K, 4] polytope corridor a . x <= b (instead of lo/hi)

    @property
    def S(self) -> int:
        return int(self.T.shape[0])

    @property
    def B(self) -> int:
        return int(self.seg_offsets.shape[0] - 1)

    @property
    def n(self) -> int:
        return self.d + 1


def problem_from_workload(w, P=None, T=None, s: Optional[int] = None,
                          fix_interior: Optional[bool] = None) -> Problem:
    """Build the oracle's problem from a ``Workload``; P and T may be given as tensors (autograd)."""
    offs = np.asarray(w.seg_offsets, dtype=np.int64)
    B = offs.shape[0] - 1
    lens = np.diff(offs)
    traj = np.repeat(np.arange(B), lens)
    S = int(offs[-1])
    local = np.arange(S) - offs[traj]
    first = local == 0
    last = local == (lens[traj] - 1)
    knot_l = np.arange(S) + traj
    p = int(w.order)
    s_ = int(s if s is not None else (w.n_cont or p))
    if P is None:
        P = torch.tensor(w.waypoints, dtype=DT)
    if T is None:
        T = torch.tensor(w.durations, dtype=DT)
    t = lambda a: None if a is None else torch.tensor(a, dtype=DT)
    return Problem(
        p=p, s=s_, d=2 * p - 1, n_samples=int(w.n_samples),
        fix_interior=bool(w.fix_interior if fix_interior is None else fix_interior),
        seg_offsets=offs, traj=torch.tensor(traj), first=torch.tensor(first),
        last=torch.tensor(last), knot_l=torch.tensor(knot_l), knot_r=torch.tensor(knot_l + 1),
        P=P, T=T, lo=t(w.box_lo), hi=t(w.box_hi), vmax=t(w.vmax), rho=t(w.rho), bc=t(w.bc),
        faces=t(getattr(w, "faces", None)))


# ---------------------------------------------------------------------------
# Per-segment matrices of Sec. III-D.1 (axis-major squeeze, m = 3).
# ---------------------------------------------------------------------------

def row_mask(pr: Problem) -> torch.Tensor:
    """[S, 2s] 1 where a boundary row exists: end knots carry only orders 0..p-1."""
    o = torch.arange(pr.s)
    left = (~pr.first[:, None]) | (o[None, :] < pr.p)
    right = (~pr.last[:, None]) | (o[None, :] < pr.p)
    return torch.cat([left, right], 1).to(DT)


def sample_times(pr: Problem) -> torch.Tensor:
    """[S, M] constraint sample instants T_ij = j T_i / (M+1), j = 1..M."""
    j = torch.arange(1, pr.n_samples + 1, dtype=DT)
    return pr.T[:, None] * j[None, :] / (pr.n_samples + 1)


def segment_matrices(pr: Problem) -> dict:
    """Q~, M~, A^o, b, A^v(T_ij) for every segment."""
    S, n, s, M = pr.S, pr.n, pr.s, pr.n_samples
    Qt = kron_axes(cost_gram(pr.T, pr.p, pr.d))                       # [S, 3n, 3n]
    Mrow = boundary_map(pr.T, s, s, pr.d) * row_mask(pr)[:, :, None]  # [S, 2s, n]
    Mt = kron_axes(Mrow)                                              # [S, 3*2s, 3n]
    out = {"Qt": Qt, "Mt": Mt, "Mrow": Mrow}
    ts = sample_times(pr)
    if pr.lo is not None:
        b0 = beta(0, ts, pr.d)                                        # [S, M, n]
        rows, rhs = [], []
        zero = torch.zeros(S, n, dtype=DT)
        for j in range(M):
            for a in range(M_AXES):
                e = torch.cat([b0[:, j, :] if q == a else zero for q in range(M_AXES)], 1)
                rows.append(e)                     # upper: beta^T c_a <= hi_a
                rhs.append(pr.hi[:, a])
                rows.append(-e)                    # lower: -beta^T c_a <= -lo_a
                rhs.append(-pr.lo[:, a])
        out["Ao"] = torch.stack(rows, 1)          # [S, 2*M*3, 3n]
        out["b"] = torch.stack(rhs, 1)            # [S, 2*M*3]
    if pr.faces is not None:
        # P_i^H sampled at the M instants: one row a_k^T sigma_i(T_ij) <= b_k per (sample j, face k)
        b0 = beta(0, ts, pr.d)                                        # [S, M, n]
        rows, rhs = [], []
        for j in range(M):
            for k in range(pr.faces.shape[1]):
                a = pr.faces[:, k, :3]                                # [S, 3]
                rows.append(torch.cat([a[:, q:q + 1] * b0[:, j, :] for q in range(M_AXES)], 1))
                rhs.append(pr.faces[:, k, 3])
        out["Ao"] = torch.stack(rows, 1)          # [S, M*K, 3n]
        out["b"] = torch.stack(rhs, 1)            # [S, M*K]
    if pr.vmax is not None:
        b1 = beta(1, ts, pr.d)                    # [S, M, n]
        out["Av"] = kron_axes(b1[:, :, None, :])  # [S, M, 3, 3n]
    return out


def system_matrix(pr: Problem, mats: dict) -> torch.Tensor:
    """2 Q~ + rho M~^T M~ + rho A^oT A^o + rho sum_j A^v(T_ij)^T A^v(T_ij) (eq. QpSubProblem)."""
    rho = pr.rho[pr.traj][:, None, None]
    Mt = mats["Mt"]
    H = 2.0 * mats["Qt"] + rho * Mt.transpose(1, 2) @ Mt
    if "Ao" in mats:
        H = H + rho * mats["Ao"].transpose(1, 2) @ mats["Ao"]
    if "Av" in mats:
        Av = mats["Av"]
        H = H + rho * torch.einsum("smai,smaj->sij", Av, Av)
    return H


def project_ball(x: torch.Tensor, vmax: torch.Tensor) -> torch.Tensor:
    """Projection onto ||phi||^2 <= vmax^2 (eq. DynamicProject): sqrt(max(||x||^2/vmax^2, 1)^-1) x."""
    nrm2 = (x * x).sum(-1, keepdim=True)
    scale = torch.sqrt(1.0 / torch.clamp(nrm2 / (vmax * vmax), min=1.0))
    return scale * x


# ---------------------------------------------------------------------------
# State and the update equations of Sec. III-D.1.
# ---------------------------------------------------------------------------

@dataclass
class State:
    c: torch.Tensor                  # [S, 3n]
    z: torch.Tensor                  # [S+B, 3, s] knot states
    u: torch.Tensor                  # [S, 3*2s] scaled consensus duals (M~ c layout)
    s: Optional[torch.Tensor]        # [S, 48] box slacks
    v: Optional[torch.Tensor]        # [S, 48] box scaled duals
    phi: Optional[torch.Tensor]      # [S, M, 3]
    w: Optional[torch.Tensor]        # [S, M, 3]


def end_states(pr: Problem) -> torch.Tensor:
    """[B, 2, p, 3] fixed end-knot states sigma_0, sigma_N: given, else rest at the end points."""
    if pr.bc is not None:
        return pr.bc
    B = pr.B
    starts = torch.tensor(pr.seg_offsets[:-1] + np.arange(B))
    ends = torch.tensor(pr.seg_offsets[1:] + np.arange(B))
    out = []
    for idx in (starts, ends):
        pos = pr.P[idx]                                       # [B, 3]
        rest = torch.zeros(B, pr.p - 1, M_AXES, dtype=DT)
        out.append(torch.cat([pos[:, None, :], rest], 1))     # [B, p, 3]
    return torch.stack(out, 1)


def initial_knots(pr: Problem) -> torch.Tensor:
    """z^0: waypoint positions with zero higher derivatives; end knots hold sigma_0 / sigma_N."""
    K = pr.P.shape[0]
    zpos = pr.P[:, :, None]                                              # [K, 3, 1]
    z = torch.cat([zpos, torch.zeros(K, M_AXES, pr.s - 1, dtype=DT)], 2)  # [K, 3, s]
    ends = end_states(pr)                                                # [B, 2, p, 3]
    B = pr.B
    starts = torch.tensor(pr.seg_offsets[:-1] + np.arange(B))
    stops = torch.tensor(pr.seg_offsets[1:] + np.arange(B))
    for idx, e in ((starts, ends[:, 0]), (stops, ends[:, 1])):
        val = torch.cat([e.transpose(1, 2), torch.zeros(B, M_AXES, pr.s - pr.p, dtype=DT)], 2)
        z = z.index_put((idx,), val)
    return z


def knot_pair(pr: Problem, z: torch.Tensor) -> torch.Tensor:
    """z~_i = (z_{i-1}, z_i) laid out like M~ c: per axis, the start knot's orders then the end knot's."""
    zl = z[pr.knot_l]             # [S, 3, s]
    zr = z[pr.knot_r]
    return torch.cat([zl, zr], 2).reshape(pr.S, -1) * row_mask(pr).repeat(1, M_AXES)


def init_state(pr: Problem, mats: dict) -> State:
    """The starting iterate (the paper leaves it open; reading stated in the module docstring)."""
    S, n, p = pr.S, pr.n, pr.p
    sc = torch.tensor([float(x) for x in smoothstep_coeffs(p)], dtype=DT)   # [n]
    P0 = pr.P[pr.knot_l]                                   # [S, 3]
    dP = pr.P[pr.knot_r] - P0
    powT = torch.stack([pr.T ** j for j in range(n)], 1)   # [S, n]
    c = dP[:, :, None] * (sc[None, None, :] / powT[:, None, :])
    c = c + torch.cat([P0[:, :, None], torch.zeros(S, M_AXES, n - 1, dtype=DT)], 2)
    c = c.reshape(S, M_AXES * n)
    z = initial_knots(pr)
    u = torch.zeros(S, M_AXES * 2 * pr.s, dtype=DT)
    s_ = v = phi = w = None
    if "Ao" in mats:
        s_ = torch.clamp(mats["b"] - (mats["Ao"] @ c[:, :, None])[..., 0], min=0.0)
        v = torch.zeros_like(s_)
    if "Av" in mats:
        vel = (mats["Av"] @ c[:, None, :, None])[..., 0]      # [S, M, 3]
        phi = project_ball(vel, pr.vmax[pr.traj][:, None, None])
        w = torch.zeros_like(phi)
    return State(c=c, z=z, u=u, s=s_, v=v, phi=phi, w=w)


def qp_subproblem(pr: Problem, chol: torch.Tensor, mats: dict, st: State) -> torch.Tensor:
    """Eq. QpSubProblem: the minimiser of each segment's augmented Lagrangian over its coefficients,
    (2Q~ + rho M~^T M~ + rho A^oT A^o + rho sum A^vT A^v) c = rho [M~^T (z~ - u) + A^oT (b - s - v)
    + sum A^vT (phi - w)], solved with the Cholesky factor of the left-hand matrix."""
    rho = pr.rho[pr.traj][:, None]
    rhs = (mats["Mt"].transpose(1, 2) @ (knot_pair(pr, st.z) - st.u)[:, :, None])[..., 0]
    if st.s is not None:
        rhs = rhs + (mats["Ao"].transpose(1, 2) @ (mats["b"] - st.s - st.v)[:, :, None])[..., 0]
    if st.phi is not None:
        rhs = rhs + torch.einsum("smai,sma->si", mats["Av"], st.phi - st.w)
    return torch.cholesky_solve((rho * rhs)[:, :, None], chol)[..., 0]


def velocity_split(pr: Problem, mats: dict, c: torch.Tensor, w: torch.Tensor):
    """Eqs. DynamicProject and UpdateCloseW: phi = Proj(A^v c + w) onto the ball |x| <= vmax, then
    w += A^v c - phi."""
    vel = (mats["Av"] @ c[:, None, :, None])[..., 0]
    phi = project_ball(vel + w, pr.vmax[pr.traj][:, None, None])
    return phi, w + vel - phi


def end_derivatives(pr: Problem, c: torch.Tensor):
    """x^L_i = beta~(0) c_i and x^R_i = beta~(T_i) c_i, each [S, 3, s]."""
    cc = c.reshape(pr.S, M_AXES, pr.n)
    kl = knot_map(torch.zeros_like(pr.T), pr.s, pr.d)     # [S, s, n]
    kr = knot_map(pr.T, pr.s, pr.d)
    xl = torch.einsum("son,san->sao", kl, cc)
    xr = torch.einsum("son,san->sao", kr, cc)
    return xl, xr


def interior(pr: Problem) -> torch.Tensor:
    """Indices of segments whose end knot is shared with a next segment."""
    return torch.nonzero(~pr.last)[:, 0]


def knot_average(pr: Problem, c: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
    """Eq. UpdateZ: z_i = (beta~(T_i) c_i + beta~(0) c_{i+1}) / 2 at interior knots (pinned orders keep
    their values)."""
    xl, xr = end_derivatives(pr, c)
    i = interior(pr)
    avg = 0.5 * (xr[i] + xl[i + 1])                       # [I, 3, s]
    free = torch.ones(pr.s, dtype=torch.bool)
    if pr.fix_interior:
        free[0] = False
    new = torch.where(free[None, None, :], avg, z[pr.knot_r[i]])
    return z.index_put((pr.knot_r[i],), new)


def residuals(pr: Problem, c: torch.Tensor, z_new: torch.Tensor, z_old: torch.Tensor):
    """Squared norms of eqs. splitting_primal_residual / splitting_dual_residual, per trajectory.

    The dual residual is read per segment, rho M~(T_i)^T (z~_i^{k+1} - z~_i^k),
    stacked over segments.
    """
    xl, xr = end_derivatives(pr, c)
    i = interior(pr)
    gap = ((xr[i] - xl[i + 1]) ** 2).sum((1, 2))
    rp2 = torch.zeros(pr.B, dtype=DT).index_add(0, pr.traj[i], gap)
    dz = knot_pair(pr, z_new) - knot_pair(pr, z_old)
    rho = pr.rho[pr.traj][:, None]
    Mt = kron_axes(boundary_map(pr.T, pr.s, pr.s, pr.d) * row_mask(pr)[:, :, None])
    rd_seg = ((rho * (Mt.transpose(1, 2) @ dz[:, :, None])[..., 0]) ** 2).sum(1)
    rd2 = torch.zeros(pr.B, dtype=DT).index_add(0, pr.traj, rd_seg)
    return rp2, rd2


def slack_projection(mats: dict, c: torch.Tensor, v: torch.Tensor) -> torch.Tensor:
    """Eq. NonNegativeProject: s = max(0, -(A^o c - b + v))."""
    Ac = (mats["Ao"] @ c[:, :, None])[..., 0]
    return torch.clamp(-(Ac - mats["b"] + v), min=0.0)


def scaled_dual_steps(pr: Problem, mats: dict, c, z_new, u, s_new, v):
    """Eq. UpdateU  u += M~ c - z~  and eq. UpdateV  v += A^o c + s - b."""
    u_new = u + (mats["Mt"] @ c[:, :, None])[..., 0] - knot_pair(pr, z_new)
    v_new = None
    if v is not None:
        v_new = v + (mats["Ao"] @ c[:, :, None])[..., 0] + s_new - mats["b"]
    return u_new, v_new


def cost(pr: Problem, c: torch.Tensor) -> torch.Tensor:
    """Objective per trajectory: sum_i c_i^T Q~(T_i) c_i (the minimum-effort cost with W = I)."""
    Qt = kron_axes(cost_gram(pr.T, pr.p, pr.d))
    per = torch.einsum("si,sij,sj->s", c, Qt, c)
    return torch.zeros(pr.B, dtype=DT).index_add(0, pr.traj, per)


@dataclass
class Result:
    c: torch.Tensor        # [S, 3n] last local solve, monomial coefficients
    J: torch.Tensor        # [B]
    rp: torch.Tensor       # [B] ||r_p|| of the last iteration
    rd: torch.Tensor       # [B] ||r_d|| of the last iteration
    state: State
    iters: int


def iterate(pr: Problem, mats: dict, chol: torch.Tensor, st: State):
    """One ADMM iteration with fixed rho (Sec. III-D.1); returns (new state, rp2, rd2).

    The coefficient minimisation comes first; everything after it depends on the new c: the
    velocity split (its projection and dual step), the knot averages, the residuals of the new
    iterate against the previous knots, the corridor slacks, and the consensus and corridor dual
    steps, which also use the new knots and slacks."""
    c = qp_subproblem(pr, chol, mats, st)
    phi, w = velocity_split(pr, mats, c, st.w) if st.phi is not None else (None, None)
    z = knot_average(pr, c, st.z)
    rp2, rd2 = residuals(pr, c, z, st.z)
    s_new = slack_projection(mats, c, st.v) if st.s is not None else None
    u, v = scaled_dual_steps(pr, mats, c, z, st.u, s_new, st.v)
    return State(c=c, z=z, u=u, s=s_new, v=v, phi=phi, w=w), rp2, rd2


def setup(pr: Problem):
    mats = segment_matrices(pr)
    H = system_matrix(pr, mats)
    chol = torch.linalg.cholesky(H)
    return mats, chol


def run(pr: Problem, K: int, state: Optional[State] = None, setup_out=None) -> Result:
    """K iterations from the starting iterate (or from ``state``): the iteration of Algorithm 1 with
    fixed rho and no stopping test."""
    mats, chol = setup_out if setup_out is not None else setup(pr)
    st = state if state is not None else init_state(pr, mats)
    rp2 = rd2 = torch.full((pr.B,), float("nan"), dtype=DT)
    for _ in range(K):
        st, rp2, rd2 = iterate(pr, mats, chol, st)
    return Result(c=st.c, J=cost(pr, st.c), rp=torch.sqrt(rp2), rd=torch.sqrt(rd2), state=st, iters=K)


def converged_flag(pr: Problem, res: Result, eps: float = 0.05) -> torch.Tensor:
    """Stopping test of eq. splitting_tolerance: ||r_p||^2 < (N eps)^2 and ||r_d||^2 < (N eps)^2."""
    N = torch.tensor(np.diff(pr.seg_offsets), dtype=DT)
    tol2 = (N * eps) ** 2
    return (res.rp ** 2 < tol2) & (res.rd ** 2 < tol2)


def coeffs_by_axis(pr: Problem, c: torch.Tensor) -> torch.Tensor:
    """[S, 3, n] view of the squeezed coefficients (axis, ascending power)."""
    return c.reshape(pr.S, M_AXES, pr.n)
