"""Algorithm 1 with the NumericSolve local update (Sec. III-C.3, general inequality constraints).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The velocity bound is treated as a general convex inequality: with
h_j(c) <= 0 a function of the velocity A^v(T_ij) c and g_j = max{0, h_j}^2 (eq. ``componentwise
maximum``) it becomes the equality g_j(c) = 0, kept in the segment's augmented
Lagrangian (eq. ``general_constraint_aug``) in scaled form; the box rows keep
their slack/dual pairs as in the closed form.  q = 2 is the Euclidean speed
ball of Sec. III-C.2 with h_j = |v_j|^2 - vmax^2 (which also has the closed-form
projection); q = 4 is the l4 ball ||v_j||_4 <= vmax with h_j = ||v_j||_4 - vmax,
a convex bound with no closed-form projection, which only this update handles.  One iteration of Alg. 1's
NumericSolve branch:

  c^{k+1} = argmin_c  c^T Q~ c + rho/2 |M~ c - z~ + u|^2 + rho/2 |A^o c - b + s + v|^2
                      + rho/2 sum_j (g_j(c) + w_j)^2
  w_j^{k+1} = w_j + g_j(c^{k+1})          (like the scaled consensus dual, eq. Consensus_dual_update)
  then the knot averages, residuals, slacks and dual steps as in ``cadmm`` (eqs. UpdateZ,
  splitting_*_residual, NonNegativeProject, UpdateU, UpdateV).

Readings (the paper names L-BFGS and nothing more):
* each local minimisation runs exactly ``inner`` L-BFGS iterations from the
  segment's previous c (warm start; Init's c^0 for the first sweep);
* L-BFGS as in Nocedal & Wright (two-loop recursion, Alg. 7.4) with memory
  ``mem`` pairs, H0 = gamma I with gamma = s^T y / y^T y of the newest pair
  (1 before any), a pair kept only when s^T y > 0; the history starts empty in
  every local solve;
* backtracking line search from step 1: accept the first step
  a in {1, 1/2, 1/4, ...} (at most ``trials``) with
  L(c + a d) <= L(c) + 1e-4 a grad^T d; if none is accepted the iteration makes
  no step and keeps no pair;
* w starts at zero.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import cadmm
from .polynomial import DT

C1 = 1e-4


@dataclass
class NumState:
    base: cadmm.State               # c, z, u, s, v (phi and w of the closed form unused)
    w: Optional[torch.Tensor]       # [S, M] scaled multipliers of g_j = 0


def velocity_excess(vel: torch.Tensor, vmax: torch.Tensor, norm: int = 2):
    """h_j at every sample (vel [S, M, 3]) and dh_j/dv_j.

    q = 2: h = |v|^2 - vmax^2 (the quadratic form of Sec. III-C.2).  q = 4: h = ||v||_4 - vmax, the
    norm itself (convex, smooth away from v = 0, where h < 0); its fourth power would make the squared
    hinge an eighth-degree polynomial in c, too steep for the line search from a far start."""
    if norm == 2:
        return (vel * vel).sum(2) - vmax * vmax, 2.0 * vel
    if norm == 4:
        v2 = vel * vel
        n4 = torch.sqrt(torch.sqrt((v2 * v2).sum(2)))                    # ||v||_4
        safe = torch.where(n4 > 0, n4, torch.ones_like(n4))
        dh = torch.where((n4 > 0)[..., None], vel * v2 / (safe * safe * safe)[..., None], torch.zeros_like(vel))
        return n4 - vmax, dh
    raise ValueError("norm must be 2 or 4")


def _parts(pr, mats, st: NumState):
    """The fixed data of one local problem per segment."""
    rho = pr.rho[pr.traj][:, None]
    zt = cadmm.knot_pair(pr, st.base.z) - st.base.u                   # M~ c should equal this
    bt = None
    if st.base.s is not None:
        bt = mats["b"] - st.base.s - st.base.v                        # A^o c should equal this
    return rho, zt, bt


def objective(pr, mats, st: NumState, c: torch.Tensor, norm: int = 2):
    """L_i(c) per segment and its gradient, c [S, 3n]; norm q of the velocity bound."""
    rho, zt, bt = _parts(pr, mats, st)
    Qc = (mats["Qt"] @ c[:, :, None])[..., 0]
    rM = (mats["Mt"] @ c[:, :, None])[..., 0] - zt
    L = (c * Qc).sum(1) + 0.5 * rho[:, 0] * (rM * rM).sum(1)
    G = 2.0 * Qc + rho * (mats["Mt"].transpose(1, 2) @ rM[:, :, None])[..., 0]
    if bt is not None:
        rA = (mats["Ao"] @ c[:, :, None])[..., 0] - bt
        L = L + 0.5 * rho[:, 0] * (rA * rA).sum(1)
        G = G + rho * (mats["Ao"].transpose(1, 2) @ rA[:, :, None])[..., 0]
    if st.w is not None:
        vel = (mats["Av"] @ c[:, None, :, None])[..., 0]              # [S, M, 3]
        vmax = pr.vmax[pr.traj][:, None]
        h, dh = velocity_excess(vel, vmax, norm)                      # [S, M], [S, M, 3]
        hp = torch.clamp(h, min=0.0)
        g = hp * hp
        e = g + st.w
        L = L + 0.5 * rho[:, 0] * (e * e).sum(1)
        # d/dc of rho/2 (g + w)^2 = rho (g + w) 2 max(0, h) A^v^T dh/dv
        coef = rho * e * 2.0 * hp                                     # [S, M]
        G = G + torch.einsum("sm,smai,sma->si", coef, mats["Av"], dh)
    return L, G


def lbfgs(pr, mats, st: NumState, c0: torch.Tensor, inner: int, mem: int = 5, trials: int = 20, norm: int = 2):
    """``inner`` L-BFGS iterations on every segment's L_i from c0 (readings in the module docstring)."""
    S, n3 = c0.shape
    c = c0.clone()
    L, G = objective(pr, mats, st, c, norm)
    Sh = torch.zeros(S, mem, n3, dtype=DT)
    Yh = torch.zeros(S, mem, n3, dtype=DT)
    Rh = torch.zeros(S, mem, dtype=DT)        # 1 / (s^T y); 0 marks an empty slot
    order = torch.zeros(S, mem, dtype=torch.long)   # slot of the i-th newest pair (i = 0 newest)
    count = torch.zeros(S, dtype=torch.long)
    gamma = torch.ones(S, dtype=DT)
    ar = torch.arange(S)
    for _ in range(inner):
        # two-loop recursion
        q = G.clone()
        alpha = torch.zeros(S, mem, dtype=DT)
        for i in range(mem):                     # newest to oldest
            slot = order[:, i]
            valid = i < count
            s_i, y_i, r_i = Sh[ar, slot], Yh[ar, slot], Rh[ar, slot]
            a_i = torch.where(valid, r_i * (s_i * q).sum(1), torch.zeros_like(r_i))
            alpha[:, i] = a_i
            q = q - a_i[:, None] * y_i
        r = gamma[:, None] * q
        for i in reversed(range(mem)):           # oldest to newest
            slot = order[:, i]
            valid = i < count
            s_i, y_i, r_i = Sh[ar, slot], Yh[ar, slot], Rh[ar, slot]
            b_i = torch.where(valid, r_i * (y_i * r).sum(1), torch.zeros_like(r_i))
            r = r + torch.where(valid[:, None], s_i * (alpha[:, i] - b_i)[:, None], torch.zeros_like(s_i))
        d = -r
        slope = (G * d).sum(1)
        # backtracking line search
        step = torch.zeros(S, dtype=DT)
        done = torch.zeros(S, dtype=torch.bool)
        a = torch.ones(S, dtype=DT)
        for _t in range(trials):
            Lt, _ = objective(pr, mats, st, c + a[:, None] * d, norm)
            ok = (~done) & (Lt <= L + C1 * a * slope)
            step = torch.where(ok, a, step)
            done = done | ok
            a = a * 0.5
        moved = step > 0
        c_new = c + step[:, None] * d
        L_new, G_new = objective(pr, mats, st, c_new, norm)
        s_vec = c_new - c
        y_vec = G_new - G
        sy = (s_vec * y_vec).sum(1)
        keep = moved & (sy > 0)
        # push the pair into the ring (the oldest slot is overwritten when full)
        new_slot = torch.where(count < mem, count, order[:, mem - 1])
        for b in torch.nonzero(keep)[:, 0].tolist():
            sl = int(new_slot[b])
            Sh[b, sl], Yh[b, sl], Rh[b, sl] = s_vec[b], y_vec[b], 1.0 / sy[b]
            prev = [int(x) for x in order[b, :min(int(count[b]), mem - 1)]]
            order[b, : len(prev) + 1] = torch.tensor([sl] + prev)
            count[b] = min(int(count[b]) + 1, mem)
            gamma[b] = sy[b] / (y_vec[b] * y_vec[b]).sum()
        c = torch.where(moved[:, None], c_new, c)
        L = torch.where(moved, L_new, L)
        G = torch.where(moved[:, None], G_new, G)
    return c


def init_state(pr, mats) -> NumState:
    base = cadmm.init_state(pr, mats)
    w = torch.zeros(pr.S, pr.n_samples, dtype=DT) if pr.vmax is not None else None
    return NumState(base=base, w=w)


def iterate(pr, mats, st: NumState, inner: int, norm: int = 2):
    """One iteration with the NumericSolve local minimisation in place of eq. QpSubProblem."""
    c = lbfgs(pr, mats, st, st.base.c, inner, norm=norm)
    w = None
    if st.w is not None:
        vel = (mats["Av"] @ c[:, None, :, None])[..., 0]
        vmax = pr.vmax[pr.traj][:, None]
        hp = torch.clamp(velocity_excess(vel, vmax, norm)[0], min=0.0)
        w = st.w + hp * hp
    z = cadmm.knot_average(pr, c, st.base.z)
    rp2, rd2 = cadmm.residuals(pr, c, z, st.base.z)
    s_new = cadmm.slack_projection(mats, c, st.base.v) if st.base.s is not None else None
    u, v = cadmm.scaled_dual_steps(pr, mats, c, z, st.base.u, s_new, st.base.v)
    base = cadmm.State(c=c, z=z, u=u, s=s_new, v=v, phi=None, w=None)
    return NumState(base=base, w=w), rp2, rd2


def run(pr, K: int, inner: int = 10, norm: int = 2) -> cadmm.Result:
    """K iterations with NumericSolve from the starting iterate; norm q of the velocity bound."""
    mats = cadmm.segment_matrices(pr)
    st = init_state(pr, mats)
    rp2 = rd2 = torch.full((pr.B,), float("nan"), dtype=DT)
    for _ in range(K):
        st, rp2, rd2 = iterate(pr, mats, st, inner, norm)
    return cadmm.Result(c=st.base.c, J=cadmm.cost(pr, st.base.c), rp=torch.sqrt(rp2), rd=torch.sqrt(rd2),
                        state=st.base, iters=K)
