"""Adaptive penalty and the stopping test around the closed-form iteration.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sources (Sec. III-D.3 of the paper):
* stopping test, eq. ``splitting_tolerance``: a trajectory of N segments has
  converged once ||r_p||^2 < (N E)^2 and ||r_d||^2 < (N E)^2 (the paper
  recommends E = 0.05);
* penalty update, eq. ``UpdateRho``: rho grows by tau_incr when ||r_p|| exceeds
  mu ||r_d||, shrinks by tau_decr when ||r_d|| exceeds mu ||r_p||, and is kept
  otherwise (the paper uses mu = 10, tau_incr = tau_decr = 1.1);
* Algorithm 1: the residuals of an iteration are formed after its consensus
  step, the penalty update is the last step of the loop body, and the loop
  ends once both residual tests pass (the printed ``while`` condition is read
  as "until", as the surrounding text states).

Readings where the paper is silent:
* the residual test and the penalty update run every ``check_every``
  iterations, counted from Init (``check_every = 1`` is the paper's
  schedule); rho is constant between checks;
* a trajectory that passes the test stops there: its result is the local
  solve of that iteration and no penalty update follows it;
* when rho changes, the scaled duals u, v, w are multiplied by
  rho_old / rho_new, so the unscaled multipliers rho u, rho v, rho w carry
  over unchanged; s, phi, z and c are kept;
* every trajectory has its own rho and its own stopping point, so each one is
  run on its own here.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np
import torch

from . import cadmm
from .polynomial import DT


@dataclass
class AdaptiveResult:
    c: torch.Tensor          # [S, 3n] result local solve of every trajectory
    J: torch.Tensor          # [B] cost of c
    rp: torch.Tensor         # [B] ||r_p|| of each trajectory's last iteration
    rd: torch.Tensor         # [B] ||r_d|| of each trajectory's last iteration
    rho: torch.Tensor        # [B] rho after the last update
    iters: np.ndarray        # [B] iterations applied
    converged: np.ndarray    # [B] bool, stopped by the residual test


def subproblem(pr: cadmm.Problem, b: int) -> cadmm.Problem:
    """Trajectory b of a batch as a problem of its own."""
    s0, s1 = int(pr.seg_offsets[b]), int(pr.seg_offsets[b + 1])
    n = s1 - s0
    seg = slice(s0, s1)
    opt = lambda a, sl: None if a is None else a[sl]
    return cadmm.Problem(
        p=pr.p, s=pr.s, d=pr.d, n_samples=pr.n_samples, fix_interior=pr.fix_interior,
        seg_offsets=np.array([0, n], dtype=np.int64), traj=torch.zeros(n, dtype=torch.long),
        first=pr.first[seg], last=pr.last[seg], knot_l=torch.arange(n), knot_r=torch.arange(n) + 1,
        P=pr.P[s0 + b:s1 + b + 1], T=pr.T[seg], lo=opt(pr.lo, seg), hi=opt(pr.hi, seg),
        vmax=opt(pr.vmax, slice(b, b + 1)), rho=pr.rho[b:b + 1].clone(), bc=opt(pr.bc, slice(b, b + 1)),
        faces=opt(pr.faces, seg))


def factor(pr: cadmm.Problem, mats: dict) -> torch.Tensor:
    """Cholesky factor of the local system matrix at the problem's current rho."""
    return torch.linalg.cholesky(cadmm.system_matrix(pr, mats))


def rescale_duals(st: cadmm.State, ratio: float) -> cadmm.State:
    """Scaled duals after rho -> rho / ratio: u, v, w times ratio (unscaled multipliers unchanged)."""
    return replace(st, u=st.u * ratio, v=None if st.v is None else st.v * ratio,
                   w=None if st.w is None else st.w * ratio)


def update_rho(rho: float, rp: float, rd: float, mu: float, tau_incr: float, tau_decr: float) -> float:
    """Eq. UpdateRho."""
    if rp > mu * rd:
        return rho * tau_incr
    if rd > mu * rp:
        return rho / tau_decr
    return rho


def run_adaptive(pr: cadmm.Problem, K: int, check_every: int = 1, adapt: bool = True, eps: float = 0.05,
                 mu: float = 10.0, tau_incr: float = 1.1, tau_decr: float = 1.1) -> AdaptiveResult:
    """At most K iterations per trajectory with the residual test (eps > 0) and the penalty update."""
    if check_every < 1:
        raise ValueError("check_every must be >= 1")
    cs, J, rp, rd, rho = [], [], [], [], []
    iters = np.zeros(pr.B, dtype=np.int64)
    conv = np.zeros(pr.B, dtype=bool)
    for b in range(pr.B):
        q = subproblem(pr, b)
        mats = cadmm.segment_matrices(q)
        chol = factor(q, mats)
        st = cadmm.init_state(q, mats)
        rp2 = rd2 = torch.full((1,), float("nan"), dtype=DT)
        tol2 = (q.S * eps) ** 2
        k = 0
        while k < K:
            st, rp2, rd2 = cadmm.iterate(q, mats, chol, st)
            k += 1
            if k % check_every != 0:
                continue
            if eps > 0 and rp2.item() < tol2 and rd2.item() < tol2:
                conv[b] = True
                break
            if adapt:
                old = q.rho.item()
                new = update_rho(old, float(np.sqrt(rp2.item())), float(np.sqrt(rd2.item())), mu,
                                 tau_incr, tau_decr)
                if new != old:
                    st = rescale_duals(st, old / new)
                    q.rho = torch.tensor([new], dtype=DT)
                    chol = factor(q, mats)
        iters[b] = k
        cs.append(st.c)
        J.append(cadmm.cost(q, st.c))
        rp.append(torch.sqrt(rp2))
        rd.append(torch.sqrt(rd2))
        rho.append(q.rho.clone())
    return AdaptiveResult(c=torch.cat(cs, 0), J=torch.cat(J), rp=torch.cat(rp), rd=torch.cat(rd),
                          rho=torch.cat(rho), iters=iters, converged=conv)
