"""The same CADMM iteration with each slack/dual pair folded into one stored value.

Used only to pin the algebra that the GPU library relies on; not a second
reference for the GPU.  With y := A^o c^{k+1} - b + v^k, eqs.
``NonNegativeProject`` and ``UpdateV`` give s^{k+1} = max(0, -y) and
v^{k+1} = max(0, y), hence b - s - v = b - |y|.  With g := A^v c^{k+1} + w^k,
eqs. ``DynamicProject`` and ``UpdateCloseW`` give phi = Proj(g), w = g - Proj(g),
hence phi - w = 2 Proj(g) - g.  The recursions become
y^{k+1} = A^o c^{k+1} - b + max(0, y^k) and g^{k+1} = A^v c^{k+1} + g^k - Proj(g^k).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import torch

from . import cadmm
from .cadmm import Problem, project_ball


@dataclass
class MinState:
    c: torch.Tensor
    z: torch.Tensor
    u: torch.Tensor
    y: Optional[torch.Tensor]
    g: Optional[torch.Tensor]


def from_paper_state(st: cadmm.State, mats: dict) -> MinState:
    """y = v - s (so s = max(0,-y), v = max(0,y) when complementary); g = phi + w."""
    y = None if st.s is None else st.v - st.s
    g = None if st.phi is None else st.phi + st.w
    return MinState(c=st.c, z=st.z, u=st.u, y=y, g=g)


def iterate(pr: Problem, mats: dict, chol: torch.Tensor, st: MinState) -> MinState:
    rho = pr.rho[pr.traj][:, None]
    rhs = (mats["Mt"].transpose(1, 2) @ (cadmm.knot_pair(pr, st.z) - st.u)[:, :, None])[..., 0]
    if st.y is not None:
        rhs = rhs + (mats["Ao"].transpose(1, 2) @ (mats["b"] - st.y.abs())[:, :, None])[..., 0]
    pg = None
    if st.g is not None:
        pg = project_ball(st.g, pr.vmax[pr.traj][:, None, None])
        rhs = rhs + torch.einsum("smai,sma->si", mats["Av"], 2.0 * pg - st.g)
    c = torch.cholesky_solve((rho * rhs)[:, :, None], chol)[..., 0]
    z = cadmm.knot_average(pr, c, st.z)
    u = st.u + (mats["Mt"] @ c[:, :, None])[..., 0] - cadmm.knot_pair(pr, z)
    y = g = None
    if st.y is not None:
        y = (mats["Ao"] @ c[:, :, None])[..., 0] - mats["b"] + torch.clamp(st.y, min=0.0)
    if st.g is not None:
        g = (mats["Av"] @ c[:, None, :, None])[..., 0] + st.g - pg
    return MinState(c=c, z=z, u=u, y=y, g=g)


def run(pr: Problem, K: int):
    mats, chol = cadmm.setup(pr)
    st = from_paper_state(cadmm.init_state(pr, mats), mats)
    for _ in range(K):
        st = iterate(pr, mats, chol, st)
    return st, cadmm.cost(pr, st.c)
