"""Shared helpers of the parity tests: run a workload through the C ABI and through the oracle."""
from __future__ import annotations

import numpy as np
import torch

from oracle import cadmm


def gpu_available() -> bool:
    return torch.cuda.is_available()


def run_gpu(w, K, precision=None, **kw):
    """Coefficients [S,3,n], cost [B], ||r_p|| [B], ||r_d|| [B] from the HIP library (numpy)."""
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, precision=precision or w.precision, **kw)
    try:
        prob.iterate(K)
        c = prob.coeffs()
        J = prob.cost()
        rp, rd = prob.residuals() if K > 0 else (None, None)
        prob.sync_status()
        torch.cuda.synchronize()
        out = (c.cpu().numpy(), J.cpu().numpy(),
               None if rp is None else rp.cpu().numpy(), None if rd is None else rd.cpu().numpy())
        return out
    finally:
        prob.close()


def run_oracle(w, K):
    pr = cadmm.problem_from_workload(w)
    res = cadmm.run(pr, K)
    c = cadmm.coeffs_by_axis(pr, res.c).numpy()
    return c, res.J.numpy(), res.rp.numpy(), res.rd.numpy()


def per_traj_rel(w, a, b):
    """max over trajectories of ||a_b - b_b||_F / ||b_b||_F over each trajectory's coefficients."""
    worst = 0.0
    for t in range(w.n_traj):
        s0, s1 = int(w.seg_offsets[t]), int(w.seg_offsets[t + 1])
        num = np.linalg.norm(a[s0:s1] - b[s0:s1])
        den = np.linalg.norm(b[s0:s1])
        worst = max(worst, num / den)
    return worst


def worst_segment(a, b):
    """(max over segments i of ||a_i - b_i|| / ||b_i||, that i) for coefficient arrays [S, 3, n]."""
    num = np.linalg.norm((a - b).reshape(a.shape[0], -1), axis=1)
    den = np.linalg.norm(b.reshape(b.shape[0], -1), axis=1)
    r = num / den
    i = int(np.argmax(r))
    return float(r[i]), i


def rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b)))
