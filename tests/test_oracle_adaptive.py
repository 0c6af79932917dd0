"""Pins of the adaptive-penalty / stopping oracle (no GPU).

* with the update off and no stopping it reduces to the fixed-rho iteration;
* its stopping point is the first check at which the fixed-rho run, restarted
  from Init for that many iterations, passes the paper's test (brute force);
* its dual rescaling agrees with an ADMM written in unscaled multipliers, where
  a change of rho needs no rescaling at all (an independent derivation);
* with the update on it still converges to the global KKT optimum.
"""
import numpy as np
import pytest
import torch

from oracle import adaptive, cadmm, references
from paper_2507_10290_amd.workloads import random_walk_batch

DT = torch.float64


def _batch(box=True, vel=True, rho=1.0, lens=(3, 5, 4), seeds=(71, 72, 73), order=3):
    return random_walk_batch("adapt", list(lens), list(seeds), order=order, box=box,
                             vmax=3.0 if vel else None, rho=rho, precision="fp64")


def _rel(a, b):
    return float(torch.linalg.norm(a - b) / torch.linalg.norm(b))


def test_no_update_no_stop_is_the_fixed_rho_run():
    w = _batch(rho=[1.0, 0.5, 2.0])
    pr = cadmm.problem_from_workload(w)
    K = 40
    ad = adaptive.run_adaptive(pr, K, check_every=1, adapt=False, eps=0.0)
    ref = cadmm.run(pr, K)
    assert _rel(ad.c, ref.c) < 1e-13
    assert _rel(ad.J, ref.J) < 1e-13
    assert _rel(ad.rp, ref.rp) < 1e-12 and _rel(ad.rd, ref.rd) < 1e-12
    assert np.all(ad.iters == K) and not ad.converged.any()
    assert torch.equal(ad.rho, pr.rho)


def test_stopping_point_by_brute_force():
    w = _batch(lens=(5, 4), seeds=(72, 73), rho=[1.0, 2.0])
    pr = cadmm.problem_from_workload(w)
    ce, K = 25, 1000
    ad = adaptive.run_adaptive(pr, K, check_every=ce, adapt=False, eps=0.15)
    assert ad.converged.all(), ad.iters
    for b in range(pr.B):
        q = adaptive.subproblem(pr, b)
        first = None
        for k in range(ce, K + 1, ce):
            if bool(cadmm.converged_flag(q, cadmm.run(q, k), eps=0.15)[0]):
                first = k
                break
        assert first == ad.iters[b], (b, first, ad.iters[b])
        s0, s1 = pr.seg_offsets[b], pr.seg_offsets[b + 1]
        assert _rel(ad.c[s0:s1], cadmm.run(q, first).c) < 1e-13


def _unscaled_run(q, rhos):
    """ADMM on the same splitting with unscaled multipliers lam, nu, om; rhos[k] is rho of iteration k+1."""
    mats = cadmm.segment_matrices(q)
    st = cadmm.init_state(q, mats)        # multipliers start at zero, as the scaled duals do
    z, s, phi = st.z, st.s, st.phi
    lam = torch.zeros_like(st.u)
    nu = torch.zeros_like(st.v)
    om = torch.zeros_like(st.w)
    Mt, Ao, bb, Av = mats["Mt"], mats["Ao"], mats["b"], mats["Av"]
    vmax = q.vmax[q.traj][:, None, None]
    out = []
    for rho in rhos:
        q.rho = torch.tensor([rho], dtype=DT)
        H = cadmm.system_matrix(q, mats)
        # stationarity of c^T Q c + lam^T(Mc - z) + rho/2|Mc - z|^2 + nu^T(Ac - b + s) + rho/2|Ac - b + s|^2
        #                + om^T(A^v c - phi) + rho/2|A^v c - phi|^2
        rhs = (Mt.transpose(1, 2) @ (rho * cadmm.knot_pair(q, z) - lam)[:, :, None])[..., 0]
        rhs = rhs + (Ao.transpose(1, 2) @ (rho * (bb - s) - nu)[:, :, None])[..., 0]
        rhs = rhs + torch.einsum("smai,sma->si", Av, rho * phi - om)
        c = torch.linalg.solve(H, rhs[:, :, None])[..., 0]
        vel = (Av @ c[:, None, :, None])[..., 0]
        phi = cadmm.project_ball(vel + om / rho, vmax)
        om = om + rho * (vel - phi)
        z = cadmm.knot_average(q, c, z)
        Ac = (Ao @ c[:, :, None])[..., 0]
        s = torch.clamp(-(Ac - bb + nu / rho), min=0.0)
        nu = nu + rho * (Ac + s - bb)
        lam = lam + rho * ((Mt @ c[:, :, None])[..., 0] - cadmm.knot_pair(q, z))
        out.append(c)
    return out


def test_dual_rescaling_matches_unscaled_multipliers():
    w = _batch(lens=(5,), seeds=(81,))
    pr = cadmm.problem_from_workload(w)
    changes = {6: 2.0, 11: 0.4, 15: 1.1}      # rho from the next iteration on
    K = 22
    rhos, r = [], 1.0
    for k in range(1, K + 1):
        rhos.append(r)
        r = changes.get(k, r)
    ref = _unscaled_run(adaptive.subproblem(pr, 0), rhos)

    q = adaptive.subproblem(pr, 0)
    mats = cadmm.segment_matrices(q)
    chol = adaptive.factor(q, mats)
    st = cadmm.init_state(q, mats)
    for k in range(1, K + 1):
        st, _, _ = cadmm.iterate(q, mats, chol, st)
        assert _rel(st.c, ref[k - 1]) < 1e-11, k
        if k in changes:
            old, new = q.rho.item(), changes[k]
            st = adaptive.rescale_duals(st, old / new)
            q.rho = torch.tensor([new], dtype=DT)
            chol = adaptive.factor(q, mats)
    # without the rescaling the two runs part after the first change
    q = adaptive.subproblem(pr, 0)
    chol = adaptive.factor(q, mats)
    st = cadmm.init_state(q, mats)
    worst = 0.0
    for k in range(1, K + 1):
        st, _, _ = cadmm.iterate(q, mats, chol, st)
        worst = max(worst, _rel(st.c, ref[k - 1]))
        if k in changes:
            q.rho = torch.tensor([changes[k]], dtype=DT)
            chol = adaptive.factor(q, mats)
    assert worst > 1e-4


def test_update_rule_cases():
    assert adaptive.update_rho(1.0, 11.0, 1.0, 10.0, 1.1, 1.1) == 1.1
    assert adaptive.update_rho(1.0, 1.0, 11.0, 10.0, 1.1, 1.1) == 1.0 / 1.1
    assert adaptive.update_rho(2.0, 9.0, 1.0, 10.0, 1.1, 1.1) == 2.0
    assert adaptive.update_rho(2.0, 1.0, 9.0, 10.0, 1.5, 3.0) == 2.0


def test_adaptive_run_reaches_the_kkt_optimum():
    # from a large rho^0 the dual residual dominates, so the rule lowers rho on the way
    w = random_walk_batch("adapt-kkt", [3], [91], order=3, box=False, vmax=None, rho=30.0, precision="fp64")
    pr = cadmm.problem_from_workload(w)
    ad = adaptive.run_adaptive(pr, 8000, check_every=1, adapt=True, eps=1e-5)
    assert ad.converged[0]
    assert ad.rho.item() < 30.0
    ck, Jk = references.kkt_reference(pr)
    ref = torch.tensor(ck, dtype=DT)
    assert _rel(cadmm.coeffs_by_axis(pr, ad.c), ref) < 1e-3
    assert abs(ad.J.item() - Jk[0]) / Jk[0] < 1e-3
