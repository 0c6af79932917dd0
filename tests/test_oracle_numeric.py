"""Pins of the NumericSolve oracle (no GPU).

* its gradient agrees with central differences of its objective;
* without a velocity bound (box rows only) the local problem is the
  closed-form quadratic, so L-BFGS must land on the closed-form solve (itself
  pinned by stationarity and an independent least-squares solve), and whole
  runs must agree with the closed-form iteration;
* with the bound active its local minimiser equals scipy's BFGS on the same
  objective (pins the L-BFGS steps);
* on a tiny velocity-active problem its iterates move toward the constrained
  optimum of an independent SQP solve: the violation of the bound shrinks and
  the cost rises toward the optimum from below (the squared hinge has a zero
  gradient on the boundary, so this approach is slow, as the paper reports for
  the numeric update).

The same local pins cover the l4 speed bound ||v||_4 <= vmax (a convex bound
with no closed-form projection, h_j = ||v_j||_4 - vmax), plus its excess h_j
checked against velocities evaluated with numpy polynomials at the sample
instants.
"""
import pytest
import numpy as np
import scipy.optimize
import torch

from oracle import cadmm, numeric, references
from oracle.polynomial import beta
from paper_2507_10290_amd.workloads import random_walk_batch

DT = torch.float64


def _mid_run_state(w, K=5, wscale=0.3, seed=3):
    pr = cadmm.problem_from_workload(w)
    mats = cadmm.segment_matrices(pr)
    res = cadmm.run(pr, K)
    st = numeric.NumState(base=res.state, w=None)
    if pr.vmax is not None:
        g = torch.Generator().manual_seed(seed)
        st.w = wscale * torch.rand(pr.S, pr.n_samples, generator=g, dtype=DT)
    return pr, mats, st


@pytest.mark.parametrize("norm,vmax,scale", [(2, 1.0, 0.1), (4, 0.7, 0.03)])
def test_gradient_matches_central_differences(norm, vmax, scale):
    # (the l4 case keeps the excess moderate: a large objective would drown the differences in rounding)
    w = random_walk_batch("numgrad", [3], [5], order=3, vmax=vmax, rho=1.5, precision="fp64")
    pr, mats, st = _mid_run_state(w)
    c = st.base.c + scale * torch.randn(st.base.c.shape, generator=torch.Generator().manual_seed(1), dtype=DT)
    vel = (mats["Av"] @ c[:, None, :, None])[..., 0]
    assert (numeric.velocity_excess(vel, pr.vmax[0], norm)[0] > 0).sum() >= 3   # the bound term is active
    _, G = numeric.objective(pr, mats, st, c, norm)
    h = 1e-6
    for k in [0, 3, 7, 11, 17]:
        e = torch.zeros_like(c)
        e[:, k] = h
        Lp, _ = numeric.objective(pr, mats, st, c + e, norm)
        Lm, _ = numeric.objective(pr, mats, st, c - e, norm)
        fd = (Lp - Lm) / (2 * h)
        assert torch.allclose(fd, G[:, k], rtol=1e-6, atol=1e-6), (k, fd, G[:, k])


@pytest.mark.parametrize("norm", [2, 4])
def test_velocity_excess_matches_numpy_polynomials(norm):
    # h_j = |v(t_j)|^2 - vmax^2 (q = 2) or ||v(t_j)||_4 - vmax (q = 4), with v from numpy's polynomial
    # derivative at t_j = j T / (M + 1) and the norm from numpy.linalg.norm
    w = random_walk_batch("numexc", [3, 2], [21, 22], order=3, vmax=1.3, rho=1.0, precision="fp64")
    pr = cadmm.problem_from_workload(w)
    mats = cadmm.segment_matrices(pr)
    c = torch.randn(pr.S, 3 * pr.n, generator=torch.Generator().manual_seed(4), dtype=DT)
    vel = (mats["Av"] @ c[:, None, :, None])[..., 0]
    h, dh = numeric.velocity_excess(vel, pr.vmax[pr.traj][:, None], norm)
    T, vmax = w.durations, w.vmax
    cc = c.numpy().reshape(pr.S, 3, pr.n)
    traj = pr.traj.numpy()
    for i in range(pr.S):
        for j in range(pr.n_samples):
            t = (j + 1) * T[i] / (pr.n_samples + 1)
            v = np.array([np.polynomial.polynomial.polyval(t, np.polynomial.polynomial.polyder(cc[i, a]))
                          for a in range(3)])
            hf = (lambda x: np.linalg.norm(x) ** 2 - vmax[traj[i]] ** 2) if norm == 2 else \
                 (lambda x: np.linalg.norm(x, ord=4) - vmax[traj[i]])
            want = hf(v)
            assert abs(h[i, j].item() - want) <= 1e-12 * (1 + abs(want)), (i, j)
            # dh/dv by central differences of the same numpy expression
            for a in range(3):
                e = np.zeros(3)
                e[a] = 1e-6
                fd = (hf(v + e) - hf(v - e)) / 2e-6
                # rounding of the differenced values: ~1e-16 of |h| over the 2e-6 step
                tol = 1e-6 * (1 + abs(fd)) + 1e-9 * (1 + abs(want))
                assert abs(dh[i, j, a].item() - fd) <= tol


def test_box_only_local_problem_gives_the_closed_form_solve():
    w = random_walk_batch("numfree", [4, 3], [6, 7], order=3, vmax=None, rho=[1.0, 2.0], precision="fp64")
    pr, mats, st = _mid_run_state(w)
    c = numeric.lbfgs(pr, mats, st, st.base.c, inner=500)
    chol = torch.linalg.cholesky(cadmm.system_matrix(pr, mats))
    c_cf = cadmm.qp_subproblem(pr, chol, mats, st.base)
    assert (c - c_cf).abs().max().item() < 1e-8 * (1 + c_cf.abs().max().item())


def test_box_only_runs_match_the_closed_form_iteration():
    w = random_walk_batch("numrun", [5], [8], order=3, vmax=None, rho=1.0, precision="fp64")
    pr = cadmm.problem_from_workload(w)
    a = numeric.run(pr, 6, inner=500)
    b = cadmm.run(pr, 6)
    # each local solve stops about 1e-8 from its minimiser (see the test above); six sweeps carry it
    assert (a.c - b.c).abs().max().item() < 2e-6 * (1 + b.c.abs().max().item())


@pytest.mark.parametrize("norm", [2, 4])
def test_active_bound_local_minimiser_matches_scipy_bfgs(norm):
    w = random_walk_batch("numact", [2], [9], order=3, vmax=0.8, rho=2.0, precision="fp64")
    pr, mats, st = _mid_run_state(w)
    c = numeric.lbfgs(pr, mats, st, st.base.c, inner=400, norm=norm)
    for i in range(pr.S):
        def f(x):
            cc = st.base.c.clone()
            cc[i] = torch.tensor(x, dtype=DT)
            L, G = numeric.objective(pr, mats, st, cc, norm)
            return L[i].item(), G[i].numpy()
        r = scipy.optimize.minimize(f, st.base.c[i].numpy(), jac=True, method="BFGS",
                                    options={"gtol": 1e-11, "maxiter": 5000})
        assert np.abs(c[i].numpy() - r.x).max() < 1e-6 * (1 + np.abs(r.x).max()), (i, r.message)
    # the velocity term is active at that minimiser (otherwise this pins nothing new)
    vel = (mats["Av"] @ c[:, None, :, None])[..., 0]
    assert (numeric.velocity_excess(vel, pr.vmax[0], norm)[0] > 0).any()


def test_numeric_iteration_moves_toward_the_constrained_optimum():
    w = random_walk_batch("numopt", [2], [11], order=3, vmax=10.0, rho=20.0, precision="fp64", dur=(1.0, 2.0))
    w.box_lo = np.minimum(w.waypoints[:-1], w.waypoints[1:]) - 1.0
    w.box_hi = np.maximum(w.waypoints[:-1], w.waypoints[1:]) + 1.0
    pr = cadmm.problem_from_workload(w)
    ck, Jk = references.kkt_reference(pr)
    ts = cadmm.sample_times(pr).numpy()
    peak = max(np.linalg.norm(ck[i] @ beta(1, torch.tensor(ts[i, j]), pr.d).numpy())
               for i in range(pr.S) for j in range(pr.n_samples))
    w.vmax[:] = 0.97 * peak
    pr = cadmm.problem_from_workload(w)
    c_ref, J_ref, res_sqp = references.constrained_reference(pr, tol=1e-12)
    assert res_sqp.status == 0 and J_ref[0] > Jk[0] * 1.05       # the bound binds
    mats = cadmm.segment_matrices(pr)
    st = numeric.init_state(pr, mats)
    hist = []
    for k in range(1, 601):
        st, _, _ = numeric.iterate(pr, mats, st, 10)
        if k in (150, 600):
            vel = (mats["Av"] @ st.base.c[:, None, :, None])[..., 0]
            viol = (torch.sqrt((vel * vel).sum(2)) - pr.vmax[0]).max().item()
            hist.append((cadmm.cost(pr, st.base.c).item(), viol))
    (J1, v1), (J2, v2) = hist
    assert 0 < v2 < v1
    assert J1 < J2 < J_ref[0]
