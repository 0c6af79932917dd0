"""GPU NumericSolve sweep (L-BFGS local update, Sec. III-C.3) against the oracle's numeric iteration.

A few warm-started L-BFGS iterations per sweep make this iteration amplify rounding differences by
roughly 10^2-10^3 per sweep (the line search and the L-BFGS scaling are steep functions of their
inputs), so two correct implementations follow the same iterates only for a couple of sweeps.  The
tests therefore compare whole runs over two sweeps, and every later sweep one step at a time: the
GPU state after K sweeps (top_get_state) is handed to the oracle, which takes one step from it, and
that step must equal the GPU's sweep K + 1.  Even one step amplifies input rounding strongly, so the
bar for each step is measured on the oracle itself: ten times the change of the oracle's own step
when its input state is jittered by a few units of the iterate precision (relative 1e-14 for
float64, 1e-6 for float32), and never tighter than 1e-10 (float64) or 1e-4 (float32).  A wrong term
of the objective or of the L-BFGS recursion moves the step by O(1), far outside that bar.
"""
from dataclasses import replace

import numpy as np
import pytest
import torch

from oracle import cadmm, numeric
from paper_2507_10290_amd.workloads import random_walk_batch
from tests._harness import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

DT = torch.float64


def _problem(w, inner, **kw):
    from paper_2507_10290_amd import TopProblem
    return TopProblem.from_workload(w, numeric=True, lbfgs_iters=inner, use_graph=False, **kw)


def _oracle_state(pr, mats, st_gpu, box):
    """The oracle's NumState equal to an exported GPU state (folded pairs unfolded by identity I1)."""
    S, s, N, M = pr.S, pr.s, pr.n, pr.n_samples
    row = lambda f: torch.tensor(st_gpu[f, :S], dtype=DT)
    zR = torch.stack([torch.stack([row(a * s + o) for o in range(s)], 1) for a in range(3)], 1)   # [S,3,s]
    z = cadmm.initial_knots(pr).index_put((pr.knot_r,), zR)
    u = torch.cat([torch.cat([torch.stack([row(3 * s + a * s + o) for o in range(s)], 1),
                              torch.stack([row(6 * s + a * s + o) for o in range(s)], 1)], 1) for a in range(3)], 1)
    s_ = v = None
    C = 9 * s
    if box:
        ys = []
        for j in range(M):
            for a in range(3):
                ys.append(row(9 * s + a * M + j))             # upper row of (j, a)
                ys.append(row(9 * s + 3 * M + a * M + j))     # lower row
        y = torch.stack(ys, 1)
        s_, v = torch.clamp(-y, min=0.0), torch.clamp(y, min=0.0)
        C += 6 * M
    wv = torch.stack([row(C + j) for j in range(M)], 1)
    iTk = (1.0 / pr.T)[:, None] ** torch.arange(N, dtype=DT)[None, :]
    c = torch.cat([torch.stack([row(C + M + a * N + k) for k in range(N)], 1) * iTk for a in range(3)], 1)
    base = cadmm.State(c=c, z=z, u=u, s=s_, v=v, phi=None, w=None)
    return numeric.NumState(base=base, w=wv)


def _jitter_step(pr, mats, ost, inner, rel, seed=7, norm=2):
    """The oracle step from ost and from ost with every state value scaled by 1 + U(-rel, rel)."""
    g = torch.Generator().manual_seed(seed)
    jit = lambda t: None if t is None else t * (1.0 + rel * (2.0 * torch.rand(t.shape, generator=g, dtype=DT) - 1.0))
    b = ost.base
    pst = numeric.NumState(base=replace(b, c=jit(b.c), z=jit(b.z), u=jit(b.u), s=jit(b.s), v=jit(b.v)), w=jit(ost.w))
    a_, _, _ = numeric.iterate(pr, mats, ost, inner, norm)
    p_, _, _ = numeric.iterate(pr, mats, pst, inner, norm)
    return a_, cadmm.coeffs_by_axis(pr, p_.base.c).numpy()


def _rel_per_seg(a, b):
    return max(np.linalg.norm(a[i] - b[i]) / np.linalg.norm(b[i]) for i in range(len(b)))


def _check_steps(w, inner, Ks, floor, rel, box, norm=2, **kw):
    pr = cadmm.problem_from_workload(w)
    mats = cadmm.segment_matrices(pr)
    prob = _problem(w, inner, vel_norm=norm, **kw)
    if "lane_form" in kw:
        assert prob.plan()["lane_form"] == kw["lane_form"]
    done = 0
    worst = 0.0
    for K in Ks:
        if K > done:
            prob.iterate(K - done)
            done = K
        st = prob.get_state()[:, :pr.S].cpu().numpy().astype(np.float64)
        ost = _oracle_state(pr, mats, st, box)
        nxt, cj = _jitter_step(pr, mats, ost, inner, rel, norm=norm)
        prob.iterate(1)
        done += 1
        c = prob.coeffs().cpu().numpy()
        co = cadmm.coeffs_by_axis(pr, nxt.base.c).numpy()
        e = _rel_per_seg(c, co)
        bar = max(floor, 10.0 * _rel_per_seg(cj, co))
        worst = max(worst, e)
        print(f"[numeric] step after K={K}: per-segment coeff rel {e:.2e} (bar {bar:.2e})", flush=True)
        assert e <= bar, (K, e, bar)
    prob.sync_status()
    prob.close()
    return worst


@pytest.mark.parametrize("lane_form", [1, 3])
@pytest.mark.parametrize("order,box,vmax,inner", [(3, True, 1.5, 10), (3, False, 1.2, 6), (4, True, 1.5, 8)])
def test_fp64_numeric_steps_match_oracle(order, box, vmax, inner, lane_form):
    w = random_walk_batch("num", [4, 6, 3], [21, 22, 23], order=order, box=box, vmax=vmax, rho=[1.0, 2.0, 0.5],
                          precision="fp64")
    _check_steps(w, inner, [0, 3, 8, 14], 1e-10, 1e-14, box, lane_form=lane_form)


@pytest.mark.parametrize("lane_form", [1, 3])
@pytest.mark.parametrize("order,box,vmax,inner", [(3, True, 1.2, 10), (4, False, 1.0, 8)])
def test_fp64_numeric_l4_bound_steps_match_oracle(order, box, vmax, inner, lane_form):
    # the l4 speed bound (no closed-form projection): h = ||v||_4 - vmax in the squared hinge
    w = random_walk_batch("numl4", [4, 6, 3], [31, 32, 33], order=order, box=box, vmax=vmax, rho=[1.0, 2.0, 0.5],
                          precision="fp64")
    _check_steps(w, inner, [0, 3, 8, 14], 1e-10, 1e-14, box, norm=4, lane_form=lane_form)


@pytest.mark.parametrize("lane_form", [1, 3])
def test_fp64_numeric_l4_first_sweeps_match_oracle_runs(lane_form):
    w = random_walk_batch("numl4", [4, 6, 3], [31, 32, 33], order=3, vmax=1.2, rho=[1.0, 2.0, 0.5], precision="fp64")
    pr = cadmm.problem_from_workload(w)
    mats = cadmm.segment_matrices(pr)
    for K in (1, 2):
        prob = _problem(w, 10, vel_norm=4, lane_form=lane_form)
        prob.iterate(K)
        c = prob.coeffs().cpu().numpy()
        prob.close()
        res = numeric.run(pr, K, inner=10, norm=4)
        co = cadmm.coeffs_by_axis(pr, res.c).numpy()
        print(f"[numeric] l4 run K={K}: coeff rel {_rel_per_seg(c, co):.2e}", flush=True)
        assert _rel_per_seg(c, co) <= 1e-8
    # the bound is active in these sweeps (else this would only repeat the closed-form tests)
    vel = (mats["Av"] @ res.c[:, None, :, None])[..., 0]
    assert (numeric.velocity_excess(vel, pr.vmax[pr.traj][:, None], 4)[0] > 0).any()


@pytest.mark.parametrize("lane_form", [1, 3])
def test_fp32_numeric_l4_steps_close_to_oracle(lane_form):
    w = random_walk_batch("numl432", [5, 7], [35, 36], order=3, vmax=1.2, rho=1.0, precision="fp32")
    _check_steps(w, 10, [0, 3], 1e-4, 1e-6, True, norm=4, lane_form=lane_form)


@pytest.mark.parametrize("lane_form", [1, 3])
def test_fp64_numeric_first_sweeps_match_oracle_runs(lane_form):
    w = random_walk_batch("num", [4, 6, 3], [21, 22, 23], order=3, vmax=1.5, rho=[1.0, 2.0, 0.5], precision="fp64")
    pr = cadmm.problem_from_workload(w)
    for K, inner in ((1, 10), (2, 10), (5, 0)):
        prob = _problem(w, inner, lane_form=lane_form)
        prob.iterate(K)
        c, J = prob.coeffs().cpu().numpy(), prob.cost().cpu().numpy()
        prob.close()
        res = numeric.run(pr, K, inner=inner)
        co = cadmm.coeffs_by_axis(pr, res.c).numpy()
        print(f"[numeric] run K={K} inner={inner}: coeff rel {_rel_per_seg(c, co):.2e}", flush=True)
        assert _rel_per_seg(c, co) <= 1e-8
        assert np.allclose(J, res.J.numpy(), rtol=1e-8)


@pytest.mark.parametrize("lane_form", [1, 3])
def test_fp64_numeric_steps_on_halo_tiles(lane_form):
    w = random_walk_batch("numhalo", [90], [24], order=3, vmax=1.5, rho=1.0, precision="fp64")
    _check_steps(w, 6, [0, 5, 11], 1e-10, 1e-14, True, tile_lanes=64, halo=4, lane_form=lane_form)


@pytest.mark.parametrize("lane_form", [1, 3])
def test_fp32_numeric_steps_close_to_oracle(lane_form):
    w = random_walk_batch("num32", [5, 7], [25, 26], order=3, vmax=1.5, rho=1.0, precision="fp32")
    _check_steps(w, 10, [0, 3], 1e-4, 1e-6, True, lane_form=lane_form)


@pytest.mark.parametrize("lane_form", [1, 3])
def test_state_round_trip_and_resume(lane_form):
    w = random_walk_batch("numrt", [5, 4], [28, 29], order=3, vmax=1.5, precision="fp64")
    a, b = _problem(w, 8, lane_form=lane_form), _problem(w, 8, lane_form=lane_form)
    assert a.get_state().shape[1] > a.S and (a.get_state()[:, a.S:] == 0).all()   # padding columns
    a.iterate(6)
    assert (a.get_state()[:, a.S:] == 0).all()
    b.set_state(a.get_state())
    a.iterate(3)
    b.iterate(3)
    assert torch.equal(a.coeffs(), b.coeffs())
    a.close()
    b.close()


def test_numeric_option_errors():
    from paper_2507_10290_amd import TopError, TopProblem
    w = random_walk_batch("numerr", [3], [27], order=3, vmax=None, precision="fp64")
    with pytest.raises(TopError, match="vmax"):
        TopProblem.from_workload(w, numeric=True)
    w = random_walk_batch("numerr", [3], [27], order=3, vmax=2.0, precision="fp64")
    with pytest.raises(TopError, match="no tape"):
        TopProblem.from_workload(w, numeric=True, checkpoint_every=5, max_taped_iters=10)
    with pytest.raises(TopError, match="no checks"):
        TopProblem.from_workload(w, numeric=True, check_every=5)
    with pytest.raises(TopError, match="l4"):
        TopProblem.from_workload(w, vel_norm=4)               # the closed form has no l4 projection
