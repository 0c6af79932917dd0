"""GPU residual checks, stopping test and adaptive penalty against the oracle (Sec. III-D.3).

The oracle runs every trajectory on its own with the same check schedule; the
GPU must stop each trajectory at the same sweep, reach the same rho (the
decisions are float64 on both sides) and return the same coefficients, to
1e-10 (float64 iterates) or 1e-4 / 1e-3 on the cost (float32 iterates).
"""
import numpy as np
import pytest
import torch

from oracle import adaptive, cadmm
from paper_2507_10290_amd.workloads import make_config, random_walk_batch
from tests._harness import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _batch(lens, seeds, rho, precision="fp64", order=3):
    return random_walk_batch("adapt", list(lens), list(seeds), order=order, rho=rho, precision=precision)


def _gpu(w, K, splits=None, **kw):
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, **kw)
    for k in (splits or [K]):
        prob.iterate(k)
    c = prob.coeffs().cpu().numpy()
    J = prob.cost().cpu().numpy()
    rp, rd = (x.cpu().numpy() for x in prob.residuals())
    it, rho, done = (x.cpu().numpy() for x in prob.convergence())
    prob.sync_status()
    prob.close()
    return dict(c=c, J=J, rp=rp, rd=rd, iters=it, rho=rho, done=done)


def _compare(w, g, o, tol_c, tol_J):
    pr = cadmm.problem_from_workload(w)
    co = cadmm.coeffs_by_axis(pr, o.c).numpy()
    offs = w.seg_offsets
    print(f"[adapt] iters gpu {g['iters'].tolist()} oracle {o.iters.tolist()}; rho gpu {g['rho'].tolist()}", flush=True)
    assert np.array_equal(g["iters"], o.iters)
    assert np.array_equal(g["done"], o.converged)
    assert np.allclose(g["rho"], o.rho.numpy(), rtol=1e-14, atol=0)
    for b in range(len(offs) - 1):
        s0, s1 = offs[b], offs[b + 1]
        e = np.linalg.norm(g["c"][s0:s1] - co[s0:s1]) / np.linalg.norm(co[s0:s1])
        assert e <= tol_c, (b, e)
    assert np.all(np.abs(g["J"] - o.J.numpy()) <= tol_J * np.abs(o.J.numpy()))


@pytest.mark.parametrize("ce,K", [(5, 300), (1, 120)])
def test_fp64_adaptive_matches_oracle(ce, K):
    w = _batch((3, 5, 4, 6), (71, 72, 73, 74), [1.0, 2.0, 0.5, 1.0])
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), K, check_every=ce, adapt=True, eps=0.15)
    g = _gpu(w, K, check_every=ce, adapt_rho=True, tol=0.15)
    _compare(w, g, o, 1e-10, 1e-10)
    # residuals are those of each trajectory's last sweep
    assert np.allclose(g["rp"], o.rp.numpy(), rtol=1e-8) and np.allclose(g["rd"], o.rd.numpy(), rtol=1e-8)


def test_fp64_stopping_without_rho_update():
    w = _batch((5, 4, 3), (72, 73, 71), [1.0, 2.0, 1.0])
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), 400, check_every=25, adapt=False, eps=0.15)
    assert o.converged.any() and not o.converged.all()
    g = _gpu(w, 400, check_every=25, adapt_rho=False, tol=0.15)
    _compare(w, g, o, 1e-10, 1e-10)


def test_fp32_adaptive_matches_oracle():
    w = _batch((3, 5, 4, 6), (71, 72, 73, 74), [1.0, 2.0, 0.5, 1.0], precision="fp32")
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), 300, check_every=10, adapt=True, eps=0.15)
    g = _gpu(w, 300, check_every=10, adapt_rho=True, tol=0.15)
    _compare(w, g, o, 1e-4, 1e-3)


def test_fp64_adaptive_halo_tiles():
    w = make_config(1, scale=200 / 1024)
    w.precision = "fp64"
    w.rho[:] = 20.0                          # far from balanced: the rule lowers rho
    K = 60
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), K, check_every=7, adapt=True, eps=0.05)
    g = _gpu(w, K, check_every=7, adapt_rho=True, tol=0.05, tile_lanes=64, halo=5)
    assert o.rho.item() != w.rho[0]          # the rule changed rho on the way
    _compare(w, g, o, 1e-10, 1e-10)


def test_adaptive_batched_subset_fp32():
    w = make_config(3, n_traj=12)
    K = 100
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), K, check_every=10, adapt=True, eps=0.05)
    g = _gpu(w, K, check_every=10, adapt_rho=True, tol=0.05)
    _compare(w, g, o, 1e-4, 1e-3)


def test_checks_are_invariant_to_splits_graphs_and_tiles():
    w = _batch((3, 5, 4, 6, 40), (71, 72, 73, 74, 75), [1.0, 2.0, 0.5, 1.0, 1.0], precision="fp32")
    kw = dict(check_every=7, adapt_rho=True, tol=0.15)
    a = _gpu(w, 250, **kw)
    b = _gpu(w, 250, splits=[13, 100, 1, 136], use_graph=False, **kw)
    c = _gpu(w, 250, splits=[50] * 5, tile_lanes=64, **kw)
    for x in (b, c):
        for key in ("c", "J", "rp", "rd", "iters", "rho", "done"):
            assert np.array_equal(a[key], x[key]), key


def test_stopped_trajectory_is_left_unchanged():
    from paper_2507_10290_amd import TopProblem
    w = _batch((5, 4), (72, 73), [1.0, 2.0], precision="fp32")
    prob = TopProblem.from_workload(w, check_every=5, adapt_rho=False, tol=0.15)
    prob.iterate(300)
    it, _, done = prob.convergence()
    assert bool(done.all()), it
    c1, J1 = prob.coeffs().clone(), prob.cost().clone()
    prob.iterate(57)
    it2, _, _ = prob.convergence()
    assert torch.equal(prob.coeffs(), c1) and torch.equal(prob.cost(), J1) and torch.equal(it, it2)
    prob.close()


def test_check_option_errors():
    from paper_2507_10290_amd import TopError, TopProblem
    w = _batch((3,), (71,), [1.0])
    with pytest.raises(TopError, match="tape"):
        TopProblem.from_workload(w, check_every=5, checkpoint_every=5, max_taped_iters=10)
    with pytest.raises(TopError, match="mu, tau_incr"):
        TopProblem.from_workload(w, check_every=5, adapt_rho=True, mu=1.0)
    with pytest.raises(TopError, match="check_every"):
        TopProblem.from_workload(w, check_every=-1)
    # without checks: all sweeps, the input rho, nothing stopped
    prob = TopProblem.from_workload(w)
    prob.iterate(9)
    it, rho, done = prob.convergence()
    assert it.tolist() == [9] and rho.tolist() == [1.0] and not bool(done.any())
    prob.close()
