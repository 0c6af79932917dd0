"""GPU sweep with general polytope corridors (a_k . x <= b_k per segment) against the oracle.

Same bars as the box path: float64 iterates to 1e-10 (coefficients, cost), float32 to 1e-4 on the
coefficients and 1e-3 on the cost.
"""
import copy

import numpy as np
import pytest
import torch

from oracle import adaptive, cadmm
from paper_2507_10290_amd.workloads import make_config, random_walk_batch
from tests._harness import gpu_available, worst_segment

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _tighten(w, h=0.05):
    P, offs = w.waypoints, w.seg_offsets
    for b in range(w.n_traj):
        for i in range(offs[b], offs[b + 1]):
            for k in range(w.faces.shape[1]):
                a = w.faces[i, k, :3]
                w.faces[i, k, 3] = max(a @ P[i + b], a @ P[i + b + 1]) + h
    return w


def _gpu(w, K, **kw):
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, **kw)
    prob.iterate(K)
    out = dict(c=prob.coeffs().cpu().numpy(), J=prob.cost().cpu().numpy(),
               r=[x.cpu().numpy() for x in prob.residuals()])
    if kw.get("check_every"):
        out["conv"] = [x.cpu().numpy() for x in prob.convergence()]
    prob.sync_status()
    prob.close()
    return out


def _oracle(w, K):
    pr = cadmm.problem_from_workload(w)
    res = cadmm.run(pr, K)
    return cadmm.coeffs_by_axis(pr, res.c).numpy(), res


def _check(w, g, co, res, tol_c, tol_J, label):
    offs = w.seg_offsets
    worst = 0.0
    for b in range(w.n_traj):
        s0, s1 = offs[b], offs[b + 1]
        worst = max(worst, np.linalg.norm(g["c"][s0:s1] - co[s0:s1]) / np.linalg.norm(co[s0:s1]))
    eJ = np.max(np.abs(g["J"] - res.J.numpy()) / np.abs(res.J.numpy()))
    print(f"[poly] {label}: coeff rel {worst:.2e} cost rel {eJ:.2e}", flush=True)
    assert worst <= tol_c and eJ <= tol_J


@pytest.mark.parametrize("order,tight", [(3, False), (3, True), (4, True)])
def test_fp64_polytope_matches_oracle(order, tight):
    w = random_walk_batch("polyfp64", [7, 12, 5], [31, 32, 33], order=order, rho=[1.0, 2.0, 0.5],
                          precision="fp64", faces=8)
    if tight:
        _tighten(w)
    K = 120
    g = _gpu(w, K)
    co, res = _oracle(w, K)
    _check(w, g, co, res, 1e-10, 1e-10, f"p={order} tight={tight}")
    assert np.allclose(g["r"][0], res.rp.numpy(), rtol=1e-8) and np.allclose(g["r"][1], res.rd.numpy(), rtol=1e-8)


def test_fp64_fewer_faces_and_no_velocity():
    w = _tighten(random_walk_batch("poly6", [6, 9], [41, 42], order=3, vmax=None, precision="fp64", faces=8))
    w.faces = w.faces[:, :6].copy()                   # six faces, padded inside the library
    g = _gpu(w, 80)
    co, res = _oracle(w, 80)
    _check(w, g, co, res, 1e-10, 1e-10, "6 faces, no velocity")


def test_fp64_box_as_faces_equals_box_path():
    w = make_config(1, scale=40 / 1024)
    w.precision = "fp64"
    wp = copy.deepcopy(w)
    F = np.zeros((w.n_seg, 6, 4))
    for a in range(3):
        F[:, 2 * a, a], F[:, 2 * a, 3] = 1.0, w.box_hi[:, a]
        F[:, 2 * a + 1, a], F[:, 2 * a + 1, 3] = -1.0, -w.box_lo[:, a]
    wp.faces, wp.box_lo, wp.box_hi = F, None, None
    a, b = _gpu(w, 100), _gpu(wp, 100)
    assert np.linalg.norm(a["c"] - b["c"]) / np.linalg.norm(a["c"]) < 1e-11
    assert np.allclose(a["J"], b["J"], rtol=1e-11)


@pytest.mark.parametrize("tile", [0, 256])
def test_fp32_polytope_batched_subset(tile):
    # default tiles (512 lanes: whole trajectories) and 256-lane tiles (the longer ones split)
    w = _tighten(make_config(5, n_traj=6), h=0.15)
    assert w.traj_lengths().max() > 256
    K = 100
    g = _gpu(w, K, tile_lanes=tile)
    co, res = _oracle(w, K)
    _check(w, g, co, res, 1e-4, 1e-3, "batched subset fp32")


def test_fp32_polytope_full_workload_sampled():
    # the benchmark's 8-face batched workload at full size, in the configuration bench.py times
    # (default 512-lane tiles, K = 200); whole trajectories checked against the oracle
    w = make_config(5)
    K = w.iters
    print(f"[poly] full S={w.n_seg} K={K}", flush=True)
    g = _gpu(w, K)
    assert np.isfinite(g["c"]).all() and np.isfinite(g["J"]).all()
    L = w.traj_lengths()
    picks = sorted({int(np.argmin(L)), int(np.argmax(L)), 0, 2047, 4095})
    sub = w.subset(picks)
    co, res = _oracle(sub, K)
    for k, t in enumerate(picks):
        s0, s1 = int(w.seg_offsets[t]), int(w.seg_offsets[t + 1])
        q0, q1 = int(sub.seg_offsets[k]), int(sub.seg_offsets[k + 1])
        e = np.linalg.norm(g["c"][s0:s1] - co[q0:q1]) / np.linalg.norm(co[q0:q1])
        eJ = abs(g["J"][t] - res.J[k].item()) / abs(res.J[k].item())
        es, i = worst_segment(g["c"][s0:s1], co[q0:q1])
        print(f"[poly]   traj {t} (N={s1 - s0}) coeff {e:.2e} cost {eJ:.2e} worst segment {i}: {es:.2e}",
              flush=True)
        assert e <= 1e-4 and eJ <= 1e-3 and es <= 1e-3


def test_fp64_polytope_halo_tiles():
    w = _tighten(random_walk_batch("polyhalo", [150], [51], order=3, precision="fp64", faces=8), h=0.1)
    K = 40
    g = _gpu(w, K, tile_lanes=64, halo=5)
    co, res = _oracle(w, K)
    _check(w, g, co, res, 1e-10, 1e-10, "halo tiles")


def test_fp64_polytope_adaptive_rho():
    w = _tighten(random_walk_batch("polyad", [4, 6], [61, 62], order=3, rho=[5.0, 0.2], precision="fp64",
                                   faces=8), h=0.1)
    K = 150
    o = adaptive.run_adaptive(cadmm.problem_from_workload(w), K, check_every=5, adapt=True, eps=0.1)
    g = _gpu(w, K, check_every=5, adapt_rho=True, tol=0.1)
    it, rho, done = g["conv"]
    print(f"[poly] adaptive iters {it.tolist()} / {o.iters.tolist()} rho {rho.tolist()}", flush=True)
    assert np.array_equal(it, o.iters) and np.array_equal(done.astype(bool), o.converged)
    assert np.allclose(rho, o.rho.numpy(), rtol=1e-14, atol=0)
    assert np.any(rho != w.rho)
    co = cadmm.coeffs_by_axis(cadmm.problem_from_workload(w), o.c).numpy()
    assert np.linalg.norm(g["c"] - co) / np.linalg.norm(co) < 1e-10


def test_polytope_errors():
    from paper_2507_10290_amd import TopError, TopProblem
    w = random_walk_batch("polyerr", [3], [71], order=3, precision="fp64", faces=8)
    with pytest.raises(TopError, match="tape"):
        TopProblem.from_workload(w, checkpoint_every=5, max_taped_iters=10)
    w9 = copy.deepcopy(w)
    w9.faces = np.concatenate([w.faces, w.faces[:, :1]], 1)
    with pytest.raises(TopError, match="n_faces"):
        TopProblem.from_workload(w9)
    wn = copy.deepcopy(w)
    wn.faces[1, 2, 3] = np.nan
    with pytest.raises(TopError, match="faces"):
        TopProblem.from_workload(wn)
    wn = copy.deepcopy(w)
    wn.faces[-1, -1, 0] = np.inf                 # the last element of the flat face array
    with pytest.raises(TopError, match="faces"):
        TopProblem.from_workload(wn)
