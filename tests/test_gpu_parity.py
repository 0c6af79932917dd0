"""GPU parity: the HIP library (through the C ABI) against the CPU oracle on the same seeded inputs.

Tolerances: float64 iterates 1e-10 relative (per-trajectory Frobenius norm of
the coefficients, and the cost); float32 iterates 1e-4 on coefficients and
1e-3 on the cost.  At full benchmark sizes the oracle checks samples: whole
trajectories of the batched workload, and light-cone windows of the long
trajectory (a segment's iterate after K sweeps depends only on segments
within K of it).
"""
import numpy as np
import pytest
import torch

from paper_2507_10290_amd.workloads import make_config, random_walk_batch
from tests._harness import gpu_available, per_traj_rel, rel, run_gpu, run_oracle, worst_segment

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]

TOL = {"fp64": (1e-10, 1e-10), "fp32": (1e-4, 1e-3)}


def _check(w, K, precision, **kw):
    print(f"[parity] {w.name} S={w.n_seg} B={w.n_traj} K={K} {precision} {kw}", flush=True)
    cg, Jg, rpg, rdg = run_gpu(w, K, precision, **kw)
    co, Jo, rpo, rdo = run_oracle(w, K)
    tc, tJ = TOL[precision]
    assert np.isfinite(cg).all()
    ec = per_traj_rel(w, cg, co)
    eJ = rel(Jg, Jo)
    print(f"[parity]   coeff rel {ec:.3e}  cost rel {eJ:.3e}", flush=True)
    assert ec <= tc, ec
    assert eJ <= tJ, eJ
    if precision == "fp64" and K > 0:
        assert np.allclose(rpg, rpo, rtol=1e-8, atol=1e-12)
        assert np.allclose(rdg, rdo, rtol=1e-8, atol=1e-12)
    return cg, Jg


def test_config0_fp64_plain():
    _check(make_config(0), 200, "fp64")


def test_config0_init_guess_is_exact_chord_step():
    w = make_config(0)
    cg, Jg, _, _ = run_gpu(w, 0, "fp64")
    co, Jo, _, _ = run_oracle(w, 0)
    assert per_traj_rel(w, cg, co) < 1e-13
    assert rel(Jg, Jo) < 1e-12                    # the Init guess's cost, reduced on request


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_config1_full(precision):
    _check(make_config(1), 500, precision)


def test_config1_fp64_halo_tiles():
    # 1024 segments in 64-lane tiles with 8-sweep halos: many tile seams, ragged last tile
    _check(make_config(1), 100, "fp64", tile_lanes=64, halo=8)


def test_config2_septic_fp32_reduced():
    _check(make_config(2, scale=1 / 32), 300, "fp32")


def test_config2_septic_fp64_reduced_halo():
    _check(make_config(2, scale=1 / 64), 120, "fp64", tile_lanes=128, halo=16)


def test_config3_batched_subset():
    w = make_config(3, n_traj=48)
    _check(w, 200, "fp32")


def test_config3_batched_subset_fp64():
    _check(make_config(3, n_traj=24), 200, "fp64")


def test_config4_subset_fp32():
    _check(make_config(4, n_traj=16), 100, "fp32")


def test_ragged_batch_edges_fp64():
    # 1-segment trajectories, lengths at and around the tile width, a long one split with halos
    lens = [1, 2, 63, 64, 65, 1, 128, 129, 300, 7]
    w = random_walk_batch("ragged", lens, list(range(100, 100 + len(lens))), order=3,
                          rho=[0.5, 1.0, 2.0, 1.0, 0.5, 2.0, 1.0, 1.0, 2.0, 0.5], precision="fp64")
    _check(w, 60, "fp64", tile_lanes=128, halo=12)


def test_free_interior_and_unconstrained_fp64():
    w = random_walk_batch("free", [5, 9], [7, 8], order=3, box=False, vmax=None, rho=[1.0, 2.0],
                          precision="fp64", fix_interior=False)
    _check(w, 150, "fp64")


def test_consensus_s_plus_one_fp64():
    w = make_config(0)
    w.n_cont = 4
    cg, Jg, _, _ = run_gpu(w, 200, "fp64")
    from oracle import cadmm
    pr = cadmm.problem_from_workload(w, s=4)
    r = cadmm.run(pr, 200)
    co = cadmm.coeffs_by_axis(pr, r.c).numpy()
    assert per_traj_rel(w, cg, co) < 1e-10
    assert rel(Jg, r.J.numpy()) < 1e-10


def test_box_only_and_vel_only_fp64():
    w = make_config(1, scale=40 / 1024)
    wb = make_config(1, scale=40 / 1024)
    wb.vmax = None
    _check(wb, 80, "fp64")
    wv = make_config(1, scale=40 / 1024)
    wv.box_lo = wv.box_hi = None
    _check(wv, 80, "fp64")
    del w


# ---------------------------------------------------------------------------
# Full benchmark sizes, sampled.
# ---------------------------------------------------------------------------

def test_config3_full_sampled_trajectories():
    w = make_config(3)
    K = w.iters
    print(f"[parity] config3 full S={w.n_seg}", flush=True)
    cg, Jg, rpg, rdg = run_gpu(w, K, "fp32")
    assert np.isfinite(cg).all() and np.isfinite(Jg).all()
    L = w.traj_lengths()
    picks = sorted({int(np.argmin(L)), int(np.argmax(L)), 0, 1, 2047, 4095})
    sub = w.subset(picks)
    co, Jo, _, _ = run_oracle(sub, K)
    for k, t in enumerate(picks):
        s0, s1 = int(w.seg_offsets[t]), int(w.seg_offsets[t + 1])
        q0, q1 = int(sub.seg_offsets[k]), int(sub.seg_offsets[k + 1])
        e = np.linalg.norm(cg[s0:s1] - co[q0:q1]) / np.linalg.norm(co[q0:q1])
        eJ = abs(Jg[t] - Jo[k]) / abs(Jo[k])
        es, i = worst_segment(cg[s0:s1], co[q0:q1])
        print(f"[parity]   traj {t} (N={s1 - s0}) coeff {e:.2e} cost {eJ:.2e} worst segment {i}: {es:.2e}",
              flush=True)
        assert e <= 1e-4 and eJ <= 1e-3 and es <= 1e-3


def test_config2_full_light_cone_samples():
    w = make_config(2)
    K = w.iters
    print(f"[parity] config2 full S={w.n_seg}", flush=True)
    cg, Jg, _, _ = run_gpu(w, K, "fp32")
    assert np.isfinite(cg).all() and np.isfinite(Jg).all()
    N = w.n_seg
    R = 8   # the window also covers the light cones of the R segments on either side of i
    for i in [0, 1, 777, N // 2, N - 2, N - 1]:
        lo, hi = max(0, i - K - 1 - R), min(N, i + K + 2 + R)
        win = w.window(0, lo, hi)
        co, _, _, _ = run_oracle(win, K)
        ci = co[i - lo]
        e = np.linalg.norm(cg[i] - ci) / np.linalg.norm(ci)
        js = list(range(max(0, i - R), min(N, i + R + 1)))
        es, jw = worst_segment(cg[js], co[[j - lo for j in js]])
        print(f"[parity]   segment {i}: coeff rel {e:.2e}; worst of segments {js[0]}..{js[-1]}: "
              f"{es:.2e} at {js[jw]}", flush=True)
        assert e <= 1e-4 and es <= 1e-3


def test_config4_full_sampled_trajectories():
    # the differentiation workload at full size (256 x 128, fp32, K = 100) in the configuration the
    # bench times (a tape every 10 sweeps): eight sampled trajectories against the oracle
    w = make_config(4)
    K = w.iters
    print(f"[parity] config4 full S={w.n_seg} K={K}", flush=True)
    cg, Jg, rpg, rdg = run_gpu(w, K, "fp32", checkpoint_every=10, max_taped_iters=K)
    assert np.isfinite(cg).all() and np.isfinite(Jg).all()
    picks = [0, 1, 37, 64, 128, 200, 254, 255]
    sub = w.subset(picks)
    co, Jo, rpo, rdo = run_oracle(sub, K)
    for k, t in enumerate(picks):
        s0, s1 = int(w.seg_offsets[t]), int(w.seg_offsets[t + 1])
        q0, q1 = int(sub.seg_offsets[k]), int(sub.seg_offsets[k + 1])
        e = np.linalg.norm(cg[s0:s1] - co[q0:q1]) / np.linalg.norm(co[q0:q1])
        eJ = abs(Jg[t] - Jo[k]) / abs(Jo[k])
        es, i = worst_segment(cg[s0:s1], co[q0:q1])
        print(f"[parity]   traj {t} coeff {e:.2e} cost {eJ:.2e} worst segment {i}: {es:.2e}", flush=True)
        assert e <= 1e-4 and eJ <= 1e-3 and es <= 1e-3
    _check_fp32_residuals(rpg[picks], rdg[picks], rpo, rdo)


def _check_fp32_residuals(rpg, rdg, rpo, rdo):
    # float32 residual norms against the oracle at 1e-3 relative
    erp = np.max(np.abs(rpg - rpo) / rpo)
    erd = np.max(np.abs(rdg - rdo) / rdo)
    print(f"[parity]   fp32 residuals: r_p rel {erp:.2e}  r_d rel {erd:.2e}", flush=True)
    assert erp <= 1e-3 and erd <= 1e-3


def test_fp32_residuals_match_oracle():
    for w, K in ((make_config(1), 500), (make_config(3, n_traj=48), 200)):
        print(f"[parity] fp32 residuals {w.name} S={w.n_seg} K={K}", flush=True)
        _, _, rpg, rdg = run_gpu(w, K, "fp32")
        _, _, rpo, rdo = run_oracle(w, K)
        _check_fp32_residuals(rpg, rdg, rpo, rdo)


def test_long_trajectory_reductions_fp64():
    # one trajectory of 9,000 segments (three reduction chunks of 4,096, the last ragged) between
    # two short ones: cost and both residual norms against the oracle
    w = random_walk_batch("longred", [5, 9000, 3], [41, 42, 43], order=3, rho=1.0, precision="fp64")
    _check(w, 3, "fp64")


def test_config2_full_cost_sums_its_coefficients():
    # the reported cost of the 65,536-segment trajectory equals the float64 cost of its own coefficients
    from oracle import cadmm
    w = make_config(2)
    cg, Jg, _, _ = run_gpu(w, 4, "fp32")
    pr = cadmm.problem_from_workload(w)
    Jc = cadmm.cost(pr, torch.from_numpy(cg).reshape(w.n_seg, -1)).numpy()
    print(f"[parity] config2 cost {Jg[0]:.12e} vs own coefficients {Jc[0]:.12e}", flush=True)
    assert rel(Jg, Jc) <= 1e-9


# ---------------------------------------------------------------------------
# Execution-form invariances (bitwise).
# ---------------------------------------------------------------------------

def test_tiling_graph_and_split_are_bitwise_invariant():
    w = make_config(3, n_traj=40)
    base, Jb, _, _ = run_gpu(w, 50, "fp32")
    for kw in ({"tile_lanes": 64, "halo": 4}, {"tile_lanes": 256}, {"use_graph": False}):
        c, J, _, _ = run_gpu(w, 50, "fp32", **kw)
        assert np.array_equal(c, base), kw
        assert np.array_equal(J, Jb), kw
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, precision="fp32")
    prob.iterate(20).iterate(1).iterate(29)
    c = prob.coeffs().cpu().numpy()
    prob.close()
    assert np.array_equal(c, base)


@pytest.mark.parametrize("case", ["config1-fp64", "config1-fp32", "septic-fp32", "septic-fp64", "ragged-fp64"])
def test_lane_forms_give_the_same_bits(case):
    # one lane per segment and axis (lane_form 3) runs each axis' arithmetic as the one-lane form
    # does: coefficients, cost and residuals agree bit for bit, whatever the tiles
    if case.startswith("config1"):
        w, K, t1, t3 = make_config(1), 120, {"tile_lanes": 256}, {}
    elif case.startswith("septic"):
        w, K, t1, t3 = make_config(2, scale=1 / 64), 70, {"tile_lanes": 128, "halo": 16}, {"halo": 16}
    else:
        lens = [1, 2, 63, 64, 65, 1, 128, 129, 300, 7]
        w = random_walk_batch("ragged", lens, list(range(100, 100 + len(lens))), order=3,
                              rho=[0.5, 1.0, 2.0, 1.0, 0.5, 2.0, 1.0, 1.0, 2.0, 0.5], precision="fp64")
        K, t1, t3 = 60, {"tile_lanes": 128, "halo": 12}, {"tile_lanes": 64, "halo": 12}
    prec = case.split("-")[1]
    print(f"[parity] lane forms {case} S={w.n_seg} K={K}", flush=True)
    one = run_gpu(w, K, prec, lane_form=1, **t1)
    three = run_gpu(w, K, prec, lane_form=3, **t3)
    for x, y in zip(one, three):
        assert np.isfinite(x).all() and np.array_equal(x, y)
    if prec == "fp64":
        co, Jo, _, _ = run_oracle(w, K)
        assert per_traj_rel(w, three[0], co) <= 1e-10 and rel(three[1], Jo) <= 1e-10


def test_lane_per_axis_graph_replays_match_eager_launches():
    # the lane-per-axis launches of a split trajectory, captured into a graph on their second
    # appearance and replayed, against a handle that never uses graphs
    from paper_2507_10290_amd import TopProblem
    w = make_config(2, scale=1 / 32)
    g = TopProblem.from_workload(w, precision="fp32", use_graph=True)
    e = TopProblem.from_workload(w, precision="fp32", use_graph=False)
    assert g.plan()["lane_form"] == 3 and g.plan()["halo"] > 0
    for step in range(5):
        g.iterate(40)
        e.iterate(40)
        torch.cuda.synchronize()
        assert torch.equal(g.coeffs(), e.coeffs()), step
        assert torch.equal(g.cost(), e.cost()), step
    g.close()
    e.close()


def test_default_lane_form():
    # three lanes per segment for trajectories longer than a one-lane tile, and for float32 problems
    # whose one-lane waves would fill fewer than half the SIMDs; one lane otherwise
    from paper_2507_10290_amd import TopProblem
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    cases = ((make_config(2, scale=1 / 16), "fp32"), (make_config(1), "fp64"), (make_config(3, n_traj=8), "fp32"),
             (make_config(3, n_traj=600), "fp32"))
    for w, prec in cases:
        prob = TopProblem.from_workload(w, precision=prec)
        plan = prob.plan()
        prob.close()
        longest = int(w.traj_lengths().max())
        print(f"[parity] {w.name} {prec} longest {longest} S={w.n_seg}: {plan}", flush=True)
        long_traj = longest > (512 if (prec == "fp32" and w.order == 3) else 256)
        few_waves = prec == "fp32" and (w.n_seg + 63) // 64 < simds // 2
        assert plan["lane_form"] == (3 if long_traj or few_waves else 1)
    # an explicit tile width keeps the one-lane form for a small problem
    w = make_config(3, n_traj=8)
    prob = TopProblem.from_workload(w, precision="fp32", tile_lanes=512)
    assert prob.plan()["lane_form"] == 1 and prob.plan()["tile_lanes"] == 512
    prob.close()


def test_graph_replays_match_eager_launches():
    # equal iterate(k) calls are captured on their second appearance and replayed afterwards; every
    # step is compared with a handle that never uses graphs, with host synchronisation between them
    from paper_2507_10290_amd import TopProblem
    w = make_config(3, n_traj=24)
    g = TopProblem.from_workload(w, precision="fp32", use_graph=True)
    e = TopProblem.from_workload(w, precision="fp32", use_graph=False)
    for step in range(7):
        g.iterate(10)
        e.iterate(10)
        torch.cuda.synchronize()
        assert torch.equal(g.coeffs(), e.coeffs()), step
        assert torch.equal(g.cost(), e.cost()), step
        rg, re_ = g.residuals(), e.residuals()
        assert torch.equal(rg[0], re_[0]) and torch.equal(rg[1], re_[1]), step
    g.close()
    e.close()


def test_repeat_runs_bitwise_equal():
    w = make_config(1, scale=0.25)
    a = run_gpu(w, 100, "fp32")[0]
    b = run_gpu(w, 100, "fp32")[0]
    assert np.array_equal(a, b)


@pytest.mark.parametrize("library_pool", [True, False])
def test_buffers_reused_across_streams_after_destroy(library_pool):
    # top_destroy does not wait: a handle created right after on another stream reuses the released
    # memory only after the released handle's queued sweeps have finished (the library's pool orders
    # that with an event; a torch workspace through the caching allocator's per-stream blocks)
    from paper_2507_10290_amd import TopProblem
    w = make_config(3, n_traj=128)
    ref = run_gpu(w, 40, "fp32")[0]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    for rep in range(3):
        with torch.cuda.stream(s1):
            a = TopProblem.from_workload(w, precision="fp32", stream=s1, use_graph=False, library_pool=library_pool)
            a.iterate(400)
            a.close()
        with torch.cuda.stream(s2):
            b = TopProblem.from_workload(w, precision="fp32", stream=s2, use_graph=False, library_pool=library_pool)
            b.iterate(40)
            c = b.coeffs()
            b.close()
        s2.synchronize()
        assert np.array_equal(c.cpu().numpy(), ref), rep
    s1.synchronize()


def test_many_live_handles_use_the_pageable_check_fallback():
    # more live handles than pinned words for the input check (1024): the later ones read the
    # check back through pageable memory; results and error reporting stay the same
    from paper_2507_10290_amd import TopError, TopProblem
    w = make_config(1, scale=4 / 1024)
    ref = run_gpu(w, 20, "fp64")[0]
    hs = [TopProblem.from_workload(w, precision="fp64", use_graph=False) for _ in range(1030)]
    try:
        bad = w.waypoints.copy()
        bad[1, 0] = np.nan
        with pytest.raises(TopError, match="waypoints"):
            TopProblem(w.seg_offsets, bad, w.durations, w.rho)
        hs[-1].iterate(20)
        c = hs[-1].coeffs().cpu().numpy()
    finally:
        for h in hs:
            h.close()
    assert np.array_equal(c, ref)


def test_autotune_keeps_results():
    w = make_config(3, n_traj=64)
    from paper_2507_10290_amd import TopProblem
    ref = run_gpu(w, 30, "fp32")[0]
    prob = TopProblem.from_workload(w, precision="fp32")
    plan = prob.tune(5)
    if plan["lane_form"] == 3:
        assert plan["tile_lanes"] in (128, 192, 256, 320)
    else:
        assert plan["tile_lanes"] in (64, 128, 256, 512)
    prob.iterate(30)
    c = prob.coeffs().cpu().numpy()
    prob.close()
    assert np.array_equal(c, ref)


# ---------------------------------------------------------------------------
# Device-side argument errors.
# ---------------------------------------------------------------------------

def test_invalid_device_inputs_are_rejected():
    from paper_2507_10290_amd import TopError, TopProblem
    w = make_config(1, scale=8 / 1024)
    bad = w.waypoints.copy()
    bad[3, 1] = np.nan
    with pytest.raises(TopError, match="waypoints"):
        TopProblem(w.seg_offsets, bad, w.durations, w.rho, box_lo=w.box_lo, box_hi=w.box_hi, vmax=w.vmax)
    T = w.durations.copy()
    T[2] = 0.0
    with pytest.raises(TopError, match="durations"):
        TopProblem(w.seg_offsets, w.waypoints, T, w.rho)
    with pytest.raises(TopError, match="rho"):
        TopProblem(w.seg_offsets, w.waypoints, w.durations, -w.rho)
    lo = w.box_lo.copy()
    lo[0, 0] = w.box_hi[0, 0] + 1
    with pytest.raises(TopError, match="box"):
        TopProblem(w.seg_offsets, w.waypoints, w.durations, w.rho, box_lo=lo, box_hi=w.box_hi)
    # last elements of each flat array (the check runs one element per lane)
    bad = w.waypoints.copy()
    bad[-1, 2] = np.inf
    with pytest.raises(TopError, match="waypoints"):
        TopProblem(w.seg_offsets, bad, w.durations, w.rho)
    hi = w.box_hi.copy()
    hi[-1, 2] = np.nan
    with pytest.raises(TopError, match="box"):
        TopProblem(w.seg_offsets, w.waypoints, w.durations, w.rho, box_lo=w.box_lo, box_hi=hi)
    T = w.durations.copy()
    T[-1] = -1.0
    with pytest.raises(TopError, match="durations"):
        TopProblem(w.seg_offsets, w.waypoints, T, w.rho)
    with pytest.raises(TopError, match="vmax"):
        TopProblem(w.seg_offsets, w.waypoints, w.durations, w.rho, vmax=np.zeros_like(w.rho))
    bc = np.zeros((w.n_traj, 2, 3, 3))
    bc[-1, 1, 2, 2] = np.nan
    with pytest.raises(TopError, match="bc"):
        TopProblem(w.seg_offsets, w.waypoints, w.durations, w.rho, bc=bc)
    prob = TopProblem(w.seg_offsets, w.waypoints, w.durations, w.rho, bc=np.zeros((w.n_traj, 2, 3, 3)))
    with pytest.raises(TopError, match="TOP_E_STATE"):
        prob.residuals()
    prob.close()


def test_tail_launch_gives_the_same_bits():
    # The batched workload packs into 2,056 tiles of 512 segments; a device that holds 256 at once
    # would run the last 8 in a round of their own, so their trajectories go to a tail launch with
    # one lane per segment and axis.  The results are the bits of the lane-per-axis plan (no tail).
    from paper_2507_10290_amd import TopProblem
    w = make_config(3)
    tail = TopProblem.from_workload(w, precision="fp32")
    ref = TopProblem.from_workload(w, precision="fp32", lane_form=3)
    try:
        plan = tail.plan()
        print(f"[tail] plan {plan}", flush=True)
        assert plan["lane_form"] == 1 and plan["tail_tiles"] > 0
        assert plan["tail_tile_lanes"] % 64 == 0 and 64 <= plan["tail_tile_lanes"] <= 320
        assert ref.plan()["tail_tiles"] == 0
        for k in (20, 20, 20, 20, 7):   # repeated calls are captured into a graph and replayed
            tail.iterate(k)
            ref.iterate(k)
            torch.cuda.synchronize()
            assert torch.equal(tail.coeffs(), ref.coeffs()), k
            assert torch.equal(tail.cost(), ref.cost()), k
            for x, y in zip(tail.residuals(), ref.residuals()):
                assert torch.equal(x, y), k
        assert torch.equal(tail.get_state(), ref.get_state())
        tail.sync_status()
        ref.sync_status()
    finally:
        tail.close()
        ref.close()


def test_no_tail_with_checks():
    # with residual checks every launch stops at the next check, so no plan gets a tail launch
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(make_config(3), precision="fp32", check_every=10, adapt_rho=True)
    try:
        assert prob.plan()["tail_tiles"] == 0
    finally:
        prob.close()


@pytest.mark.parametrize("case", ["polytope"])
def test_one_lane_tail_gives_the_same_bits(case):
    # Where one lane per axis is not available (polytope corridors) the tail runs the plan's own
    # kernel on tiles of half the width; 64-segment tiles (no tail: half of them is too narrow) give
    # the reference bits.
    from paper_2507_10290_amd import TopProblem
    kw = {}
    w = make_config(5)
    tail = TopProblem.from_workload(w, precision="fp32", **kw)
    ref = TopProblem.from_workload(w, precision="fp32", tile_lanes=64, **kw)
    try:
        plan = tail.plan()
        print(f"[tail] {case} plan {plan}", flush=True)
        assert plan["lane_form"] == 1 and plan["tail_tiles"] > 0 and plan["tail_tile_lanes"] <= plan["tile_lanes"] // 2
        assert ref.plan()["tail_tiles"] == 0
        for k in (20, 10):
            tail.iterate(k)
            ref.iterate(k)
            torch.cuda.synchronize()
            assert torch.equal(tail.coeffs(), ref.coeffs()), k
            assert torch.equal(tail.cost(), ref.cost()), k
        tail.sync_status()
        ref.sync_status()
    finally:
        tail.close()
        ref.close()
