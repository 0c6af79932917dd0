"""Chained launches: the halo epochs of one iterate call in one cooperative launch.

A chained launch must give the same bits as one launch per epoch (the ordinary form, chain=1):
the halo copies a tile reloads between epochs are the values its neighbours publish, which are
the values a fresh launch would load.  Coefficients, cost, residuals and the whole iterate state
are compared bit for bit, over calls whose sweep counts are and are not multiples of the halo,
and the results are held to the oracle in float64.
"""
import numpy as np
import pytest
import torch

from paper_2507_10290_amd.workloads import curve_workload, make_config, random_walk_batch
from tests._harness import gpu_available, per_traj_rel, rel, run_oracle

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _ragged(precision):
    lens = [1, 2, 63, 64, 65, 1, 128, 129, 300, 7]
    return random_walk_batch("ragged", lens, list(range(100, 100 + len(lens))), order=3,
                             rho=[0.5, 1.0, 2.0, 1.0, 0.5, 2.0, 1.0, 1.0, 2.0, 0.5], precision=precision)


def _run(w, calls, precision, **kw):
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, precision=precision, lane_form=3, **kw)
    try:
        plan = prob.plan()
        for k in calls:
            prob.iterate(k)
        out = [prob.coeffs(), prob.cost(), *prob.residuals(), prob.get_state()]
        prob.sync_status()
        torch.cuda.synchronize()
        return [x.cpu().numpy() for x in out], plan
    finally:
        prob.close()


CASES = {
    # name: (workload, calls, precision, plan options)
    "septic-fp32": (lambda: make_config(2, scale=1 / 32), (70, 33, 1), "fp32", {"halo": 16}),
    "septic-fp64": (lambda: make_config(2, scale=1 / 64), (45, 19), "fp64", {"halo": 8}),
    "quintic-fp64-halo": (lambda: make_config(1), (50, 7), "fp64", {"tile_lanes": 128, "halo": 8}),
    "ragged-fp64": (lambda: _ragged("fp64"), (60,), "fp64", {"tile_lanes": 64, "halo": 12}),
    "ragged-fp32": (lambda: _ragged("fp32"), (25, 26), "fp32", {"tile_lanes": 128, "halo": 12}),
    # the other corridor / bound instances and consensus orders
    "septic-box-only-fp32": (lambda: random_walk_batch("sbox", [700, 90], [5, 6], order=4, box=True, vmax=None,
                                                       precision="fp32"), (40,), "fp32", {"halo": 16}),
    "quintic-vel-only-fp64": (lambda: random_walk_batch("qvel", [400, 250], [7, 8], order=3, box=False, vmax=3.0,
                                                        precision="fp64"), (30,), "fp64",
                              {"tile_lanes": 128, "halo": 8}),
    "quintic-s4-fp64": (lambda: random_walk_batch("q4", [300], [9], order=3, n_cont=4, precision="fp64"), (27,),
                        "fp64", {"tile_lanes": 128, "halo": 8}),
    "septic-s5-fp32": (lambda: random_walk_batch("s5", [900], [10], order=4, n_cont=5, precision="fp32"), (50,),
                       "fp32", {"halo": 16}),
    "curve-end-states-fp32": (lambda: curve_workload(1500, order=3, precision="fp32"), (100,), "fp32", {"halo": 32}),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_chained_launches_give_the_same_bits(case):
    make, calls, prec, kw = CASES[case]
    w = make()
    print(f"[chain] {case} S={w.n_seg} calls={calls} {kw}", flush=True)
    chained, plan_c = _run(w, calls, prec, chain=0, **kw)
    plain, plan_p = _run(w, calls, prec, chain=1, **kw)
    print(f"[chain] plans {plan_c} / {plan_p}", flush=True)
    assert plan_c["chained"] == 1 and plan_p["chained"] == 0
    assert plan_c["halo"] > 0 and max(calls) > plan_c["halo"]
    for name, x, y in zip(("coeffs", "cost", "r_primal", "r_dual", "state"), chained, plain):
        assert np.isfinite(x).all(), name
        assert np.array_equal(x, y), name
    if prec == "fp64":
        co, Jo, _, _ = run_oracle(w, sum(calls))
        assert per_traj_rel(w, chained[0], co) <= 1e-10 and rel(chained[1], Jo) <= 1e-10


def test_tiles_whose_cores_are_too_short_do_not_chain():
    # 64-segment tiles with 24-segment halos keep 16-segment cores, fewer than the 25 a neighbour's
    # copies and their start knots reach into: the plan runs one launch per epoch
    w = _ragged("fp64")
    out, plan = _run(w, (60,), "fp64", chain=0, tile_lanes=64, halo=24)
    assert plan["chained"] == 0
    ref, _ = _run(w, (60,), "fp64", chain=1, tile_lanes=64, halo=24)
    for x, y in zip(out, ref):
        assert np.array_equal(x, y)
    co, Jo, _, _ = run_oracle(w, 60)
    assert per_traj_rel(w, out[0], co) <= 1e-10


def test_chained_calls_mixed_with_single_epoch_calls():
    # calls of at most `halo` sweeps take the ordinary single launch, longer ones chain; the state
    # passes between them through the same buffers
    w = make_config(2, scale=1 / 32)
    calls = (5, 40, 16, 3, 50)
    chained, plan = _run(w, calls, "fp32", chain=0, halo=16)
    plain, _ = _run(w, calls, "fp32", chain=1, halo=16)
    assert plan["chained"] == 1
    for x, y in zip(chained, plain):
        assert np.array_equal(x, y)


def test_a_wait_that_gives_up_is_reported(monkeypatch):
    # the neighbour waits of a chained launch are bounded; with the bound forced to zero polls from
    # the host every wait gives up at once, the launch still ends, and top_sync_status reports it
    from paper_2507_10290_amd import TopProblem
    from paper_2507_10290_amd.binding import TOP_E_HIP, TopError
    w = make_config(2, scale=1 / 32)
    monkeypatch.setenv("TOP_CHAIN_SPIN", "0")
    prob = TopProblem.from_workload(w, precision="fp32", lane_form=3, halo=16)
    try:
        assert prob.plan()["chained"] == 1
        prob.iterate(40)
        with pytest.raises(TopError) as ei:
            prob.sync_status()
        assert ei.value.status == TOP_E_HIP and "gave up waiting" in str(ei.value)
    finally:
        prob.close()
    monkeypatch.delenv("TOP_CHAIN_SPIN")
    ok, _ = _run(w, (40,), "fp32", chain=0, halo=16)
    ref, _ = _run(w, (40,), "fp32", chain=1, halo=16)
    for x, y in zip(ok, ref):
        assert np.array_equal(x, y)


def test_iterate_in_a_callers_graph_capture_runs_one_launch_per_epoch():
    # a caller capturing the handle's stream gets the ordinary launches (a cooperative launch is not
    # captured); two epochs return the state to its buffer, so the graph can be replayed in turn
    from paper_2507_10290_amd import TopProblem
    w = make_config(2, scale=1 / 32)
    s = torch.cuda.Stream()
    cap = TopProblem.from_workload(w, precision="fp32", lane_form=3, halo=16, use_graph=False, stream=s)
    ref = TopProblem.from_workload(w, precision="fp32", lane_form=3, halo=16, use_graph=False)
    try:
        assert cap.plan()["chained"] == 1
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            cap.iterate(32)
        for step in range(3):
            graph.replay()
            ref.iterate(32)
            torch.cuda.synchronize()
            assert torch.equal(cap.coeffs(), ref.coeffs()), step
            assert torch.equal(cap.cost(), ref.cost()), step
        cap.sync_status()
        ref.sync_status()
    finally:
        cap.close()
        ref.close()


def test_tuning_times_chained_candidates_on_a_copy():
    # top_tune runs a candidate that would chain as a chained launch, on a copy of the iterate: the
    # iterate is untouched, and the solve goes on to the same bits as an untuned handle (the results
    # do not depend on the tiling)
    from paper_2507_10290_amd import TopProblem
    w = random_walk_batch("tunechain", [3000], [11], order=4, precision="fp32")
    tuned = TopProblem.from_workload(w, precision="fp32")
    plain = TopProblem.from_workload(w, precision="fp32")
    try:
        assert tuned.plan()["lane_form"] == 3
        tuned.iterate(20)
        plain.iterate(20)
        before = tuned.get_state().clone()
        plan = tuned.tune(40)   # more sweeps than any candidate halo: the axis candidates chain
        print(f"[chain] tuned plan {plan}", flush=True)
        assert torch.equal(tuned.get_state(), before)
        tuned.iterate(40)
        plain.iterate(40)
        torch.cuda.synchronize()
        assert torch.equal(tuned.coeffs(), plain.coeffs())
        assert torch.equal(tuned.cost(), plain.cost())
        tuned.sync_status()
        plain.sync_status()
    finally:
        tuned.close()
        plain.close()
