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

from paper_2507_10290_amd.workloads import make_config, random_walk_batch
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
