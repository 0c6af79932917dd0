"""Paper-literal consensus on every order (s = 2p - 1) and the segment-count study workload (a
parametric curve with pinned points, Sec. IV) on the GPU against the oracle."""
import numpy as np
import pytest

from oracle import cadmm
from paper_2507_10290_amd.metrics import e_simi
from paper_2507_10290_amd.workloads import curve, curve_workload, random_walk_batch
from tests._harness import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _gpu(w, K, **kw):
    from paper_2507_10290_amd import TopProblem
    prob = TopProblem.from_workload(w, **kw)
    prob.iterate(K)
    c, J = prob.coeffs().cpu().numpy(), prob.cost().cpu().numpy()
    prob.sync_status()
    prob.close()
    return c, J


@pytest.mark.parametrize("order,precision,tol", [(3, "fp64", 1e-10), (4, "fp64", 1e-10), (3, "fp32", 1e-4)])
def test_full_order_consensus_matches_oracle(order, precision, tol):
    w = random_walk_batch("s2p", [6, 9, 4], [5, 6, 7], order=order, rho=[1.0, 2.0, 0.5], precision=precision)
    w.n_cont = 2 * order - 1
    K = 60
    c, J = _gpu(w, K)
    pr = cadmm.problem_from_workload(w)
    assert pr.s == 2 * order - 1
    res = cadmm.run(pr, K)
    co = cadmm.coeffs_by_axis(pr, res.c).numpy()
    e = np.linalg.norm(c - co) / np.linalg.norm(co)
    eJ = np.max(np.abs(J - res.J.numpy()) / res.J.numpy())
    print(f"[f3] s=2p-1 p={order} {precision}: coeff {e:.2e} cost {eJ:.2e}", flush=True)
    assert e <= tol and eJ <= (tol if precision == "fp64" else 1e-3)


def test_curve_workload_and_e_simi_match_oracle():
    w = curve_workload(24, precision="fp64", iters=300)
    c, J = _gpu(w, w.iters)
    pr = cadmm.problem_from_workload(w)
    res = cadmm.run(pr, w.iters)
    co = cadmm.coeffs_by_axis(pr, res.c).numpy()
    assert np.linalg.norm(c - co) / np.linalg.norm(co) <= 1e-10
    span = 2 * np.pi
    ref = lambda t: curve(t * span / w.durations.sum())
    eg, eo = e_simi(c, w.durations, ref), e_simi(co, w.durations, ref)
    print(f"[f3] curve N=24: e_simi gpu {eg:.6f} oracle {eo:.6f}", flush=True)
    assert abs(eg - eo) < 1e-8


def test_full_order_consensus_rejects_a_tape():
    from paper_2507_10290_amd import TopError, TopProblem
    w = random_walk_batch("s2p", [3], [5], order=3, precision="fp64")
    w.n_cont = 5
    with pytest.raises(TopError, match="2p-1"):
        TopProblem.from_workload(w, checkpoint_every=5, max_taped_iters=10)
