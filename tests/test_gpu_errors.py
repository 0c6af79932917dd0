"""GPU: the deferred error path.  Finite inputs whose iterates overflow pass the input check, queue
their sweeps without error, and are reported by top_sync_status as TOP_E_NONFINITE."""
import numpy as np
import pytest

from paper_2507_10290_amd import binding
from paper_2507_10290_amd.binding import TopProblem
from paper_2507_10290_amd.workloads import make_config
from tests._harness import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


@pytest.mark.parametrize("precision,scale", [("fp64", 1e200), ("fp32", 1e38)])
def test_overflowing_iterates_are_reported_by_sync_status(precision, scale):
    # float64: the cost ~ |dP|^2 / T^5 exceeds the float64 range; float32: the step polynomial's
    # coefficients (10 dP, ...) exceed the float32 range.  Every input is finite.
    w = make_config(1, scale=64 / 1024)
    w.waypoints = w.waypoints * scale
    w.box_lo, w.box_hi = w.box_lo * scale, w.box_hi * scale
    print(f"[errors] {precision} waypoints x {scale:g}", flush=True)
    prob = TopProblem.from_workload(w, precision=precision)
    try:
        prob.iterate(5)                      # queued without error: the check is deferred
        with pytest.raises(binding.TopError) as ei:
            prob.sync_status()
        assert ei.value.status == binding.TOP_E_NONFINITE
        assert "non-finite" in str(ei.value)
    finally:
        prob.close()


def test_finite_run_reports_ok_and_invalid_input_is_refused():
    w = make_config(1, scale=64 / 1024)
    prob = TopProblem.from_workload(w, precision="fp32")
    try:
        prob.iterate(5)
        prob.sync_status()
    finally:
        prob.close()
    w.durations = w.durations.copy()
    w.durations[3] = np.inf                  # not finite: refused at create (TOP_E_INVALID)
    with pytest.raises(binding.TopError) as ei:
        TopProblem.from_workload(w, precision="fp32")
    assert ei.value.status == binding.TOP_E_INVALID and "durations" in str(ei.value)
