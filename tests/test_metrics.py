"""Pins of the host-side trajectory evaluation and the e_simi metric (no GPU)."""
import numpy as np
import numpy.polynomial.polynomial as nppoly

from paper_2507_10290_amd.metrics import e_simi, evaluate
from paper_2507_10290_amd.workloads import curve, curve_workload


def test_evaluate_matches_numpy_polyval():
    rng = np.random.default_rng(3)
    N, n = 5, 6
    coeffs = rng.standard_normal((N, 3, n))
    T = rng.uniform(0.5, 2.0, N)
    starts = np.concatenate([[0.0], np.cumsum(T)[:-1]])
    t = np.sort(rng.uniform(0, T.sum(), 200))
    got = evaluate(coeffs, T, t)
    for k, tk in enumerate(t):
        i = min(np.searchsorted(starts, tk, side="right") - 1, N - 1)
        want = [nppoly.polyval(tk - starts[i], coeffs[i, a]) for a in range(3)]
        assert np.allclose(got[k], want, rtol=1e-12, atol=1e-12)


def test_e_simi_of_a_shifted_copy():
    rng = np.random.default_rng(4)
    coeffs = rng.standard_normal((4, 3, 6))
    T = np.ones(4)
    delta = np.array([3e-3, -4e-3, 0.0])                   # |delta| = 5e-3
    ref = lambda t: evaluate(coeffs, T, t) + delta
    assert abs(e_simi(coeffs, T, ref, m=8192) - np.log10(8192 * 5e-3)) < 1e-9


def test_curve_samples_and_end_states():
    w = curve_workload(10, total_time=5.0)
    th = np.linspace(0, 2 * np.pi, 11)
    assert np.allclose(w.waypoints, curve(th))
    # end velocities are the curve's theta-derivative times d theta / dt
    assert np.allclose(w.bc[0, 0, 1], curve(th[:1], 1)[0] * (2 * np.pi / 5.0))
    assert np.allclose(w.bc[0, 1, 0], w.waypoints[-1])
