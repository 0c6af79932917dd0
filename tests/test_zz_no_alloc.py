"""GPU: top_solve_static (no device allocation; state in the library's static scratch) against the
handle path (top_create on the pool, top_iterate, outputs) on the same inputs, two calls in a row,
the second with a smaller problem."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2507_10290_amd import binding
from paper_2507_10290_amd.workloads import make_config, random_walk_batch
from tests._harness import gpu_available

pytestmark = [pytest.mark.gpu, pytest.mark.skipif(not gpu_available(), reason="needs a GPU")]


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def _outputs(w):
    B, S, n = w.n_traj, w.n_seg, 2 * w.order
    return (torch.full((S, 3, n), np.nan, dtype=torch.float64, device="cuda"),
            *(torch.full((B,), np.nan, dtype=torch.float64, device="cuda") for _ in range(3)))


def _opts(w, precision):
    o = binding.default_options()
    o.order = w.order
    o.precision = binding.TOP_FP64 if precision == "fp64" else binding.TOP_FP32
    return o


def _handle_path(w, K, precision):
    d = {k: _dev(getattr(w, k)) for k in ("waypoints", "durations", "rho", "box_lo", "box_hi", "vmax", "bc")}
    o = _opts(w, precision)
    h = binding.top_create(w.seg_offsets, d["waypoints"], d["durations"], d["rho"], bc=d["bc"], box_lo=d["box_lo"],
                           box_hi=d["box_hi"], vmax=d["vmax"], options=o,
                           stream=torch.cuda.current_stream().cuda_stream)
    try:
        c, J, rp, rd = _outputs(w)
        binding.top_iterate(h, K)
        binding.top_coeffs(h, c)
        binding.top_cost(h, J)
        binding.top_residuals(h, rp, rd)
        binding.top_sync_status(h)
        return [t.cpu().numpy() for t in (c, J, rp, rd)]
    finally:
        binding.top_destroy(h)


def _static_path(w, K, precision):
    d = {k: _dev(getattr(w, k)) for k in ("waypoints", "durations", "rho", "box_lo", "box_hi", "vmax", "bc")}
    o = _opts(w, precision)
    c, J, rp, rd = _outputs(w)
    offs = np.ascontiguousarray(w.seg_offsets, dtype=np.int64)
    p = lambda t: None if t is None else t.data_ptr()
    st = binding.lib().top_solve_static(
        w.n_traj, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), p(d["waypoints"]), p(d["durations"]),
        p(d["bc"]), p(d["box_lo"]), p(d["box_hi"]), p(d["vmax"]), p(d["rho"]), ctypes.byref(o), K, p(c), p(J),
        p(rp), p(rd), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    binding._check(st)
    return [t.cpu().numpy() for t in (c, J, rp, rd)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_solve_matches_handle_path_twice(precision):
    big = make_config(1, scale=600 / 1024)                    # 600 segments, box + velocity
    small = random_walk_batch("small", [5, 70, 1, 33], [11, 12, 13, 14], order=3,
                              rho=[0.5, 1.0, 2.0, 1.0], precision=precision)
    for w, K in ((big, 80), (small, 40)):                     # the second call is smaller
        print(f"[no-alloc] {precision} S={w.n_seg} B={w.n_traj} K={K}", flush=True)
        a = _static_path(w, K, precision)
        b = _handle_path(w, K, precision)
        for x, y in zip(a, b):
            assert np.isfinite(x).all()
            assert np.array_equal(x, y), float(np.max(np.abs(x - y)))


def test_static_solve_limits():
    o = binding.default_options()
    # larger than the scratch: refused before any device work
    w = make_config(1, scale=64 / 1024)
    L = binding.lib()
    offs = np.array([0, 4_000_000], dtype=np.int64)
    st = L.top_solve_static(1, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0x1000, 0x1000, None, None,
                            None, None, 0x1000, ctypes.byref(o), 10, None, None, None, None, None)
    assert st == binding.TOP_E_WORKSPACE and b"static scratch" in L.top_last_error()
    o.checkpoint_every, o.max_taped_iters = 10, 10
    st = L.top_solve_static(1, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 0x1000, 0x1000, None, None,
                            None, None, 0x1000, ctypes.byref(o), 10, None, None, None, None, None)
    assert st == binding.TOP_E_UNSUPPORTED
    del w
