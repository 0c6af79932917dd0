"""The C-ABI library loads and exports every entry point include/top.h declares (no GPU needed).

Host-side argument checks run before any HIP call, so their error codes are
tested here too.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2507_10290_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "top.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(top_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    names = declared_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n
    assert sorted(binding.EXPORTED) == names


def test_default_options_and_error_text():
    o = binding.default_options()
    assert (o.order, o.n_cont, o.fix_interior, o.n_samples, o.precision, o.use_graph) == (3, 0, 1, 8, 0, 1)
    assert (o.local_solve, o.lbfgs_iters, o.vel_norm, o.lane_form, o.chain) == (0, 10, 2, 0, 0)
    assert isinstance(binding.lib().top_last_error(), bytes)


def _create(n_traj, offs, opts=None, with_ptrs=True, ws=None, ws_bytes=0, box=False, vmax=False):
    L = binding.lib()
    offs = np.asarray(offs, dtype=np.int64)
    h = ctypes.c_void_p()
    fake = 0x1000 if with_ptrs else None   # never dereferenced: host checks fail first
    st = L.top_create(n_traj, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), fake, fake, None,
                      fake if box else None, fake if box else None, fake if vmax else None, fake,
                      None if opts is None else ctypes.byref(opts), ws, ws_bytes, None, ctypes.byref(h))
    return st, h.value, L.top_last_error().decode()


def test_host_argument_errors():
    st, h, msg = _create(0, [0])
    assert st == binding.TOP_E_INVALID and h is None and "n_traj" in msg
    st, h, msg = _create(2, [0, 3, 3])
    assert st == binding.TOP_E_INVALID and "no segment" in msg
    st, h, msg = _create(1, [1, 3])
    assert st == binding.TOP_E_INVALID
    st, h, msg = _create(1, [0, 3], with_ptrs=False)
    assert st == binding.TOP_E_INVALID and "required" in msg
    o = binding.default_options()
    o.order = 5
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_UNSUPPORTED and "order" in msg
    o = binding.default_options()
    o.n_cont = 6                      # p = 3 takes s in {3, 4, 5}
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_UNSUPPORTED and "n_cont" in msg
    o = binding.default_options()
    o.local_solve = 2
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "local_solve" in msg
    o = binding.default_options()
    o.vel_norm = 4                     # the l4 speed bound needs NumericSolve
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_UNSUPPORTED and "l4" in msg
    o.vel_norm = 3
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "vel_norm" in msg
    o = binding.default_options()
    o.lane_form = 3                    # one lane per axis: not with a tape
    o.checkpoint_every, o.max_taped_iters = 5, 10
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_UNSUPPORTED and "lane per axis" in msg
    o = binding.default_options()
    o.lane_form = 2
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "lane_form" in msg
    o = binding.default_options()
    o.chain = 2
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "chain" in msg
    o = binding.default_options()
    o.check_every = -1
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "check_every" in msg
    o = binding.default_options()
    o.n_samples = 6
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_UNSUPPORTED
    o = binding.default_options()
    o.tile_lanes = 100
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID and "tile_lanes" in msg
    o = binding.default_options()
    o.checkpoint_every = 5
    o.max_taped_iters = 0
    st, h, msg = _create(1, [0, 3], o)
    assert st == binding.TOP_E_INVALID
    o = binding.default_options()
    o.check_every = 10                 # residual checks: trajectory-major grids bound the length
    st, h, msg = _create(2, [0, 3, 3 + 65535 * 128 + 1], o)
    assert st == binding.TOP_E_UNSUPPORTED and "at most" in msg


def test_null_handle_calls():
    L = binding.lib()
    assert L.top_iterate(None, 3) == binding.TOP_E_INVALID
    assert L.top_residuals(None, None, None) == binding.TOP_E_INVALID
    assert L.top_cost(None, None) == binding.TOP_E_INVALID
    assert L.top_coeffs(None, None) == binding.TOP_E_INVALID
    assert L.top_sync_status(None) == binding.TOP_E_INVALID
    assert L.top_tune(None, 3) == binding.TOP_E_INVALID
    L.top_destroy(None)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(binding, "_lib", None)
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "libtop.so"))
    with pytest.raises(ImportError, match="missing"):
        binding.lib()


# ---------------------------------------------------------------------------
# Caller-owned workspace: the size query and the too-small error are host-only.
# ---------------------------------------------------------------------------

def _ws(B, S, **kw):
    o = binding.default_options()
    for k, v in kw.items():
        setattr(o, k, v)
    return binding.lib().top_workspace_bytes(B, S, ctypes.byref(o))


def test_workspace_bytes_query():
    S = 10_000
    n32, n64 = _ws(4, S), _ws(4, S, precision=binding.TOP_FP64)
    assert n32 > 0 and n64 > n32
    # at least the two iterate buffers: 99 float fields per segment (quintic, box + velocity)
    ld = (S + 63) // 64 * 64
    assert n32 >= 2 * 99 * ld * 4
    assert _ws(4, 2 * S) > n32                                   # grows with the segment count
    assert _ws(4, S, order=4) > n32                              # septic: more fields, larger factors
    taped = _ws(4, S, checkpoint_every=10, max_taped_iters=100)
    assert taped - n32 >= 11 * 99 * ld * 4                       # the tape holds 100 / 10 + 1 states
    assert _ws(4, S, check_every=10) > n32                       # per-trajectory check state
    o = binding.default_options()
    npoly = binding.lib().top_workspace_bytes_polytope(4, S, 8, ctypes.byref(o))
    assert npoly > n32                                           # per-axis factors, rotation, faces
    assert binding.top_workspace_bytes(4, S) == n32              # the Python wrapper


def test_workspace_bytes_query_errors():
    L = binding.lib()
    assert L.top_workspace_bytes(0, 10, None) == 0 and "n_traj" in L.top_last_error().decode()
    assert L.top_workspace_bytes(4, 3, None) == 0                # fewer segments than trajectories
    o = binding.default_options()
    o.order = 5
    assert L.top_workspace_bytes(1, 10, ctypes.byref(o)) == 0 and "order" in L.top_last_error().decode()
    assert L.top_workspace_bytes_polytope(1, 10, 9, None) == 0   # at most 8 faces
    with pytest.raises(binding.TopError):
        binding.top_workspace_bytes(0, 10)


def test_workspace_too_small_is_rejected_before_device_work():
    offs = [0, 300, 1000]
    st, h, msg = _create(2, offs, ws=0x100000, ws_bytes=4096, box=True, vmax=True)
    assert st == binding.TOP_E_WORKSPACE and h is None, msg
    need = int(re.search(r"needs (\d+)", msg).group(1))
    assert 0 < need <= _ws(2, 1000)                             # the query is an upper bound
    # one byte short (256-aligned base: no alignment padding) is still refused
    st, h, msg = _create(2, offs, ws=0x100000, ws_bytes=need - 1, box=True, vmax=True)
    assert st == binding.TOP_E_WORKSPACE and h is None
    # an unaligned base needs the padding on top
    st, h, msg = _create(2, offs, ws=0x100010, ws_bytes=need, box=True, vmax=True)
    assert st == binding.TOP_E_WORKSPACE and "align" in msg
    # a pointer without a size, or a size without a pointer
    st, h, msg = _create(2, offs, ws=0x100000, ws_bytes=0)
    assert st == binding.TOP_E_INVALID and "workspace" in msg
    st, h, msg = _create(2, offs, ws=None, ws_bytes=4096)
    assert st == binding.TOP_E_INVALID and "workspace" in msg
