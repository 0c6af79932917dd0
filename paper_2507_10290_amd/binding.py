"""ctypes binding of libtop.so (include/top.h): argument marshalling only.

Every step of the sweep runs in the HIP library; PyTorch only supplies device
memory and the stream.  Importing this module does not touch the GPU; the
first call loads ``libtop.so`` from this package directory and raises if it
is missing (build it with ``python -m paper_2507_10290_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libtop.so")

TOP_OK = 0
TOP_E_INVALID = -1
TOP_E_WORKSPACE = -2
TOP_E_HIP = -3
TOP_E_STATE = -4
TOP_E_NONFINITE = -5
TOP_E_UNSUPPORTED = -6
TOP_E_NOMEM = -7
TOP_FP32 = 0
TOP_FP64 = 1

STATUS_NAMES = {0: "TOP_OK", -1: "TOP_E_INVALID", -2: "TOP_E_WORKSPACE", -3: "TOP_E_HIP", -4: "TOP_E_STATE",
                -5: "TOP_E_NONFINITE", -6: "TOP_E_UNSUPPORTED", -7: "TOP_E_NOMEM"}

# Every entry point declared in include/top.h.
EXPORTED = ["top_default_options", "top_workspace_bytes", "top_workspace_bytes_polytope", "top_create",
            "top_create_polytope", "top_iterate", "top_time_sweeps", "top_residuals", "top_cost",
            "top_coeffs", "top_backward", "top_tune", "top_convergence", "top_get_state", "top_set_state",
            "top_sync_status", "top_get_plan", "top_plan_tiles", "top_destroy", "top_trim", "top_solve_static", "top_last_error"]


class TopOptions(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("n_cont", ctypes.c_int32), ("fix_interior", ctypes.c_int32),
                ("n_samples", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("checkpoint_every", ctypes.c_int32), ("max_taped_iters", ctypes.c_int32),
                ("tile_lanes", ctypes.c_int32), ("halo", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("adapt_rho", ctypes.c_int32), ("tol", ctypes.c_double),
                ("mu", ctypes.c_double), ("tau_incr", ctypes.c_double), ("tau_decr", ctypes.c_double),
                ("local_solve", ctypes.c_int32), ("lbfgs_iters", ctypes.c_int32), ("vel_norm", ctypes.c_int32),
                ("lane_form", ctypes.c_int32), ("chain", ctypes.c_int32)]


class TopPlanInfo(ctypes.Structure):
    _fields_ = [("tile_lanes", ctypes.c_int32), ("n_tiles", ctypes.c_int32), ("halo", ctypes.c_int32),
                ("n_traj", ctypes.c_int32), ("n_seg", ctypes.c_int64), ("used_lanes", ctypes.c_int64),
                ("precision", ctypes.c_int32), ("order", ctypes.c_int32), ("n_cont", ctypes.c_int32),
                ("iters_done", ctypes.c_int32), ("n_fields", ctypes.c_int32), ("ld", ctypes.c_int64),
                ("lane_form", ctypes.c_int32), ("chained", ctypes.c_int32), ("tail_tiles", ctypes.c_int32),
                ("tail_tile_lanes", ctypes.c_int32)]


class TopError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if libtop.so has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2507_10290_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64p, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p
    L.top_default_options.argtypes = [ctypes.POINTER(TopOptions)]
    L.top_default_options.restype = None
    L.top_workspace_bytes.argtypes = [i32, ctypes.c_int64, ctypes.POINTER(TopOptions)]
    L.top_workspace_bytes.restype = ctypes.c_size_t
    L.top_workspace_bytes_polytope.argtypes = [i32, ctypes.c_int64, i32, ctypes.POINTER(TopOptions)]
    L.top_workspace_bytes_polytope.restype = ctypes.c_size_t
    L.top_create.argtypes = [i32, i64p, dp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(TopOptions), vp,
                             ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.top_create.restype = ctypes.c_int
    L.top_create_polytope.argtypes = [i32, i64p, dp, dp, dp, i32, dp, dp, dp, ctypes.POINTER(TopOptions), vp,
                                      ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.top_create_polytope.restype = ctypes.c_int
    L.top_iterate.argtypes = [vp, i32]
    L.top_iterate.restype = ctypes.c_int
    L.top_time_sweeps.argtypes = [vp, i32, ctypes.POINTER(ctypes.c_float)]
    L.top_time_sweeps.restype = ctypes.c_int
    L.top_residuals.argtypes = [vp, dp, dp]
    L.top_residuals.restype = ctypes.c_int
    L.top_cost.argtypes = [vp, dp]
    L.top_cost.restype = ctypes.c_int
    L.top_coeffs.argtypes = [vp, dp]
    L.top_coeffs.restype = ctypes.c_int
    L.top_backward.argtypes = [vp, dp, dp, dp]
    L.top_backward.restype = ctypes.c_int
    L.top_tune.argtypes = [vp, i32]
    L.top_tune.restype = ctypes.c_int
    L.top_get_state.argtypes = [vp, vp]
    L.top_get_state.restype = ctypes.c_int
    L.top_set_state.argtypes = [vp, vp]
    L.top_set_state.restype = ctypes.c_int
    L.top_convergence.argtypes = [vp, vp, vp, vp]
    L.top_convergence.restype = ctypes.c_int
    L.top_sync_status.argtypes = [vp]
    L.top_sync_status.restype = ctypes.c_int
    L.top_get_plan.argtypes = [vp, ctypes.POINTER(TopPlanInfo)]
    L.top_get_plan.restype = ctypes.c_int
    L.top_plan_tiles.argtypes = [i32, i64p, i32, i32, i32, i32, vp, ctypes.c_int64, vp, ctypes.c_int64,
                                 ctypes.POINTER(TopPlanInfo)]
    L.top_plan_tiles.restype = ctypes.c_int
    L.top_destroy.argtypes = [vp]
    L.top_destroy.restype = None
    L.top_trim.argtypes = []
    L.top_trim.restype = None
    L.top_solve_static.argtypes = [i32, i64p, dp, dp, dp, dp, dp, dp, dp, ctypes.POINTER(TopOptions), i32,
                                   dp, dp, dp, dp, vp]
    L.top_solve_static.restype = ctypes.c_int
    L.top_last_error.argtypes = []
    L.top_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int) -> None:
    if status != TOP_OK:
        raise TopError(status, lib().top_last_error().decode(errors="replace"))


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def _dev(x, device):
    """float64, contiguous, on the device (torch is only the allocator here)."""
    import torch
    if x is None:
        return None
    if isinstance(x, np.ndarray):
        x = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64))
    return x.to(device=device, dtype=torch.float64).contiguous()


def default_options() -> TopOptions:
    o = TopOptions()
    lib().top_default_options(ctypes.byref(o))
    return o


# ---------------------------------------------------------------------------
# Thin functions with the C names (handles are integers).
# ---------------------------------------------------------------------------

def top_workspace_bytes(n_traj: int, n_seg_total: int, options: Optional[TopOptions] = None) -> int:
    """Workspace bytes top_create needs for this size (host-only; no device call)."""
    n = lib().top_workspace_bytes(int(n_traj), int(n_seg_total), None if options is None else ctypes.byref(options))
    if n == 0:
        raise TopError(TOP_E_INVALID, lib().top_last_error().decode(errors="replace"))
    return int(n)


def top_workspace_bytes_polytope(n_traj: int, n_seg_total: int, n_faces: int,
                                 options: Optional[TopOptions] = None) -> int:
    n = lib().top_workspace_bytes_polytope(int(n_traj), int(n_seg_total), int(n_faces),
                                           None if options is None else ctypes.byref(options))
    if n == 0:
        raise TopError(TOP_E_INVALID, lib().top_last_error().decode(errors="replace"))
    return int(n)


def _ws_args(workspace, workspace_bytes):
    """(pointer, bytes) of a workspace given as a device tensor or a raw pointer, or (None, 0)."""
    if workspace is None:
        return None, 0
    if isinstance(workspace, int):
        return ctypes.c_void_p(workspace), int(workspace_bytes)
    nbytes = workspace.numel() * workspace.element_size()
    return ctypes.c_void_p(workspace.data_ptr()), int(workspace_bytes if workspace_bytes else nbytes)


def top_create(seg_offsets: Sequence[int], waypoints, durations, rho, *, bc=None, box_lo=None,
               box_hi=None, vmax=None, options: Optional[TopOptions] = None, workspace=None,
               workspace_bytes: int = 0, stream: int = 0) -> int:
    """Device tensors (float64) in, handle out.  seg_offsets is a host int64 sequence; workspace is a
    device tensor (or pointer) of at least top_workspace_bytes bytes, or None for the library's pool."""
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.int64))
    h = ctypes.c_void_p()
    wp, wb = _ws_args(workspace, workspace_bytes)
    st = lib().top_create(int(offs.shape[0] - 1), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                          _ptr(waypoints), _ptr(durations), _ptr(bc), _ptr(box_lo), _ptr(box_hi),
                          _ptr(vmax), _ptr(rho), None if options is None else ctypes.byref(options),
                          wp, wb, ctypes.c_void_p(stream), ctypes.byref(h))
    _check(st)
    return h.value


def top_create_polytope(seg_offsets: Sequence[int], waypoints, durations, rho, faces, *, bc=None, vmax=None,
                        options: Optional[TopOptions] = None, workspace=None, workspace_bytes: int = 0,
                        stream: int = 0) -> int:
    """Like top_create with a polytope corridor: faces is a float64 device tensor [S, K, 4] (a, b)."""
    offs = np.ascontiguousarray(np.asarray(seg_offsets, dtype=np.int64))
    h = ctypes.c_void_p()
    wp, wb = _ws_args(workspace, workspace_bytes)
    st = lib().top_create_polytope(int(offs.shape[0] - 1), offs.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _ptr(waypoints), _ptr(durations), _ptr(bc), int(faces.shape[1]), _ptr(faces),
                                   _ptr(vmax), _ptr(rho), None if options is None else ctypes.byref(options),
                                   wp, wb, ctypes.c_void_p(stream), ctypes.byref(h))
    _check(st)
    return h.value


def top_iterate(h: int, k: int) -> None:
    _check(lib().top_iterate(ctypes.c_void_p(h), int(k)))


def top_time_sweeps(h: int, k: int) -> float:
    ms = ctypes.c_float()
    _check(lib().top_time_sweeps(ctypes.c_void_p(h), int(k), ctypes.byref(ms)))
    return float(ms.value)


def top_residuals(h: int, r_primal, r_dual) -> None:
    _check(lib().top_residuals(ctypes.c_void_p(h), _ptr(r_primal), _ptr(r_dual)))


def top_cost(h: int, cost) -> None:
    _check(lib().top_cost(ctypes.c_void_p(h), _ptr(cost)))


def top_coeffs(h: int, coeffs) -> None:
    _check(lib().top_coeffs(ctypes.c_void_p(h), _ptr(coeffs)))


def top_backward(h: int, dcost, dwaypoints, ddurations) -> None:
    _check(lib().top_backward(ctypes.c_void_p(h), _ptr(dcost), _ptr(dwaypoints), _ptr(ddurations)))


def top_tune(h: int, k_probe: int) -> None:
    _check(lib().top_tune(ctypes.c_void_p(h), int(k_probe)))


def top_convergence(h: int, iters, rho, done) -> None:
    _check(lib().top_convergence(ctypes.c_void_p(h), _ptr(iters), _ptr(rho), _ptr(done)))


def top_get_state(h: int, state) -> None:
    _check(lib().top_get_state(ctypes.c_void_p(h), _ptr(state)))


def top_set_state(h: int, state) -> None:
    _check(lib().top_set_state(ctypes.c_void_p(h), _ptr(state)))


def top_sync_status(h: int) -> None:
    _check(lib().top_sync_status(ctypes.c_void_p(h)))


def top_get_plan(h: int) -> dict:
    info = TopPlanInfo()
    _check(lib().top_get_plan(ctypes.c_void_p(h), ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in TopPlanInfo._fields_}


TOP_HALO_BIT = 1 << 30


def top_plan_tiles(seg_offsets, tile_lanes: int, halo: int, tiles_per_round: int = 0, tail_tile_lanes: int = 0):
    """Host only: the tile plan for these trajectory lengths (top_plan_tiles).  Returns (info dict,
    lanes int32 [n_tiles, tile_lanes], chain int32 [n_tiles, 4] or an empty [0, 4] array, tail lanes
    int32 [tail_tiles, tail_tile_lanes])."""
    off = np.ascontiguousarray(seg_offsets, dtype=np.int64)
    n_traj = len(off) - 1
    offp = off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    info = TopPlanInfo()
    _check(lib().top_plan_tiles(n_traj, offp, tile_lanes, halo, tiles_per_round, tail_tile_lanes, None, 0, None, 0,
                                ctypes.byref(info)))
    n_main = info.n_tiles * tile_lanes
    allv = np.empty(n_main + info.tail_tiles * info.tail_tile_lanes, dtype=np.int32)
    chain = np.empty((info.n_tiles if info.chained else 0, 4), dtype=np.int32)
    _check(lib().top_plan_tiles(n_traj, offp, tile_lanes, halo, tiles_per_round, tail_tile_lanes, allv.ctypes.data,
                                allv.size, chain.ctypes.data, chain.size, ctypes.byref(info)))
    lanes = allv[:n_main].reshape(info.n_tiles, tile_lanes)
    tail = allv[n_main:].reshape(info.tail_tiles, max(info.tail_tile_lanes, 1))
    return {f: getattr(info, f) for f, _ in TopPlanInfo._fields_}, lanes, chain, tail


def top_destroy(h: int) -> None:
    lib().top_destroy(ctypes.c_void_p(h))


def top_trim() -> None:
    lib().top_trim()


# ---------------------------------------------------------------------------
# Convenience wrapper.
# ---------------------------------------------------------------------------

class TopProblem:
    """A batch of trajectories on one GPU, owned by one library handle."""

    def __init__(self, seg_offsets, waypoints, durations, rho, *, order: int = 3, n_cont: int = 0,
                 bc=None, box_lo=None, box_hi=None, faces=None, vmax=None, precision: str = "fp32",
                 fix_interior: bool = True, checkpoint_every: int = 0, max_taped_iters: int = 0,
                 tile_lanes: int = 0, halo: int = 0, use_graph: bool = True, check_every: int = 0,
                 adapt_rho: bool = False, tol: float = 0.05, mu: float = 10.0, tau_incr: float = 1.1,
                 tau_decr: float = 1.1, numeric: bool = False, lbfgs_iters: int = 10, vel_norm: int = 2,
                 lane_form: int = 0, chain: int = 0, device: str = "cuda:0", stream=None,
                 library_pool: bool = False):
        """Create the handle.  By default its state lives in a workspace allocated by torch on the
        handle's stream (released with the handle); library_pool=True uses the library's pool."""
        import torch
        self.device = torch.device(device)
        self.seg_offsets = np.asarray(seg_offsets, dtype=np.int64)
        self.B = int(self.seg_offsets.shape[0] - 1)
        self.S = int(self.seg_offsets[-1])
        self.order = int(order)
        self.n = 2 * self.order
        o = default_options()
        o.order = self.order
        o.n_cont = int(n_cont)
        o.fix_interior = 1 if fix_interior else 0
        o.precision = TOP_FP64 if precision == "fp64" else TOP_FP32
        o.checkpoint_every = int(checkpoint_every)
        o.max_taped_iters = int(max_taped_iters)
        o.tile_lanes = int(tile_lanes)
        o.halo = int(halo)
        o.use_graph = 1 if use_graph else 0
        o.check_every = int(check_every)
        o.adapt_rho = 1 if adapt_rho else 0
        o.tol, o.mu, o.tau_incr, o.tau_decr = float(tol), float(mu), float(tau_incr), float(tau_decr)
        o.local_solve = 1 if numeric else 0
        o.lbfgs_iters = int(lbfgs_iters)
        o.vel_norm = int(vel_norm)
        o.lane_form = int(lane_form)
        o.chain = int(chain)
        self.options = o
        self.h = None
        self.workspace = None
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if faces is not None and (box_lo is not None or box_hi is not None):
            raise ValueError("give a box corridor or polytope faces, not both")
        cur = torch.cuda.current_stream(self.device)
        if self.stream != cur:
            self.stream.wait_stream(cur)  # inputs produced on the current stream
        # Staging copies and the workspace are allocated on the handle's stream, so the caching
        # allocator reuses their memory only after the work queued there (which reads them).
        with torch.cuda.stream(self.stream):
            args = [_dev(x, self.device) for x in (waypoints, durations, rho, bc, box_lo, box_hi, vmax, faces)]
            if not library_pool:
                nb = (top_workspace_bytes_polytope(self.B, self.S, int(args[7].shape[1]), o) if faces is not None
                      else top_workspace_bytes(self.B, self.S, o))
                self.workspace = torch.empty(nb, dtype=torch.uint8, device=self.device)
            if faces is not None:
                self.h = top_create_polytope(self.seg_offsets, args[0], args[1], args[2], args[7], bc=args[3],
                                             vmax=args[6], options=o, workspace=self.workspace,
                                             stream=self.stream.cuda_stream)
            else:
                self.h = top_create(self.seg_offsets, args[0], args[1], args[2], bc=args[3], box_lo=args[4],
                                    box_hi=args[5], vmax=args[6], options=o, workspace=self.workspace,
                                    stream=self.stream.cuda_stream)

    @classmethod
    def from_workload(cls, w, **kw):
        kw.setdefault("precision", w.precision)
        return cls(w.seg_offsets, w.waypoints, w.durations, w.rho, order=w.order, n_cont=w.n_cont,
                   bc=w.bc, box_lo=w.box_lo, box_hi=w.box_hi, faces=getattr(w, "faces", None), vmax=w.vmax,
                   fix_interior=w.fix_interior, **kw)

    def _empty(self, *shape):
        import torch
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def iterate(self, k: int) -> "TopProblem":
        top_iterate(self.h, k)
        return self

    def time_sweeps(self, k: int) -> float:
        """Run k sweeps and return the device milliseconds of the sweep launches alone."""
        return top_time_sweeps(self.h, k)

    def residuals(self):
        rp, rd = self._empty(self.B), self._empty(self.B)
        top_residuals(self.h, rp, rd)
        return rp, rd

    def cost(self):
        J = self._empty(self.B)
        top_cost(self.h, J)
        return J

    def coeffs(self):
        c = self._empty(self.S, 3, self.n)
        top_coeffs(self.h, c)
        return c

    def backward(self, dcost):
        dcost = _dev(dcost, self.device)
        dP, dT = self._empty(self.S + self.B, 3), self._empty(self.S)
        top_backward(self.h, dcost, dP, dT)
        return dP, dT

    def tune(self, k_probe: int = 20) -> dict:
        top_tune(self.h, k_probe)
        return self.plan()

    def convergence(self):
        """(sweeps applied, current rho, stopped) per trajectory, as device tensors."""
        import torch
        it = torch.empty(self.B, dtype=torch.int32, device=self.device)
        done = torch.empty(self.B, dtype=torch.uint8, device=self.device)
        rho = self._empty(self.B)
        top_convergence(self.h, it, rho, done)
        return it, rho, done.bool()

    def get_state(self):
        """The iterate state as a device tensor [n_fields, ld] in the iterate precision."""
        import torch
        info = self.plan()
        dt = torch.float64 if self.options.precision == TOP_FP64 else torch.float32
        st = torch.empty(info["n_fields"], info["ld"], dtype=dt, device=self.device)
        top_get_state(self.h, st)
        return st

    def set_state(self, state) -> None:
        """Replace the iterate (a tensor shaped and typed like get_state's)."""
        import torch
        dt = torch.float64 if self.options.precision == TOP_FP64 else torch.float32
        info = self.plan()
        if tuple(state.shape) != (info["n_fields"], info["ld"]) or state.dtype != dt:
            raise ValueError("state must be shaped and typed like get_state()")
        top_set_state(self.h, state.contiguous())

    def sync_status(self) -> None:
        top_sync_status(self.h)

    def plan(self) -> dict:
        return top_get_plan(self.h)

    def close(self) -> None:
        if getattr(self, "h", None):
            top_destroy(self.h)
            self.h = None
        # The workspace was allocated on the handle's stream: the caching allocator hands it out
        # again only in that stream's order, after the work queued there.
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Autograd: J(waypoints, durations) through Init and K sweeps.
# ---------------------------------------------------------------------------

def _autograd_function():
    import torch

    class TopCost(torch.autograd.Function):
        """Cost per trajectory after `iters` sweeps; backward runs the library's reverse pass.

        Gradients flow to waypoints [S+B,3] and durations [S]; corridor, vmax and rho are
        held constant.  The tape keeps the state every `checkpoint_every` sweeps.
        """

        @staticmethod
        def forward(ctx, waypoints, durations, seg_offsets, rho, box_lo, box_hi, vmax, iters,
                    checkpoint_every, precision, order):
            prob = TopProblem(seg_offsets, waypoints.detach(), durations.detach(), rho, order=order,
                              box_lo=box_lo, box_hi=box_hi, vmax=vmax, precision=precision,
                              checkpoint_every=checkpoint_every, max_taped_iters=iters,
                              device=str(waypoints.device))
            prob.iterate(iters)
            ctx.prob = prob
            return prob.cost()

        @staticmethod
        def backward(ctx, gJ):
            # The handle stays open until ctx is released, so a graph kept with retain_graph=True
            # can be differentiated again (the reverse pass replays the blocks it needs).
            dP, dT = ctx.prob.backward(gJ.detach().to(torch.float64).contiguous())
            return dP, dT, None, None, None, None, None, None, None, None, None

    return TopCost


_TopCost = None


def top_cost_fn(waypoints, durations, seg_offsets, rho, *, box_lo=None, box_hi=None, vmax=None,
                iters: int = 100, checkpoint_every: int = 10, precision: str = "fp32", order: int = 3):
    """Differentiable cost J[B] of the trajectories after `iters` sweeps (torch tensors on the GPU)."""
    global _TopCost
    if _TopCost is None:
        _TopCost = _autograd_function()
    return _TopCost.apply(waypoints, durations, seg_offsets, rho, box_lo, box_hi, vmax, iters,
                          checkpoint_every, precision, order)
