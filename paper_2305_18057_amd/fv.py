"""ctypes binding of ``libfv.so`` (the C ABI declared in ``include/fv.h``).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch supplies device memory (the grid workspace and the server arena are
``torch.uint8`` CUDA tensors) and the HIP stream (torch's current stream).
Importing this module loads the library and fails loudly if it is missing;
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

from . import cases as _cases

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FV_LIBRARY") or os.path.join(_HERE, "libfv.so")

FV_OK, FV_PENDING = 0, 1
FV_E_INVAL, FV_E_NOMEM, FV_E_DEVICE, FV_E_NONPHYSICAL = -1, -2, -3, -4
FV_E_UNSUPPORTED, FV_E_BUSY, FV_E_NOTFOUND, FV_E_CANCELLED = -5, -6, -7, -8
FLAG_NONPHYSICAL, FLAG_CONVERGED, FLAG_T_END, FLAG_STEP_LIMIT = 1, 2, 4, 8


class FVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fv status {status}: {msg}")
        self.status = status


class fv_bc(C.Structure):
    _fields_ = [("kind", C.c_int), ("nbr_block", C.c_int), ("nbr_face", C.c_int),
                ("orient", C.c_int), ("prim_in", C.c_double * 5)]


class fv_block_desc(C.Structure):
    _fields_ = [("ni", C.c_int), ("nj", C.c_int), ("nk", C.c_int),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double)),
                ("origin", C.c_double * 3), ("h", C.c_double * 3), ("face", fv_bc * 6)]


class fv_grid_desc(C.Structure):
    _fields_ = [("ndim", C.c_int), ("nblocks", C.c_int),
                ("blocks", C.POINTER(fv_block_desc)), ("gamma", C.c_double),
                ("with_source", C.c_int)]


class fv_params(C.Structure):
    _fields_ = [("cfl", C.c_double), ("dt_fixed", C.c_double), ("t_end", C.c_double),
                ("precision", C.c_int), ("limiter", C.c_int), ("eps", C.c_double),
                ("kappa", C.c_double), ("entropy_fix", C.c_double), ("rk", C.c_int),
                ("qref", C.c_double * 5), ("mu", C.c_double), ("prandtl", C.c_double)]


class fv_step_info(C.Structure):
    _fields_ = [("steps", C.c_longlong), ("t", C.c_double), ("dt_last", C.c_double),
                ("norms", C.c_double * 5), ("norm", C.c_double), ("drop", C.c_double),
                ("flags", C.c_int)]


class fv_grid_stats(C.Structure):
    _fields_ = [("cells", C.c_longlong), ("tiles", C.c_longlong), ("tile_rows", C.c_int),
                ("tile_cols", C.c_int), ("tile_ny", C.c_int), ("launch_blocks", C.c_int),
                ("workspace_bytes", C.c_size_t), ("last_stage_ms", C.c_double * 4)]


class fv_server_desc(C.Structure):
    _fields_ = [("d_arena", C.c_void_p), ("arena_bytes", C.c_size_t), ("hip_stream", C.c_void_p),
                ("max_instances", C.c_int), ("autotune_cache", C.c_char_p),
                ("precision", C.c_int), ("steps_per_launch", C.c_int), ("flags", C.c_int)]


class fv_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_longlong), ("admitted", C.c_longlong),
                ("completed", C.c_longlong), ("cancelled", C.c_longlong),
                ("failed", C.c_longlong), ("launches", C.c_longlong),
                ("cell_steps", C.c_longlong), ("resident", C.c_int), ("queued", C.c_int),
                ("arena_used", C.c_size_t), ("arena_peak", C.c_size_t)]


EXPORTS = [
    "fv_strerror", "fv_last_error", "fv_default_params", "fv_grid_workspace_bytes",
    "fv_create_grid", "fv_destroy_grid", "fv_set_state", "fv_get_state", "fv_set_source",
    "fv_residual",
    "fv_ghost_count", "fv_ghosts", "fv_step", "fv_step_timed", "fv_solve", "fv_tune",
    "fv_grid_get_stats",
    "fv_server_create", "fv_submit", "fv_submit_with_source", "fv_poll", "fv_cancel",
    "fv_request_times",
    "fv_server_clock", "fv_server_get_stats", "fv_server_destroy",
    "fv_noalloc_scratch_bytes", "fv_step_noalloc",
    "fv_hetero_workspace_bytes", "fv_hetero_create", "fv_hetero_set_state", "fv_hetero_get_state",
    "fv_hetero_step", "fv_hetero_destroy",
]

_lib = None


def lib():
    """Load libfv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FileNotFoundError(
            f"{LIB_PATH} is missing: build it with paper_2305_18057_amd/build.py "
            "(there is no CPU fallback)")
    # device memory and streams come from PyTorch, so the library must run on
    # PyTorch's HIP runtime: importing torch first makes the dynamic loader
    # resolve the library's libamdhip64 to that copy (loaded the other way
    # round, two runtimes would share the process and neither would know the
    # other's memory and streams)
    _torch()
    L = C.CDLL(LIB_PATH)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    L.fv_strerror.restype = C.c_char_p
    L.fv_strerror.argtypes = [C.c_int]
    L.fv_last_error.restype = C.c_char_p
    L.fv_default_params.argtypes = [C.POINTER(fv_params)]
    L.fv_grid_workspace_bytes.restype = C.c_size_t
    L.fv_grid_workspace_bytes.argtypes = [C.POINTER(fv_grid_desc), C.c_int]
    L.fv_create_grid.argtypes = [C.POINTER(fv_grid_desc), vp, C.c_size_t, vp, C.POINTER(vp)]
    L.fv_destroy_grid.argtypes = [vp]
    L.fv_set_state.argtypes = [vp, vp, C.c_int]
    L.fv_get_state.argtypes = [vp, vp, C.c_int]
    L.fv_set_source.argtypes = [vp, vp, C.c_int]
    L.fv_residual.argtypes = [vp, C.POINTER(fv_params), vp, C.c_int, dp]
    L.fv_ghost_count.restype = C.c_size_t
    L.fv_ghost_count.argtypes = [vp]
    L.fv_ghosts.argtypes = [vp, vp, C.c_int]
    L.fv_step.argtypes = [vp, C.POINTER(fv_params), C.c_int, C.POINTER(fv_step_info)]
    L.fv_step_timed.argtypes = [vp, C.POINTER(fv_params), C.c_int, C.POINTER(fv_step_info), dp]
    L.fv_solve.argtypes = [vp, C.POINTER(fv_params), C.c_double, C.c_longlong,
                           C.POINTER(fv_step_info)]
    L.fv_tune.argtypes = [vp, C.POINTER(fv_params), C.c_char_p]
    L.fv_grid_get_stats.argtypes = [vp, C.POINTER(fv_grid_stats)]
    L.fv_server_create.argtypes = [C.POINTER(fv_server_desc), C.POINTER(vp)]
    L.fv_submit.argtypes = [vp, C.POINTER(fv_grid_desc), dp, C.POINTER(fv_params), C.c_double,
                            C.c_longlong, C.POINTER(C.c_ulonglong)]
    L.fv_submit_with_source.argtypes = [vp, C.POINTER(fv_grid_desc), dp, dp, C.POINTER(fv_params),
                                        C.c_double, C.c_longlong, C.POINTER(C.c_ulonglong)]
    L.fv_poll.argtypes = [vp, C.c_ulonglong, dp, C.c_size_t, C.POINTER(fv_step_info)]
    L.fv_cancel.argtypes = [vp, C.c_ulonglong]
    L.fv_request_times.argtypes = [vp, C.c_ulonglong, dp]
    L.fv_server_clock.restype = C.c_double
    L.fv_server_clock.argtypes = [vp]
    L.fv_server_get_stats.argtypes = [vp, C.POINTER(fv_server_stats)]
    L.fv_server_destroy.argtypes = [vp]
    L.fv_noalloc_scratch_bytes.restype = C.c_size_t
    L.fv_noalloc_scratch_bytes.argtypes = []
    L.fv_step_noalloc.argtypes = [C.POINTER(fv_grid_desc), vp, C.POINTER(fv_params), C.c_int, vp,
                                  C.POINTER(fv_step_info)]
    L.fv_hetero_workspace_bytes.restype = C.c_size_t
    L.fv_hetero_workspace_bytes.argtypes = [C.POINTER(fv_grid_desc), C.c_int]
    L.fv_hetero_create.argtypes = [C.POINTER(fv_grid_desc), C.c_int, C.c_int, vp, C.c_size_t, vp,
                                   C.POINTER(vp)]
    L.fv_hetero_set_state.argtypes = [vp, dp]
    L.fv_hetero_get_state.argtypes = [vp, dp]
    L.fv_hetero_step.argtypes = [vp, C.POINTER(fv_params), C.c_int, C.POINTER(fv_step_info), dp]
    L.fv_hetero_destroy.argtypes = [vp]
    _lib = L
    return L


def _check(status: int, ok=(FV_OK,)):
    if status not in ok:
        raise FVError(status, lib().fv_last_error().decode(errors="replace"))
    return status


# ---------------------------------------------------------------------------
# marshalling of the case objects of ``cases``
# ---------------------------------------------------------------------------
class GridDesc:
    """Keeps the ctypes descriptor and the host arrays it points to alive."""

    def __init__(self, case: "_cases.Case"):
        nb = len(case.blocks)
        self.arr = (fv_block_desc * nb)()
        self.keep = []
        for b, blk in enumerate(case.blocks):
            d = self.arr[b]
            d.ni, d.nj, d.nk = blk.ni, blk.nj, blk.nk
            if blk.x is not None:
                x = np.ascontiguousarray(blk.x, dtype=np.float64)
                y = np.ascontiguousarray(blk.y, dtype=np.float64)
                self.keep += [x, y]
                d.x = x.ctypes.data_as(C.POINTER(C.c_double))
                d.y = y.ctypes.data_as(C.POINTER(C.c_double))
            if getattr(blk, "z", None) is not None:
                z = np.ascontiguousarray(blk.z, dtype=np.float64)
                self.keep.append(z)
                d.z = z.ctypes.data_as(C.POINTER(C.c_double))
            for a in range(3):
                d.origin[a] = blk.origin[a]
                d.h[a] = blk.h[a]
            for f in range(6):
                bc = blk.bc[f]
                d.face[f].kind = bc.kind
                d.face[f].nbr_block = bc.nbr_block
                d.face[f].nbr_face = bc.nbr_face
                d.face[f].orient = getattr(bc, "orient", 0)
                for a in range(5):
                    d.face[f].prim_in[a] = bc.prim[a]
        self.desc = fv_grid_desc(case.ndim, nb, self.arr, case.gamma,
                                 1 if getattr(case, "source", None) is not None else 0)


def make_params(p: "_cases.Params") -> fv_params:
    q = list(p.qref) + [1.0] * (5 - len(p.qref))
    return fv_params(p.cfl, p.dt_fixed, p.t_end, p.precision, p.limiter, p.eps, p.kappa,
                     p.entropy_fix, getattr(p, "rk", 3), (C.c_double * 5)(*q[:5]),
                     getattr(p, "mu", 0.0), getattr(p, "prandtl", 0.72))


def info_dict(info: fv_step_info) -> dict:
    return dict(steps=info.steps, t=info.t, dt_last=info.dt_last, norms=np.array(info.norms[:]),
                norm=info.norm, drop=info.drop, flags=info.flags)


def _torch():
    import torch
    return torch


def current_stream_handle(device=None) -> int:
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


class Grid:
    """One grid instance resident in a torch-allocated device workspace."""

    def __init__(self, case: "_cases.Case", device="cuda", stream: Optional[int] = None):
        torch = _torch()
        L = lib()
        self.case = case
        self.nv = case.nv
        self.size = sum(self.nv * b.ncells for b in case.blocks)
        self._gd = GridDesc(case)
        nbytes = L.fv_grid_workspace_bytes(C.byref(self._gd.desc), case.params.precision)
        if nbytes == 0:
            _check(FV_E_INVAL)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.stream = current_stream_handle(self.workspace.device) if stream is None else stream
        h = C.c_void_p()
        _check(L.fv_create_grid(C.byref(self._gd.desc), C.c_void_p(self.workspace.data_ptr()),
                                C.c_size_t(nbytes), C.c_void_p(self.stream), C.byref(h)))
        self._h = h
        self.workspace_bytes = int(nbytes)
        if getattr(case, "source", None) is not None:
            self.set_source(case.source_flat())

    def close(self):
        if getattr(self, "_h", None):
            lib().fv_destroy_grid(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # state --------------------------------------------------------------
    def set_state(self, U, check=True) -> int:
        torch = _torch()
        if isinstance(U, torch.Tensor):
            assert U.dtype == torch.float64 and U.is_contiguous() and U.numel() == self.size
            st = lib().fv_set_state(self._h, C.c_void_p(U.data_ptr()), 1 if U.is_cuda else 0)
        else:
            a = np.ascontiguousarray(U, dtype=np.float64).ravel()
            assert a.size == self.size
            st = lib().fv_set_state(self._h, C.c_void_p(a.ctypes.data), 0)
        if check:
            _check(st)
        return st

    def set_source(self, S) -> None:
        """Cell-averaged source S_h in the state layout (None: zero)."""
        torch = _torch()
        if S is None:
            _check(lib().fv_set_source(self._h, None, 0))
        elif isinstance(S, torch.Tensor):
            assert S.dtype == torch.float64 and S.is_contiguous() and S.numel() == self.size
            _check(lib().fv_set_source(self._h, C.c_void_p(S.data_ptr()), 1 if S.is_cuda else 0))
        else:
            a = np.ascontiguousarray(S, dtype=np.float64).ravel()
            assert a.size == self.size
            _check(lib().fv_set_source(self._h, C.c_void_p(a.ctypes.data), 0))

    def get_state(self, out=None):
        torch = _torch()
        if out is not None and isinstance(out, torch.Tensor):
            _check(lib().fv_get_state(self._h, C.c_void_p(out.data_ptr()), 1 if out.is_cuda else 0))
            return out
        a = np.empty(self.size)
        _check(lib().fv_get_state(self._h, C.c_void_p(a.ctypes.data), 0))
        return a

    # evaluation ----------------------------------------------------------
    def residual(self, params=None, out=None):
        p = make_params(params or self.case.params)
        norms = (C.c_double * 5)()
        torch = _torch()
        if out is not None and isinstance(out, torch.Tensor):
            _check(lib().fv_residual(self._h, C.byref(p), C.c_void_p(out.data_ptr()), 1, norms))
            return out, np.array(norms[:])
        R = np.empty(self.size)
        _check(lib().fv_residual(self._h, C.byref(p), C.c_void_p(R.ctypes.data), 0, norms))
        return R, np.array(norms[:])

    def ghosts(self):
        n = lib().fv_ghost_count(self._h)
        G = np.empty(int(n))
        _check(lib().fv_ghosts(self._h, C.c_void_p(G.ctypes.data), 0))
        return G

    def step(self, params=None, nsteps=1, check=True):
        p = make_params(params or self.case.params)
        info = fv_step_info()
        st = lib().fv_step(self._h, C.byref(p), int(nsteps), C.byref(info))
        if check:
            _check(st)
        d = info_dict(info)
        d["status"] = st
        return d

    def step_timed(self, params=None, nsteps=1):
        """Steps launched one by one with HIP events; returns (info, stage_ms[4])."""
        p = make_params(params or self.case.params)
        info = fv_step_info()
        ms = (C.c_double * 4)()
        _check(lib().fv_step_timed(self._h, C.byref(p), int(nsteps), C.byref(info), ms))
        return info_dict(info), np.array(ms[:])

    def solve(self, params=None, drop_tol=1e-8, max_steps=2000, check=True):
        p = make_params(params or self.case.params)
        info = fv_step_info()
        st = lib().fv_solve(self._h, C.byref(p), float(drop_tol), int(max_steps), C.byref(info))
        if check:
            _check(st)
        d = info_dict(info)
        d["status"] = st
        return d

    def tune(self, params=None, cache_path: Optional[str] = None):
        p = make_params(params or self.case.params)
        _check(lib().fv_tune(self._h, C.byref(p), cache_path.encode() if cache_path else None))
        return self.stats()

    def stats(self) -> dict:
        s = fv_grid_stats()
        _check(lib().fv_grid_get_stats(self._h, C.byref(s)))
        return dict(cells=s.cells, tiles=s.tiles, tile_rows=s.tile_rows, tile_cols=s.tile_cols,
                    tile_ny=s.tile_ny, launch_blocks=s.launch_blocks,
                    workspace_bytes=s.workspace_bytes)


def step_noalloc(case: "_cases.Case", U, params=None, nsteps=1, stream: Optional[int] = None,
                 check=True) -> dict:
    """fv_step_noalloc: advance the device state tensor U (float64, contiguous,
    the case's size) in place by nsteps steps, with no workspace."""
    torch = _torch()
    assert isinstance(U, torch.Tensor) and U.is_cuda and U.dtype == torch.float64
    assert U.is_contiguous() and U.numel() == sum(case.nv * b.ncells for b in case.blocks)
    gd = GridDesc(case)
    p = make_params(params or case.params)
    info = fv_step_info()
    s = current_stream_handle(U.device) if stream is None else stream
    st = lib().fv_step_noalloc(C.byref(gd.desc), C.c_void_p(U.data_ptr()), C.byref(p), int(nsteps),
                               C.c_void_p(s), C.byref(info))
    if check:
        _check(st)
    d = info_dict(info)
    d["status"] = st
    return d


def workspace_bytes(case) -> int:
    gd = GridDesc(case)
    return int(lib().fv_grid_workspace_bytes(C.byref(gd.desc), case.params.precision))


# ---------------------------------------------------------------------------
# server
# ---------------------------------------------------------------------------
class Server:
    """Continuous-batching solver service over one torch-allocated arena.

    ``dry_run=True`` exercises the scheduler without touching a device (every
    request takes one step per step slot and returns its initial state)."""

    FLAG_DRYRUN = 1

    def __init__(self, arena_bytes: int, max_instances=64, precision=_cases.FP32_FLUX,
                 steps_per_launch=10, autotune_cache: Optional[str] = None, device="cuda",
                 dry_run=False):
        self._cache = autotune_cache.encode() if autotune_cache else None
        if dry_run:
            self.arena = None
            ptr, stream = None, None
        else:
            torch = _torch()
            self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=device)
            ptr = self.arena.data_ptr()
            stream = current_stream_handle(self.arena.device)
        self.stream = stream
        d = fv_server_desc(C.c_void_p(ptr), C.c_size_t(int(arena_bytes)), C.c_void_p(stream),
                           int(max_instances), self._cache, int(precision), int(steps_per_launch),
                           self.FLAG_DRYRUN if dry_run else 0)
        h = C.c_void_p()
        _check(lib().fv_server_create(C.byref(d), C.byref(h)))
        self._h = h
        self._sizes = {}

    def submit(self, case, drop_tol=1e-8, max_steps=2000, params=None) -> int:
        gd = GridDesc(case)
        U = np.ascontiguousarray(case.state_flat(), dtype=np.float64)
        p = make_params(params or case.params)
        t = C.c_ulonglong()
        Up = U.ctypes.data_as(C.POINTER(C.c_double))
        if getattr(case, "source", None) is not None:
            S = np.ascontiguousarray(case.source_flat(), dtype=np.float64)
            _check(lib().fv_submit_with_source(self._h, C.byref(gd.desc), Up,
                                               S.ctypes.data_as(C.POINTER(C.c_double)), C.byref(p),
                                               float(drop_tol), int(max_steps), C.byref(t)))
        else:
            _check(lib().fv_submit(self._h, C.byref(gd.desc), Up, C.byref(p), float(drop_tol),
                                   int(max_steps), C.byref(t)))
        self._sizes[t.value] = U.size
        return t.value

    def times(self, ticket: int):
        """(submitted, admitted, done) on the server clock; negative = not yet."""
        out = (C.c_double * 3)()
        _check(lib().fv_request_times(self._h, C.c_ulonglong(ticket), out))
        return tuple(out[:])

    def clock(self) -> float:
        return lib().fv_server_clock(self._h)

    def poll(self, ticket: int):
        """None while pending, else (status, U, info); info["times"] holds the
        request's (submitted, admitted, done) server-clock times."""
        n = self._sizes.get(ticket, 0)
        tm = (C.c_double * 3)()
        if lib().fv_request_times(self._h, C.c_ulonglong(ticket), tm) == FV_OK and tm[2] < 0:
            return None
        U = np.empty(n)
        info = fv_step_info()
        st = lib().fv_poll(self._h, C.c_ulonglong(ticket), U.ctypes.data_as(C.POINTER(C.c_double)),
                           C.c_size_t(n), C.byref(info))
        if st == FV_PENDING:
            return None
        if st not in (FV_OK, FV_E_NONPHYSICAL, FV_E_CANCELLED):
            _check(st)
        self._sizes.pop(ticket, None)
        d = info_dict(info)
        d["times"] = tuple(tm[:])
        return st, U, d

    def cancel(self, ticket: int) -> int:
        return lib().fv_cancel(self._h, C.c_ulonglong(ticket))

    def stats(self) -> dict:
        s = fv_server_stats()
        _check(lib().fv_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in fv_server_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            lib().fv_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Hetero:
    """One 2D block stepped by the GPU (columns [0, split)) and a pool of
    host-core workers (columns [split, ni)) together, exchanging the two
    columns on each side of the cut every RK substep."""

    def __init__(self, case: "_cases.Case", split: int, cpu_workers: int, device="cuda",
                 stream: Optional[int] = None):
        torch = _torch()
        L = lib()
        self.case = case
        self.size = sum(case.nv * b.ncells for b in case.blocks)
        self._gd = GridDesc(case)
        nbytes = L.fv_hetero_workspace_bytes(C.byref(self._gd.desc), int(split))
        if nbytes == 0:
            _check(FV_E_INVAL)
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
        self.stream = current_stream_handle(self.workspace.device) if stream is None else stream
        h = C.c_void_p()
        _check(L.fv_hetero_create(C.byref(self._gd.desc), int(split), int(cpu_workers),
                                  C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes),
                                  C.c_void_p(self.stream), C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().fv_hetero_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_state(self, U, check=True) -> int:
        a = np.ascontiguousarray(U, dtype=np.float64).ravel()
        assert a.size == self.size
        st = lib().fv_hetero_set_state(self._h, a.ctypes.data_as(C.POINTER(C.c_double)))
        if check:
            _check(st)
        return st

    def get_state(self):
        a = np.empty(self.size)
        _check(lib().fv_hetero_get_state(self._h, a.ctypes.data_as(C.POINTER(C.c_double))))
        return a

    def step(self, params=None, nsteps=1, check=True):
        """nsteps steps; the info dict also holds times_ms = (GPU stage kernels,
        host substeps, exchanges with their synchronizations, whole call)."""
        p = make_params(params or self.case.params)
        info = fv_step_info()
        tm = (C.c_double * 4)()
        st = lib().fv_hetero_step(self._h, C.byref(p), int(nsteps), C.byref(info), tm)
        if check:
            _check(st)
        d = info_dict(info)
        d["status"] = st
        d["times_ms"] = list(tm)
        return d
