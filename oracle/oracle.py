"""Python handle on the plain FP64 CPU reference (``oracle/fv_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the package smoke check
and by the benchmark's CPU-baseline leg.  The product path never imports it.
It marshals a case description (duck-typed: ``ndim``, ``gamma``, ``blocks``,
``state_flat()``) into the oracle's own C structures; no arithmetic of the
method happens here.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fv_oracle.c")
LIB = os.path.join(HERE, "liborc.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math", "-ffp-contract=off"]
# host sanitizer build (ORC_SANITIZE=1): AddressSanitizer and UndefinedBehaviorSanitizer,
# loaded by a Python started with the matching runtime preloaded (see sanitize_env)
SAN_LIB = os.path.join(HERE, "liborc_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
SANITIZE = os.environ.get("ORC_SANITIZE") == "1"

OK, E_INVAL, E_NOMEM, E_NONPHYSICAL = 0, -1, -2, -4


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction); with
    sanitize, the AddressSanitizer / UndefinedBehaviorSanitizer build."""
    out = SAN_LIB if sanitize else LIB
    if force or not os.path.exists(out):
        cmd = ["gcc", *CFLAGS, *(SAN_FLAGS if sanitize else []), "-o", out + ".tmp", SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(out + ".tmp", out)
    return out


def sanitize_env() -> dict:
    """Environment for a Python process that loads the sanitizer build: the
    gcc ASan runtime preloaded, leak checks off (the interpreter's own
    allocations are not ours), every report fatal."""
    env = dict(os.environ)
    asan = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    ubsan = subprocess.check_output(["gcc", "-print-file-name=libubsan.so"], text=True).strip()
    env["LD_PRELOAD"] = f"{asan}:{ubsan}"
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["ORC_SANITIZE"] = "1"
    return env


class _BC(C.Structure):
    _fields_ = [("kind", C.c_int), ("nbr_block", C.c_int), ("nbr_face", C.c_int),
                ("orient", C.c_int), ("prim", C.c_double * 5)]


class _Block(C.Structure):
    _fields_ = [("ni", C.c_int), ("nj", C.c_int), ("nk", C.c_int),
                ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double)), ("origin", C.c_double * 3), ("h", C.c_double * 3), ("bc", _BC * 6)]


class _Params(C.Structure):
    _fields_ = [("cfl", C.c_double), ("dt_fixed", C.c_double), ("t_end", C.c_double),
                ("limiter", C.c_int), ("eps", C.c_double), ("kappa", C.c_double),
                ("entropy_fix", C.c_double), ("qref", C.c_double * 5), ("rk", C.c_int),
                ("mu", C.c_double), ("prandtl", C.c_double)]


class _Info(C.Structure):
    _fields_ = [("steps", C.c_longlong), ("t", C.c_double), ("dt_last", C.c_double),
                ("norms", C.c_double * 5), ("norm", C.c_double), ("norm_first", C.c_double),
                ("drop", C.c_double), ("status", C.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = SAN_LIB if SANITIZE else LIB
        if not os.path.exists(path):
            build(force=True, sanitize=SANITIZE)
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, C.POINTER(_Block), C.c_double]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_set_state.argtypes = [C.c_void_p, dp]
        L.orc_get_state.argtypes = [C.c_void_p, dp]
        L.orc_residual.argtypes = [C.c_void_p, C.POINTER(_Params), dp, dp, dp]
        L.orc_run.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_longlong, C.c_double,
                              C.POINTER(_Info), dp]
        L.orc_get_info.argtypes = [C.c_void_p, C.POINTER(_Info)]
        L.orc_ghosts.argtypes = [C.c_void_p, dp]
        L.orc_spectral_min.argtypes = [C.c_void_p, dp]
        L.orc_face_flux.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_int, C.c_int, C.c_int,
                                    C.c_int, C.c_int, dp]
        L.orc_metrics_2d.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        L.orc_metrics_3d.argtypes = [C.c_void_p, C.c_int, dp, dp]
        L.orc_set_source.argtypes = [C.c_void_p, dp]
        L.orc_viscous_flux.argtypes = [C.c_void_p, C.POINTER(_Params), C.c_int, C.c_int, C.c_int,
                                       C.c_int, dp]
        L.orc_roe.argtypes = [dp, dp, dp, C.c_int, C.c_double, C.c_double, C.c_int, dp]
        L.orc_reconstruct.argtypes = [dp, C.c_int, C.c_double, C.c_double, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(p) -> _Params:
    q = list(p.qref) + [1.0] * (5 - len(p.qref))
    return _Params(p.cfl, p.dt_fixed, p.t_end, p.limiter, p.eps, p.kappa, p.entropy_fix,
                   (C.c_double * 5)(*q[:5]), getattr(p, "rk", 3), getattr(p, "mu", 0.0),
                   getattr(p, "prandtl", 0.72))


def num_threads() -> int:
    return lib().orc_num_threads()


def set_threads(n: int) -> None:
    """Threads of the following oracle runs (timing only)."""
    lib().orc_set_threads(int(n))


# ---------------------------------------------------------------------------
# point functions (used by the pins)
# ---------------------------------------------------------------------------
def roe(qL, qR, n, gamma=1.4, entropy_fix=0.1, mode=-1):
    """mode -1: Roe flux per unit area; 0: |lambda| wave sum; 1: signed wave
    sum; 2: unit-eigenvalue wave sum; 3: F(Q_L).n."""
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    nn = np.zeros(3)
    nn[:len(n)] = n
    nd = len(qL) - 2
    out = np.zeros(5)
    lib().orc_roe(_ptr(qL), _ptr(qR), _ptr(nn), nd, gamma, entropy_fix, mode, _ptr(out))
    return out[:nd + 2]


def reconstruct(q4, limiter=0, eps=1.0, kappa=-1.0):
    q4 = np.ascontiguousarray(q4, dtype=np.float64)
    a, b = np.zeros(1), np.zeros(1)
    lib().orc_reconstruct(_ptr(q4), limiter, eps, kappa, _ptr(a), _ptr(b))
    return float(a[0]), float(b[0])


# ---------------------------------------------------------------------------
# grid handle
# ---------------------------------------------------------------------------
class OracleGrid:
    def __init__(self, case):
        self.case = case
        self.ndim = case.ndim
        self.nv = case.ndim + 2
        nb = len(case.blocks)
        arr = (_Block * nb)()
        self._keep = []
        for b, blk in enumerate(case.blocks):
            d = arr[b]
            d.ni, d.nj, d.nk = blk.ni, blk.nj, blk.nk
            if blk.x is not None:
                x = np.ascontiguousarray(blk.x, dtype=np.float64)
                y = np.ascontiguousarray(blk.y, dtype=np.float64)
                self._keep += [x, y]
                d.x, d.y = _ptr(x), _ptr(y)
            if getattr(blk, "z", None) is not None:
                z = np.ascontiguousarray(blk.z, dtype=np.float64)
                self._keep.append(z)
                d.z = _ptr(z)
            for a in range(3):
                d.origin[a] = blk.origin[a]
                d.h[a] = blk.h[a]
            for f in range(6):
                bc = blk.bc[f]
                d.bc[f].kind = bc.kind
                d.bc[f].nbr_block = bc.nbr_block
                d.bc[f].nbr_face = bc.nbr_face
                d.bc[f].orient = getattr(bc, "orient", 0)
                for a in range(5):
                    d.bc[f].prim[a] = bc.prim[a]
        self._h = lib().orc_create(case.ndim, nb, arr, case.gamma)
        if not self._h:
            raise ValueError("oracle rejected the grid description")
        self.size = sum(self.nv * b.ncells for b in case.blocks)
        src = case.source_flat() if hasattr(case, "source_flat") else None
        if src is not None:
            self.set_source(src)
        self.status = self.set_state(case.state_flat())

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_destroy(h)
            self._h = None

    def set_state(self, U) -> int:
        U = np.ascontiguousarray(U, dtype=np.float64).ravel()
        assert U.size == self.size
        self.status = lib().orc_set_state(self._h, _ptr(U))
        return self.status

    def set_source(self, S) -> None:
        """Cell-averaged source S_h, [block][var][k][j][i] (None removes it)."""
        if S is None:
            lib().orc_set_source(self._h, None)
            return
        S = np.ascontiguousarray(S, dtype=np.float64).ravel()
        assert S.size == self.size
        if lib().orc_set_source(self._h, _ptr(S)) != OK:
            raise MemoryError("oracle could not store the source")

    def get_state(self) -> np.ndarray:
        out = np.empty(self.size)
        lib().orc_get_state(self._h, _ptr(out))
        return out

    def residual(self, params, with_scale=False):
        R = np.empty(self.size)
        norms = np.zeros(5)
        scale = np.empty(self.size) if with_scale else None
        P = make_params(params)
        lib().orc_residual(self._h, C.byref(P), _ptr(R), _ptr(norms),
                           _ptr(scale) if with_scale else None)
        return (R, norms, scale) if with_scale else (R, norms)

    def run(self, params, nsteps, drop_tol=0.0, dt_hist=False):
        P = make_params(params)
        info = _Info()
        hist = np.zeros(max(int(nsteps), 1)) if dt_hist else None
        st = lib().orc_run(self._h, C.byref(P), int(nsteps), float(drop_tol), C.byref(info),
                           _ptr(hist) if dt_hist else None)
        d = dict(status=st, steps=info.steps, t=info.t, dt_last=info.dt_last,
                 norms=np.array(info.norms[:]), norm=info.norm, norm_first=info.norm_first,
                 drop=info.drop)
        if dt_hist:
            d["dt_hist"] = hist[:info.steps]
        return d

    def ghosts(self) -> np.ndarray:
        n = 0
        for b in self.case.blocks:
            dims = (b.ni, b.nj, b.nk)
            for f in range(2 * self.ndim):
                d = f // 2
                t = [dims[a] for a in range(3) if a != d]
                n += 2 * self.nv * t[0] * t[1]
        out = np.empty(n)
        lib().orc_ghosts(self._h, _ptr(out))
        return out

    def spectral_min(self):
        out = np.zeros(1)
        st = lib().orc_spectral_min(self._h, _ptr(out))
        return st, float(out[0])

    def face_flux(self, params, block, d, i, j, k=0):
        out = np.zeros(5)
        P = make_params(params)
        lib().orc_face_flux(self._h, C.byref(P), block, d, i, j, k, _ptr(out))
        return out[:self.nv]

    def viscous_flux(self, params, block, d, i, j):
        """F_nu,n ds of face (d, i, j) of a block (2D) for the current state."""
        out = np.zeros(4)
        P = make_params(params)
        st = lib().orc_viscous_flux(self._h, C.byref(P), block, d, i, j, _ptr(out))
        if st != OK:
            raise ValueError("oracle rejected the viscous flux request")
        return out

    def metrics_2d(self, block):
        b = self.case.blocks[block]
        Sxi = np.empty((b.nj, b.ni + 1, 2))
        Seta = np.empty((b.nj + 1, b.ni, 2))
        vol = np.empty((b.nj, b.ni))
        lib().orc_metrics_2d(self._h, block, _ptr(Sxi), _ptr(Seta), _ptr(vol))
        return Sxi, Seta, vol

    def metrics_3d(self, block):
        """Face area vectors of the three directions and cell volumes of a 3D block."""
        b = self.case.blocks[block]
        shapes = [(b.nk, b.nj, b.ni + 1, 3), (b.nk, b.nj + 1, b.ni, 3), (b.nk + 1, b.nj, b.ni, 3)]
        n = sum(int(np.prod(s)) for s in shapes)
        S = np.empty(n)
        vol = np.empty((b.nk, b.nj, b.ni))
        lib().orc_metrics_3d(self._h, block, _ptr(S), _ptr(vol))
        out, o = [], 0
        for s in shapes:
            m = int(np.prod(s))
            out.append(S[o:o + m].reshape(s))
            o += m
        return out, vol
