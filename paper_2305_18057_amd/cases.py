"""Seeded synthetic inputs: meshes, initial conserved states, boundary specs.

This module holds none of the method's arithmetic.  It only lays out node
coordinates, converts prescribed primitive fields (rho, velocity, p) into the
conserved vector Q = (rho, rho*u, rho*v[, rho*w], rho*e_t) that the method
takes as input (Sec. 2, conserved vector), and names the boundary condition of
each block face.  Both the HIP path and the CPU reference consume the objects
built here; neither side's arithmetic lives here.

Workloads (all synthetic; the paper's inlet grid is not public):

* ``vortex_2d``  - 128x64 periodic uniform block, isentropic vortex of
  strength 5 in a Mach 0.5 free stream plus a seeded density perturbation.
* ``inlet_2d``   - 4 blocks of 512x256 cells on the sheared, wavy
  inlet-like mesh x = I*dx + 0.05 sin(2 pi J/Nj), y = J*dy*(1 + 0.2 I/Ni)
  (global node indices I, J), supersonic inflow with the state of the
  paper's inflow table (Sec. 8: M = 4, p = 12270 Pa, T = 217 K), slip walls
  at J = 0 and J = Nj, zeroth-order extrapolation at the outflow.
* ``blobs_3d``   - 256^3 uniform block, Mach 2 free stream carrying seeded
  Gaussian density blobs, inflow at x-min, extrapolation at x-max,
  periodic in y and z.
* ``batch_2d``   - 64 seeded inlet-like instances of uneven size, 1-4 blocks.
* ``serving_trace`` - a seeded Poisson arrival stream of mixed 2D/3D solves.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# boundary kinds (match the C ABI enumeration)
PERIODIC, BLOCK, INFLOW, EXTRAP, SLIPWALL, NOSLIP = 0, 1, 2, 3, 4, 5
# face order
IMIN, IMAX, JMIN, JMAX, KMIN, KMAX = 0, 1, 2, 3, 4, 5
# reconstruction
MINMOD, UNLIMITED, FIRST_ORDER = 0, 1, 2
# arithmetic of the reconstruction + flux
FP64, FP32_FLUX = 0, 1

GAMMA = 1.4
R_GAS = 287.0  # J/(kg K): gas constant of air, used to turn (p, T) into rho

# Inflow state of the paper's supersonic inlet (Sec. 8, inflow table).
INLET_MACH = 4.0
INLET_P = 12270.0
INLET_T = 217.0


@dataclass
class BC:
    kind: int
    nbr_block: int = -1
    nbr_face: int = -1
    prim: Sequence[float] = (0.0, 0.0, 0.0, 0.0, 0.0)  # rho, u, v, w, p (NOSLIP: wall u, v, w)
    orient: int = 0  # BLOCK, 3D: bit 0 swaps the transverse indices, bits 1, 2 reverse them


@dataclass
class Block:
    ni: int
    nj: int
    nk: int = 1
    x: Optional[np.ndarray] = None  # node coordinates: 2D (nj+1, ni+1); 3D (nk+1, nj+1, ni+1)
    y: Optional[np.ndarray] = None
    origin: Sequence[float] = (0.0, 0.0, 0.0)
    h: Sequence[float] = (1.0, 1.0, 1.0)
    bc: List[BC] = field(default_factory=list)
    z: Optional[np.ndarray] = None  # 3D curvilinear: z of the nodes, shape (nk+1, nj+1, ni+1)

    @property
    def ncells(self) -> int:
        return self.ni * self.nj * self.nk


@dataclass
class Params:
    cfl: float = 0.5
    dt_fixed: float = 0.0
    t_end: float = 0.0
    precision: int = FP64
    limiter: int = MINMOD
    eps: float = 1.0
    kappa: float = -1.0
    entropy_fix: float = 0.1
    qref: Sequence[float] = (1.0, 1.0, 1.0, 1.0, 1.0)
    rk: int = 3  # 3: SSP-RK3; 2, 4: the 2- and 4-stage second-order schemes
    mu: float = 0.0        # dynamic viscosity (0: Euler)
    prandtl: float = 0.72  # Prandtl number of the heat flux


@dataclass
class Case:
    name: str
    ndim: int
    blocks: List[Block]
    U0: List[np.ndarray]  # per block, float64 (nv, nk, nj, ni)
    params: Params
    nsteps: int = 1
    gamma: float = GAMMA
    meta: dict = field(default_factory=dict)
    # cell-averaged source S_h per block, (nv, nk, nj, ni), or None
    source: Optional[List[np.ndarray]] = None

    @property
    def nv(self) -> int:
        return self.ndim + 2

    @property
    def ncells(self) -> int:
        return sum(b.ncells for b in self.blocks)

    def state_flat(self) -> np.ndarray:
        """Interior state, layout [block][var][k][j][i], float64."""
        return np.concatenate([np.ascontiguousarray(u, dtype=np.float64).ravel() for u in self.U0])

    def source_flat(self) -> Optional[np.ndarray]:
        """Source S_h in the state's layout, float64, or None."""
        if self.source is None:
            return None
        return np.concatenate([np.ascontiguousarray(s, dtype=np.float64).ravel() for s in self.source])

    def split_flat(self, flat: np.ndarray) -> List[np.ndarray]:
        out, o = [], 0
        for b in self.blocks:
            n = self.nv * b.ncells
            out.append(np.asarray(flat[o:o + n]).reshape(self.nv, b.nk, b.nj, b.ni))
            o += n
        return out


# --------------------------------------------------------------------------
# primitive -> conserved (input construction only)
# --------------------------------------------------------------------------
def conserved(rho, vel, p, gamma=GAMMA):
    """Stack Q = (rho, rho*u_a..., rho*e_t) with rho*e_t = p/(g-1) + rho|u|^2/2."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = [np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape) for v in vel]
    ke = sum(v * v for v in vel)
    out = [rho] + [rho * v for v in vel] + [np.asarray(p, dtype=np.float64) / (gamma - 1.0) + 0.5 * rho * ke]
    return np.stack([np.broadcast_to(a, rho.shape) for a in out]).astype(np.float64)


def inlet_freestream(mach=INLET_MACH, angle_deg=0.0, ndim=2):
    """(rho, u, v, w, p) of the inlet inflow table at a given Mach number."""
    rho = INLET_P / (R_GAS * INLET_T)
    c = math.sqrt(GAMMA * INLET_P / rho)
    a = math.radians(angle_deg)
    return (rho, mach * c * math.cos(a), mach * c * math.sin(a), 0.0, INLET_P)


def qref_of(prim, ndim):
    rho, u, v, w, p = prim
    speed = math.sqrt(u * u + v * v + w * w)
    rhoE = p / (GAMMA - 1.0) + 0.5 * rho * speed * speed
    q = [rho] + [rho * speed] * ndim + [rhoE]
    q += [1.0] * (5 - len(q))
    return tuple(q)


def _round8(v, lo):
    return max(lo, int(round(v / 8.0)) * 8)


def _split_even(n, nb, quantum=8):
    """Split n cells into nb chunks that are multiples of ``quantum`` when possible."""
    q = n // quantum
    nb = max(1, min(nb, q if q > 0 else 1))
    if q == 0:
        return [n]
    sizes = [(q // nb + (1 if b < q % nb else 0)) * quantum for b in range(nb)]
    sizes[-1] += n - sum(sizes)
    return sizes


# --------------------------------------------------------------------------
# workload 1: isentropic vortex on a periodic uniform block
# --------------------------------------------------------------------------
def vortex_fields(xc, yc, x, y, beta=5.0, uinf=0.5 * math.sqrt(GAMMA), vinf=0.0, gamma=GAMMA):
    """Primitive fields of the translating isentropic vortex (rho_inf = p_inf = 1)."""
    dx, dy = x - xc, y - yc
    r2 = dx * dx + dy * dy
    e = np.exp(0.5 * (1.0 - r2))
    u = uinf - beta / (2.0 * math.pi) * e * dy
    v = vinf + beta / (2.0 * math.pi) * e * dx
    T = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * e * e
    rho = T ** (1.0 / (gamma - 1.0))
    p = rho ** gamma
    return rho, u, v, p


def vortex_2d(ni=128, nj=64, seed=1, noise=1e-3, Lx=20.0, Ly=10.0, beta=5.0,
              limiter=MINMOD, nsteps=100, cfl=0.5):
    h = (Lx / ni, Ly / nj, 1.0)
    xc = (np.arange(ni) + 0.5) * h[0]
    yc = (np.arange(nj) + 0.5) * h[1]
    X, Y = np.meshgrid(xc, yc)  # (nj, ni)
    rho, u, v, p = vortex_fields(0.5 * Lx, 0.5 * Ly, X, Y, beta=beta)
    if noise > 0:
        rng = np.random.default_rng(seed)
        rho = rho + rng.uniform(-noise, noise, size=rho.shape)
    U = conserved(rho, [u, v], p)[:, None, :, :]
    bcs = [BC(PERIODIC) for _ in range(4)] + [BC(PERIODIC), BC(PERIODIC)]
    blk = Block(ni, nj, 1, None, None, (0.0, 0.0, 0.0), h, bcs)
    uinf = 0.5 * math.sqrt(GAMMA)
    qref = qref_of((1.0, uinf, 0.0, 0.0, 1.0), 2)
    prm = Params(cfl=cfl, limiter=limiter, qref=qref)
    return Case("vortex_2d", 2, [blk], [U], prm, nsteps,
                meta=dict(Lx=Lx, Ly=Ly, beta=beta, uinf=uinf, seed=seed))


# --------------------------------------------------------------------------
# workload 2: inlet-like multi-block curvilinear mesh
# --------------------------------------------------------------------------
def inlet_mesh(Ni, Nj, Lx=4.0, Ly=1.0, wave=0.05, shear=0.2):
    """Global node coordinates (Nj+1, Ni+1) of the sheared wavy inlet-like mesh."""
    I = np.arange(Ni + 1, dtype=np.float64)[None, :]
    J = np.arange(Nj + 1, dtype=np.float64)[:, None]
    dx, dy = Lx / Ni, Ly / Nj
    x = I * dx + wave * np.sin(2.0 * math.pi * J / Nj)
    y = J * dy * (1.0 + shear * I / Ni)
    return np.ascontiguousarray(x), np.ascontiguousarray(y)


def inlet_case(Ni, Nj, nblocks, mach=INLET_MACH, angle_deg=0.0, name="inlet_2d",
               nsteps=500, precision=FP64, cfl=0.5):
    X, Y = inlet_mesh(Ni, Nj)
    prim = inlet_freestream(mach, angle_deg)
    sizes = _split_even(Ni, nblocks)
    nb = len(sizes)
    blocks, U0 = [], []
    i0 = 0
    for b, n in enumerate(sizes):
        bcs = [BC(BLOCK, b - 1, IMAX) if b > 0 else BC(INFLOW, prim=prim),
               BC(BLOCK, b + 1, IMIN) if b < nb - 1 else BC(EXTRAP),
               BC(SLIPWALL), BC(SLIPWALL), BC(PERIODIC), BC(PERIODIC)]
        x = np.ascontiguousarray(X[:, i0:i0 + n + 1])
        y = np.ascontiguousarray(Y[:, i0:i0 + n + 1])
        blocks.append(Block(n, Nj, 1, x, y, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), bcs))
        U = conserved(np.full((Nj, n), prim[0]), [np.full((Nj, n), prim[1]), np.full((Nj, n), prim[2])],
                      np.full((Nj, n), prim[4]))
        U0.append(U[:, None, :, :].copy())
        i0 += n
    prm = Params(cfl=cfl, precision=precision, qref=qref_of(prim, 2))
    return Case(name, 2, blocks, U0, prm, nsteps,
                meta=dict(Ni=Ni, Nj=Nj, mach=mach, angle=angle_deg, prim=prim))


def inlet_2d(nblocks=4, ni=512, nj=256, precision=FP64, nsteps=500):
    return inlet_case(nblocks * ni, nj, nblocks, name="inlet_2d", nsteps=nsteps, precision=precision)


# --------------------------------------------------------------------------
# workload 3: 3D uniform block with seeded density blobs
# --------------------------------------------------------------------------
def inlet_2d_ns(mu=1.5e-2, prandtl=0.72, precision=FP64, nsteps=500):
    """The inlet-like grid (4 x 512 x 256 cells, Mach 4 inflow of the paper's
    inflow table) with no-slip walls at rest at j-min and j-max and a
    viscosity in the grid's units (metres, SI state): mu = 1.5e-2 Pa s gives
    a cell Reynolds number of about 30 at the inflow."""
    case = inlet_2d(precision=precision, nsteps=nsteps)
    for blk in case.blocks:
        blk.bc[2] = BC(NOSLIP)
        blk.bc[3] = BC(NOSLIP)
    case.name = "inlet_2d_ns"
    case.params = Params(**{**case.params.__dict__, "mu": mu, "prandtl": prandtl})
    return case


def blobs_fields(n, centres, amp=0.05, width_cells=8.0, rho_inf=1.0, chunk=16):
    """rho(k, j, i) = rho_inf (1 + amp sum_b exp(-|x - x_b|^2 / (2 w^2))).

    Distances use the minimum image in y and z (periodic directions).
    """
    h = 1.0 / n
    w = width_cells * h
    c = (np.arange(n) + 0.5) * h
    rho = np.zeros((n, n, n), dtype=np.float64)
    for (bx, by, bz) in centres:
        dx = (c - bx)[None, None, :]
        dy = c - by
        dy = (dy - np.round(dy))[None, :, None]
        dz = c - bz
        dz = (dz - np.round(dz))[:, None, None]
        ex = np.exp(-(dx * dx) / (2 * w * w))
        ey = np.exp(-(dy * dy) / (2 * w * w))
        ez = np.exp(-(dz * dz) / (2 * w * w))
        rho += ez * ey * ex
    return rho_inf * (1.0 + amp * rho)


def blobs_case(n, nblobs=16, seed=3, mach=2.0, name="blobs_3d", nsteps=50, precision=FP64,
               cfl=0.5, amp=0.05, width_cells=8.0):
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, 1.0, size=(nblobs, 3))
    prim = inlet_freestream(mach, 0.0)
    rho = blobs_fields(n, centres, amp, width_cells, prim[0])
    U = conserved(rho, [np.full_like(rho, prim[1]), 0.0, 0.0], np.full_like(rho, prim[4]))
    h = 1.0 / n
    bcs = [BC(INFLOW, prim=prim), BC(EXTRAP), BC(PERIODIC), BC(PERIODIC), BC(PERIODIC), BC(PERIODIC)]
    blk = Block(n, n, n, None, None, (0.0, 0.0, 0.0), (h, h, h), bcs)
    prm = Params(cfl=cfl, precision=precision, qref=qref_of(prim, 3))
    return Case(name, 3, [blk], [U], prm, nsteps,
                meta=dict(n=n, seed=seed, mach=mach, prim=prim, centres=centres))


def blobs_3d(n=256, precision=FP64, nsteps=50):
    return blobs_case(n, 16, 3, 2.0, "blobs_3d", nsteps, precision)


# --------------------------------------------------------------------------
# workload 4: batch of uneven inlet-like instances
# --------------------------------------------------------------------------
def batch_2d(count=64, seed=4, precision=FP32_FLUX, nsteps=100):
    rng = np.random.default_rng(seed)
    out = []
    for r in range(count):
        Ni = _round8(math.exp(rng.uniform(math.log(64), math.log(1024))), 64)
        Nj = _round8(math.exp(rng.uniform(math.log(64), math.log(512))), 64)
        mach = rng.uniform(1.5, 4.0)
        nb = int(rng.integers(1, 5))
        out.append(inlet_case(Ni, Nj, nb, mach=mach, name=f"batch_{r}", nsteps=nsteps, precision=precision))
    return out


# --------------------------------------------------------------------------
# workload 5: Poisson arrival stream of mixed 2D / 3D solves
# --------------------------------------------------------------------------
@dataclass
class Request:
    arrival: float  # seconds after the stream starts
    kind: str       # "2d" or "3d"
    spec: dict      # arguments that build the case (see ``build_request``)


def serving_trace(count=256, seed=5, rate=200.0, max_steps=2000, drop_tol=1e-8):
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for r in range(count):
        t += rng.exponential(1.0 / rate)
        if rng.uniform() < 0.5:
            Ni = _round8(math.exp(rng.uniform(math.log(64), math.log(2048))), 64)
            Nj = _round8(math.exp(rng.uniform(math.log(64), math.log(1024))), 64)
            spec = dict(Ni=Ni, Nj=Nj, mach=float(rng.uniform(1.5, 4.0)),
                        angle=float(rng.uniform(0.0, 10.0)), nblocks=int(rng.integers(1, 5)))
            kind = "2d"
        else:
            n = _round8(math.exp(rng.uniform(math.log(32), math.log(192))), 32)
            spec = dict(n=n, mach=float(rng.uniform(1.5, 4.0)), seed=int(rng.integers(0, 2**31 - 1)))
            kind = "3d"
        spec.update(max_steps=max_steps, drop_tol=drop_tol)
        reqs.append(Request(t, kind, spec))
    return reqs


def build_request(req: Request, precision=FP32_FLUX) -> Case:
    s = req.spec
    if req.kind == "2d":
        return inlet_case(s["Ni"], s["Nj"], s["nblocks"], mach=s["mach"], angle_deg=s["angle"],
                          name="req2d", nsteps=s["max_steps"], precision=precision)
    return blobs_case(s["n"], nblobs=8, seed=s["seed"], mach=s["mach"], name="req3d",
                      nsteps=s["max_steps"], precision=precision)


# --------------------------------------------------------------------------
# small cases used by the correctness pins
# --------------------------------------------------------------------------
def uniform_2d(ni, nj, prim, bcs, h=(1.0, 1.0, 1.0), x=None, y=None, name="uniform_2d"):
    U = conserved(np.full((nj, ni), prim[0]), [np.full((nj, ni), prim[1]), np.full((nj, ni), prim[2])],
                  np.full((nj, ni), prim[4]))[:, None]
    blk = Block(ni, nj, 1, x, y, (0.0, 0.0, 0.0), h, bcs)
    return Case(name, 2, [blk], [U.copy()], Params(qref=qref_of(prim, 2)), 1)


def sod_2d(n=400, nj=4, x0=0.5, t_end=0.2, limiter=MINMOD, cfl=0.5, transpose=False):
    """Sod shock tube along x (or along y when ``transpose``), slip walls on the sides."""
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    rho1 = np.where(xc < x0, 1.0, 0.125)
    p1 = np.where(xc < x0, 1.0, 0.1)
    if not transpose:
        rho = np.tile(rho1, (nj, 1))
        p = np.tile(p1, (nj, 1))
        U = conserved(rho, [np.zeros_like(rho), np.zeros_like(rho)], p)[:, None]
        bcs = [BC(EXTRAP), BC(EXTRAP), BC(SLIPWALL), BC(SLIPWALL), BC(PERIODIC), BC(PERIODIC)]
        blk = Block(n, nj, 1, None, None, (0.0, 0.0, 0.0), (h, h, 1.0), bcs)
    else:
        rho = np.tile(rho1[:, None], (1, nj))
        p = np.tile(p1[:, None], (1, nj))
        U = conserved(rho, [np.zeros_like(rho), np.zeros_like(rho)], p)[:, None]
        bcs = [BC(SLIPWALL), BC(SLIPWALL), BC(EXTRAP), BC(EXTRAP), BC(PERIODIC), BC(PERIODIC)]
        blk = Block(nj, n, 1, None, None, (0.0, 0.0, 0.0), (h, h, 1.0), bcs)
    prm = Params(cfl=cfl, t_end=t_end, limiter=limiter, qref=(1.0, 1.0, 1.0, 2.5, 1.0))
    return Case("sod", 2, [blk], [U.copy()], prm, 10 ** 6, meta=dict(x0=x0, t_end=t_end))


# --------------------------------------------------------------------------
# 3D curvilinear multi-block grids and manufactured solutions
# --------------------------------------------------------------------------
def curv3d_nodes(ni, nj, nk, L=(1.0, 1.0, 1.0), amp=0.04, walls_k=False):
    """Nodes (x, y, z), each of shape (nk+1, nj+1, ni+1), of a box of sides L
    deformed by smooth displacements of relative size ``amp``:
        x = X + amp Lx sin(2 pi Y/Ly) sin(2 pi Z/Lz)
        y = Y + amp Ly sin(2 pi Z/Lz) sin(2 pi X/Lx)
        z = Z + amp Lz sin(2 pi X/Lx) sin(2 pi Y/Ly) s(Z)
    with s = 1, or s = sin(pi Z/Lz) when ``walls_k`` (then the k-min and
    k-max planes stay flat and undeformed).  The displacement is periodic
    in every direction, so opposite faces of the box are translates of each
    other and the grid can be periodic; the cells are not parallelepipeds
    and their faces are not planar."""
    Lx, Ly, Lz = L
    X = np.linspace(0.0, Lx, ni + 1)[None, None, :]
    Y = np.linspace(0.0, Ly, nj + 1)[None, :, None]
    Z = np.linspace(0.0, Lz, nk + 1)[:, None, None]
    tp = 2.0 * math.pi
    sz = np.sin(math.pi * Z / Lz) if walls_k else 1.0
    x = X + amp * Lx * np.sin(tp * Y / Ly) * np.sin(tp * Z / Lz)
    y = Y + amp * Ly * np.sin(tp * Z / Lz) * np.sin(tp * X / Lx)
    z = Z + amp * Lz * np.sin(tp * X / Lx) * np.sin(tp * Y / Ly) * sz
    shape = (nk + 1, nj + 1, ni + 1)
    return [np.ascontiguousarray(np.broadcast_to(a, shape), dtype=np.float64) for a in (x, y, z)]


def cell_centres_3d(x, y, z):
    """Mean of the eight nodes of each cell, each of shape (nk, nj, ni)."""
    def c(a):
        return 0.125 * (a[:-1, :-1, :-1] + a[:-1, :-1, 1:] + a[:-1, 1:, :-1] + a[:-1, 1:, 1:]
                        + a[1:, :-1, :-1] + a[1:, :-1, 1:] + a[1:, 1:, :-1] + a[1:, 1:, 1:])
    return c(x), c(y), c(z)


def mms_primitives(x, y, z, L=(1.0, 1.0, 1.0)):
    """A smooth manufactured state, periodic on the box L: (rho, u, v, w, p).
    Works on complex arguments (the source below differentiates it by the
    complex step)."""
    tp = 2.0 * np.pi
    a, b, c = tp * x / L[0], tp * y / L[1], tp * z / L[2]
    rho = 1.0 + 0.15 * np.sin(a + 0.3) * np.cos(b) + 0.1 * np.cos(c + 0.7)
    u = 0.7 + 0.12 * np.cos(a) * np.sin(c + 0.2)
    v = 0.35 + 0.1 * np.sin(b + 0.5) * np.cos(a + 0.1)
    w = -0.25 + 0.08 * np.cos(c) * np.sin(b + 0.9)
    p = 1.0 / GAMMA + 0.12 * np.cos(a + b) + 0.05 * np.sin(c + 0.4)
    return rho, u, v, w, p


def _mms_physical_flux(prim, a, gamma):
    """Component a (0, 1, 2) of the Cartesian Euler flux (Sec. 2) of the
    manufactured state: the analytic input of the source below."""
    rho, u, v, w, p = prim
    vel = (u, v, w)
    ua = vel[a]
    et = p / ((gamma - 1.0) * rho) + 0.5 * (u * u + v * v + w * w)
    out = [rho * ua]
    for b in range(3):
        out.append(rho * vel[b] * ua + (p if a == b else 0.0))
    out.append((rho * et + p) * ua)
    return out


def mms_source(x, y, z, L=(1.0, 1.0, 1.0), gamma=GAMMA, h=1e-30, chunk=8):
    """S = div F(U_m) of the manufactured state (the steady Euler equations
    with S on the right-hand side hold for U_m), by the complex-step
    derivative of each flux component: exact to rounding.  Shape (5, ...);
    evaluated in slabs of ``chunk`` entries of the first axis."""
    x, y, z = (np.asarray(t, dtype=np.float64) for t in (x, y, z))
    out = np.empty((5,) + x.shape)
    n0 = x.shape[0] if x.ndim else 1
    for a0 in range(0, n0, chunk):
        sl = slice(a0, a0 + chunk) if x.ndim else slice(None)
        pts = [t[sl].astype(np.complex128) for t in (x, y, z)]
        S = None
        for a in range(3):
            q = list(pts)
            q[a] = q[a] + 1j * h
            F = _mms_physical_flux(mms_primitives(*q, L=L), a, gamma)
            d = np.stack([np.imag(f) / h for f in F])
            S = d if S is None else S + d
        out[(slice(None),) + (sl,)] = S
    return out


def curv3d_case(ni=24, nj=16, nk=16, nblocks=2, amp=0.04, state="random", seed=6,
                walls_k=False, precision=FP64, nsteps=5, L=(1.0, 1.0, 1.0), cfl=0.5):
    """A 3D curvilinear multi-block grid: the deformed box above, split along
    i into ``nblocks`` blocks linked face to face; periodic in i and j, and in
    k unless ``walls_k`` (slip walls).  ``state``: "uniform" (a free stream),
    "random" (a smooth field plus seeded noise) or "mms" (the manufactured
    state, with its source S_h at the cell centres)."""
    x, y, z = curv3d_nodes(ni, nj, nk, L, amp, walls_k)
    xc, yc, zc = cell_centres_3d(x, y, z)
    prim_inf = (1.0, 0.6, 0.3, 0.0, 1.0 / GAMMA)
    if state == "uniform":
        rho = np.full(xc.shape, prim_inf[0])
        vel = [np.full(xc.shape, prim_inf[1]), np.full(xc.shape, prim_inf[2]), np.zeros(xc.shape)]
        p = np.full(xc.shape, prim_inf[4])
    elif state == "mms":
        rho, u, v, w, p = mms_primitives(xc, yc, zc, L)
        vel = [u, v, w]
    elif state == "random":
        rng = np.random.default_rng(seed)
        rho, u, v, w, p = mms_primitives(xc, yc, zc, L)
        rho = rho * (1.0 + 0.02 * rng.standard_normal(xc.shape))
        p = p * (1.0 + 0.02 * rng.standard_normal(xc.shape))
        vel = [u + 0.02 * rng.standard_normal(xc.shape), v, w]
    else:
        raise ValueError(state)
    U = conserved(rho, vel, p)
    S = mms_source(xc, yc, zc, L) if state == "mms" else None
    cuts = np.cumsum([0] + _split_even(ni, nblocks))
    nb = len(cuts) - 1
    blocks, U0, src = [], [], []
    kbc = BC(SLIPWALL) if walls_k else BC(PERIODIC)
    for b in range(nb):
        i0, i1 = int(cuts[b]), int(cuts[b + 1])
        lo = BC(BLOCK, b - 1, 1) if b > 0 else (BC(BLOCK, nb - 1, 1) if nb > 1 else BC(PERIODIC))
        hi = BC(BLOCK, b + 1, 0) if b < nb - 1 else (BC(BLOCK, 0, 0) if nb > 1 else BC(PERIODIC))
        bcs = [lo, hi, BC(PERIODIC), BC(PERIODIC), kbc, kbc]
        sl = (slice(None), slice(None), slice(i0, i1 + 1))
        blocks.append(Block(i1 - i0, nj, nk, x[sl].copy(), y[sl].copy(), (0.0, 0.0, 0.0),
                            (1.0, 1.0, 1.0), bcs, z[sl].copy()))
        U0.append(np.ascontiguousarray(U[:, :, :, i0:i1]))
        if S is not None:
            src.append(np.ascontiguousarray(S[:, :, :, i0:i1]))
    prm = Params(cfl=cfl, precision=precision, qref=qref_of(prim_inf, 3))
    return Case(f"curv3d_{state}", 3, blocks, U0, prm, nsteps,
                meta=dict(amp=amp, L=L, seed=seed, walls_k=walls_k),
                source=src if S is not None else None)


def curv3d_mms(n=256, precision=FP64, nsteps=20):
    """The manufactured-solution workload on the deformed periodic box:
    n^3 cells in two blocks linked around in i, the manufactured state and its
    source S_h at the cell centres."""
    c = curv3d_case(ni=n, nj=n, nk=n, nblocks=2, amp=0.04, state="mms", precision=precision,
                    nsteps=nsteps)
    c.name = "curv3d_mms"
    return c


# --------------------------------------------------------------------------
# 3D blocks in rotated index frames, linked face to face with orientations
# --------------------------------------------------------------------------
# Index frames of pieces: local axis m runs along global axis a_m, forwards
# (s = +1) or backwards (s = -1), frame = ((a0, s0), (a1, s1), (a2, s2)).
# "swapped" exchanges transverse axes (links of orientation 0 and 1);
# "reversed" also reverses them (orientations 3, 5 and 7, each reversal bit
# alone on some link).
ROTATED_FRAMES = {
    "swapped": [((0, 1), (1, 1), (2, 1)), ((1, 1), (0, -1), (2, 1)), ((2, 1), (0, 1), (1, 1))],
    "reversed": [((0, 1), (1, -1), (2, -1)), ((1, -1), (0, -1), (2, -1)),
                 ((2, 1), (1, -1), (0, 1)), ((0, -1), (1, 1), (2, -1))],
}


def twisted_box_3d(n=24, nblobs=4, seed=5):
    """A uniform n^3 box of density blobs whose opposite faces are joined to
    each other with a twist: the i-faces with their transverse indices
    swapped and both reversed (orientation 7), the j-faces with i reversed
    (2), the k-faces with j reversed (4).  Each map is its own inverse, so
    the two sides of every link agree."""
    c = blobs_case(n, nblobs=nblobs, seed=seed, name="twisted_box")
    b = c.blocks[0]
    b.bc = [BC(BLOCK, 0, 1, orient=7), BC(BLOCK, 0, 0, orient=7),
            BC(BLOCK, 0, 3, orient=2), BC(BLOCK, 0, 2, orient=2),
            BC(BLOCK, 0, 5, orient=4), BC(BLOCK, 0, 4, orient=4)]
    return c


def reindex_3d(case, cuts, frames, name="reindexed"):
    """Split a one-block 3D curvilinear case along i at the global columns
    `cuts` and give each piece the index frame `frames[p]` (a right-handed
    signed permutation, see ROTATED_FRAMES).  Faces inside the box become
    block links with the orientation that maps each side's transverse
    indices onto the other's; the box's own faces keep their rules (periodic
    faces stay within a piece and must not be cut).  Returns the new case
    and, per piece, the map from its state layout to the single block's
    (index arrays)."""
    B0 = case.blocks[0]
    ni, nj, nk = B0.ni, B0.nj, B0.nk
    for fr in frames:
        M = np.zeros((3, 3))
        for m, (a, sg) in enumerate(fr):
            M[a, m] = sg
        if round(np.linalg.det(M)) != 1:
            raise ValueError(f"frame {fr} is not right-handed")
    edges = [0, *cuts, ni]
    pieces = []
    for p in range(len(edges) - 1):
        i0, i1 = edges[p], edges[p + 1]
        ext = (i1 - i0, nj, nk)
        loc_ext = [ext[a] for a, _ in frames[p]]
        pieces.append(dict(i0=i0, ext=ext, loc=loc_ext, frame=frames[p]))
    # the face of a piece (local face index) that lies on a global face
    def local_face(piece, gaxis, gside):
        for m, (a, sg) in enumerate(piece["frame"]):
            if a == gaxis:
                return 2 * m + (gside if sg > 0 else 1 - gside)
        raise AssertionError

    def to_local(P, g):  # global cell -> local cell of piece P
        off = [g[0] - P["i0"], g[1], g[2]]
        loc = [0, 0, 0]
        for m, (a, sg) in enumerate(P["frame"]):
            loc[m] = off[a] if sg > 0 else P["ext"][a] - 1 - off[a]
        return loc

    def trans_axes(m):
        return [x for x in range(3) if x != m]
    blocks, U0, maps = [], [], []
    X, Y, Z, U = B0.x, B0.y, B0.z, case.U0[0]
    for p, P in enumerate(pieces):
        li, lj, lk = P["loc"]
        kk, jj, ii = np.meshgrid(np.arange(lk), np.arange(lj), np.arange(li), indexing="ij")
        gi = np.empty_like(ii); gj = np.empty_like(ii); gk = np.empty_like(ii)
        for m, (a, sg) in enumerate(P["frame"]):
            lm = (ii, jj, kk)[m]
            g = lm if sg > 0 else P["ext"][a] - 1 - lm
            (gi, gj, gk)[a][...] = g
        gi = gi + P["i0"]
        maps.append((gk, gj, gi))
        U0.append(np.ascontiguousarray(U[:, gk, gj, gi]))
        nk_, nj_, ni_ = np.meshgrid(np.arange(lk + 1), np.arange(lj + 1), np.arange(li + 1), indexing="ij")
        gn = [None, None, None]
        for m, (a, sg) in enumerate(P["frame"]):
            lm = (ni_, nj_, nk_)[m]
            gn[a] = lm if sg > 0 else P["ext"][a] - lm
        gn[0] = gn[0] + P["i0"]
        xs = [np.ascontiguousarray(A[gn[2], gn[1], gn[0]]) for A in (X, Y, Z)]
        bcs = [None] * 6
        for gaxis in range(3):
            for gside in range(2):
                f = local_face(P, gaxis, gside)
                rule = B0.bc[2 * gaxis + gside]
                if gaxis == 0 and ((gside == 0 and P["i0"] > 0) or
                                   (gside == 1 and P["i0"] + P["ext"][0] < ni)):
                    q = p - 1 if gside == 0 else p + 1
                    Q = pieces[q]
                    fq = local_face(Q, 0, 1 - gside)
                    # orientation: brute force over the 8 codes
                    m0 = f // 2
                    ta = trans_axes(m0)
                    mq = fq // 2
                    tq = trans_axes(mq)
                    nq = [Q["loc"][x] for x in tq]
                    found = None
                    for o in range(8):
                        ok = True
                        for t1 in (0, P["loc"][ta[0]] - 1):
                            for t2 in (0, P["loc"][ta[1]] - 1):
                                # the ghost layer-1 cell beyond face f at (t1, t2)
                                loc = [0, 0, 0]
                                loc[m0] = -1 if f % 2 == 0 else P["loc"][m0]
                                loc[ta[0]], loc[ta[1]] = t1, t2
                                off = [0, 0, 0]
                                for m, (a, sg) in enumerate(P["frame"]):
                                    off[a] = loc[m] if sg > 0 else P["ext"][a] - 1 - loc[m]
                                g = [off[0] + P["i0"], off[1], off[2]]
                                want = to_local(Q, g)
                                s1, s2 = (t2, t1) if o & 1 else (t1, t2)
                                if o & 2: s1 = nq[0] - 1 - s1
                                if o & 4: s2 = nq[1] - 1 - s2
                                got = [0, 0, 0]
                                got[mq] = 0 if fq % 2 == 0 else Q["loc"][mq] - 1
                                got[tq[0]], got[tq[1]] = s1, s2
                                ok = ok and got == want
                        if ok:
                            found = o
                            break
                    assert found is not None
                    bcs[f] = BC(BLOCK, q, fq, orient=found)
                else:
                    bcs[f] = BC(rule.kind, rule.nbr_block, rule.nbr_face, tuple(rule.prim))
        blocks.append(Block(li, lj, lk, xs[0], xs[1], (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), bcs, xs[2]))
    src = None
    if case.source is not None:
        src = [np.ascontiguousarray(case.source[0][:, gk, gj, gi]) for (gk, gj, gi) in maps]
    out = Case(name, 3, blocks, U0, Params(**case.params.__dict__), case.nsteps,
               gamma=case.gamma, meta=dict(case.meta), source=src)
    return out, maps
