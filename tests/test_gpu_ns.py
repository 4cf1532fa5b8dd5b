"""Navier-Stokes path on the GPU (through the C ABI) against the CPU
reference, element by element: the viscous normal flux of Sec. 2 added to
Eq. (residual), no-slip walls, corner ghosts, the viscous time-step term.

FP64: relative error <= 1e-12 (U metric; R on the flux scale, see parity.py).
FP32-flux: <= 1e-5 for one step from the same FP64 state, <= 1e-4 after N.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

from paper_2305_18057_amd import cases as CS
from tests import parity as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()
    P.report(os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0], msg.strip())


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2305_18057_amd import fv
    from oracle import oracle as O
    fv.lib()
    O.lib()
    return fv, O


def with_(params, **kw):
    return CS.Params(**{**params.__dict__, **kw})


def centres(X, Y):
    cx = 0.25 * (X[:-1, :-1] + X[:-1, 1:] + X[1:, :-1] + X[1:, 1:])
    cy = 0.25 * (Y[:-1, :-1] + Y[:-1, 1:] + Y[1:, :-1] + Y[1:, 1:])
    return cx, cy


def split_mesh(X, Y, icut, jcut, outer, fields, name, periodic_i=False):
    """Blocks cut from a node array at node columns icut / rows jcut and
    linked 1:1; outer = rules of the imin, imax, jmin, jmax faces of the whole
    mesh (with periodic_i, the i-ends are linked around instead); the state
    fields(cx, cy) -> (rho, u, v, p) at the cell centres."""
    Nj, Ni = X.shape[0] - 1, X.shape[1] - 1
    ib, jb = [0, *icut, Ni], [0, *jcut, Nj]
    nbi, nbj = len(ib) - 1, len(jb) - 1
    idx = lambda a, b: b * nbi + a
    blocks, U0 = [], []
    for bj in range(nbj):
        for bi in range(nbi):
            i0, i1, j0, j1 = ib[bi], ib[bi + 1], jb[bj], jb[bj + 1]
            x = np.ascontiguousarray(X[j0:j1 + 1, i0:i1 + 1])
            y = np.ascontiguousarray(Y[j0:j1 + 1, i0:i1 + 1])
            if periodic_i and nbi == 1:
                fi = [CS.BC(CS.PERIODIC), CS.BC(CS.PERIODIC)]
            elif periodic_i:
                fi = [CS.BC(CS.BLOCK, idx((bi - 1) % nbi, bj), CS.IMAX),
                      CS.BC(CS.BLOCK, idx((bi + 1) % nbi, bj), CS.IMIN)]
            else:
                fi = [outer[0] if bi == 0 else CS.BC(CS.BLOCK, idx(bi - 1, bj), CS.IMAX),
                      outer[1] if bi == nbi - 1 else CS.BC(CS.BLOCK, idx(bi + 1, bj), CS.IMIN)]
            fj = [outer[2] if bj == 0 else CS.BC(CS.BLOCK, idx(bi, bj - 1), CS.JMAX),
                  outer[3] if bj == nbj - 1 else CS.BC(CS.BLOCK, idx(bi, bj + 1), CS.JMIN)]
            bc = fi + fj + [CS.BC(CS.PERIODIC), CS.BC(CS.PERIODIC)]
            blocks.append(CS.Block(i1 - i0, j1 - j0, 1, x, y, (0, 0, 0), (1, 1, 1), bc))
            cx, cy = centres(x, y)
            rho, u, v, p = fields(cx, cy)
            U0.append(CS.conserved(rho, [u, v], p)[:, None].copy())
    return CS.Case(name, 2, blocks, U0, CS.Params(), 1)


def curved_channel(Ni=150, Nj=37, icut=(64, 97), jcut=(20,), mu=2e-3, wall_u=0.3):
    """A channel with a curved lower wall (no-slip at rest) and a moving
    upper no-slip wall, inflow and outflow at the i-ends, cut into uneven
    linked blocks (ragged against 64-column tiles and 4-row slabs); Mach
    0.8 flow with seeded perturbations; cell Reynolds number about 10, so
    the viscous flux matters everywhere."""
    I, J = np.meshgrid(np.arange(Ni + 1), np.arange(Nj + 1))
    X = 3.0 * I / Ni + 0.04 * np.sin(2 * np.pi * J / Nj + 0.4)
    Y = (J / Nj) * (1 + 0.15 * I / Ni) + 0.05 * np.sin(2 * np.pi * I / Ni) * (1 - J / Nj)
    rng = np.random.default_rng(41)
    prim = (1.0, 0.8 * math.sqrt(1.4), 0.05, 0.0, 1.0)

    def fields(cx, cy):
        rho = 1.0 + 0.05 * np.sin(4 * cx) * np.cos(5 * cy) + 0.01 * rng.uniform(-1, 1, cx.shape)
        u = prim[1] * (0.6 + 0.4 * np.sin(np.pi * cy))
        v = 0.05 * np.cos(3 * cx)
        p = 1.0 + 0.03 * np.cos(2 * cx + cy)
        return rho, u, v, p
    outer = [CS.BC(CS.INFLOW, prim=prim), CS.BC(CS.EXTRAP), CS.BC(CS.NOSLIP),
             CS.BC(CS.NOSLIP, prim=(0.0, wall_u, 0.0, 0.0, 0.0))]
    case = split_mesh(X, Y, list(icut), list(jcut), outer, fields, "curved_channel")
    case.params = CS.Params(mu=mu, prandtl=0.72, qref=(1.0, 1.0, 1.0, 2.5, 1.0))
    return case


def periodic_wavy(N=96, mu=5e-3):
    """A doubly periodic wavy mesh cut into 2 x 2 blocks linked around in
    both directions (every corner ghost is a block-link corner)."""
    I, J = np.meshgrid(np.arange(N + 1), np.arange(N + 1))
    h = 1.0 / N
    X = I * h + 0.03 * np.sin(2 * np.pi * J / N + 0.3)
    Y = J * h + 0.04 * np.sin(2 * np.pi * I / N + 0.7)

    def fields(cx, cy):
        rho = 1.0 + 0.1 * np.sin(2 * np.pi * cx) * np.cos(2 * np.pi * cy)
        u = 0.3 + 0.2 * np.cos(2 * np.pi * cy)
        v = -0.2 + 0.2 * np.sin(2 * np.pi * cx)
        p = 1.0 + 0.05 * np.cos(2 * np.pi * (cx + cy))
        return rho, u, v, p
    # j-links around: the outer j faces of the bottom and top rows link to each other
    case = split_mesh(X, Y, [50], [41], [None, None, None, None], fields, "periodic_wavy",
                      periodic_i=True)
    for b, blk in enumerate(case.blocks):
        bi, bj = b % 2, b // 2
        if bj == 0:
            blk.bc[2] = CS.BC(CS.BLOCK, 2 + bi, CS.JMAX)
        else:
            blk.bc[3] = CS.BC(CS.BLOCK, bi, CS.JMIN)
    case.params = CS.Params(mu=mu, prandtl=0.72)
    return case


def ns_inlet_full():
    """The inlet-like grid of the throughput workload with no-slip walls and
    a viscosity that makes the viscous flux a visible part of every face
    flux (cell Reynolds number about 30)."""
    return CS.inlet_2d_ns()


def check_residual(fv, O, case, params=None, tol=P.FP64_TOL):
    params = params or case.params
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Rg, ng = g.residual(params)
    ref = O.OracleGrid(case)
    Ro, no, scale = ref.residual(params, with_scale=True)
    e = P.residual_err(case, Rg, Ro, scale)
    # the viscous part is really there: R with and without mu differ
    R0, _ = ref.residual(with_(params, mu=0.0))
    dv = np.max(np.abs(Ro - R0)) / np.max(np.abs(Ro))
    say(f"  residual {case.name} mu={params.mu:g}: e_R = {e:.3e} (viscous share of R {dv:.2e})")
    assert e <= tol
    assert np.allclose(ng[:4], no[:4], rtol=1e-11, atol=0)
    return g, dv


def check_steps(fv, O, case, nsteps, params=None):
    params = params or case.params
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    info = g.step(params, nsteps)
    ref = O.OracleGrid(case)
    io = ref.run(params, nsteps)
    Uo = ref.get_state()
    e = P.state_err(case, g.get_state(), Uo)
    say(f"  {nsteps} steps {case.name} mu={params.mu:g} rk={params.rk}: e_U = {e:.3e} "
        f"(per component {P.component_errs(case, g.get_state(), Uo)}), t gpu {info['t']:.12g} "
        f"ref {io['t']:.12g}")
    assert info["steps"] == io["steps"] == nsteps
    assert e <= P.FP64_TOL
    assert abs(info["t"] - io["t"]) <= 1e-11 * abs(io["t"])
    assert abs(info["norm"] - io["norm"]) <= 1e-10 * io["norm"]
    return g, info, io, Uo


def check_fp32(fv, O, case, nsteps, Uo_n, io_n):
    """FP32-flux: one step from the same FP64 state, and nsteps against the
    oracle's FP64 run (state Uo_n, info io_n)."""
    p32 = with_(case.params, precision=CS.FP32_FLUX)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    g.step(p32, 1)
    ref = O.OracleGrid(case)
    ref.run(case.params, 1)
    e1 = P.state_err(case, g.get_state(), ref.get_state())
    g.set_state(case.state_flat())
    info = g.step(p32, nsteps)
    eN = P.state_err(case, g.get_state(), Uo_n)
    say(f"  fp32-flux {case.name}: one step {e1:.2e}, {nsteps} steps {eN:.2e}")
    assert 1e-12 < e1 <= P.FP32_STEP_TOL
    assert eN <= P.FP32_RUN_TOL
    assert abs(info["t"] - io_n["t"]) <= P.FP32_RUN_TOL * io_n["t"]


@pytest.mark.parametrize("maker", [curved_channel, periodic_wavy])
def test_ns_small_grids(env, maker):
    """Curved channel with moving and fixed no-slip walls, inflow and outflow
    (3 x 2 ragged blocks), and a doubly periodic wavy mesh linked around
    (2 x 2 blocks): ghosts, residual, 25 steps FP64, FP32-flux bars."""
    fv, O = env
    case = maker()
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Gg = g.ghosts()
    Go = O.OracleGrid(case).ghosts()
    eg = np.max(np.abs(Gg - Go)) / np.max(np.abs(Go))
    say(f"  {case.name}: ghost values e = {eg:.2e}")
    assert eg <= 1e-14
    _, dv = check_residual(fv, O, case)
    assert dv > 1e-3
    _, _, io, Uo = check_steps(fv, O, case, 25)
    check_fp32(fv, O, case, 25, Uo, io)


def test_ns_rk4_and_stage_kinds(env):
    """The 4-stage scheme runs the other stage kinds of the viscous kernel."""
    fv, O = env
    case = curved_channel(Ni=90, Nj=21, icut=(40,), jcut=(11,))
    check_steps(fv, O, case, 12, with_(case.params, rk=4))
    check_steps(fv, O, case, 12, with_(case.params, rk=2, limiter=CS.UNLIMITED))


def test_ns_inviscid_kernel_with_noslip_walls(env):
    """mu = 0 on a grid with no-slip walls: the viscous kernel's inviscid
    part and wall ghosts alone, against the oracle."""
    fv, O = env
    case = curved_channel(Ni=90, Nj=21, icut=(40,), jcut=(11,))
    prm = with_(case.params, mu=0.0)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Rg, _ = g.residual(prm)
    ref = O.OracleGrid(case)
    Ro, _, scale = ref.residual(prm, with_scale=True)
    e = P.residual_err(case, Rg, Ro, scale)
    say(f"  residual {case.name} mu=0: e_R = {e:.3e}")
    assert e <= P.FP64_TOL
    check_steps(fv, O, case, 15, prm)


def test_ns_tile_shape_independence(env, tmp_path):
    """Every tile shape gives the viscous state bit for bit."""
    fv, O = env
    case = curved_channel()
    cls = int(math.floor(math.log2(case.ncells)))
    outs = []
    for rows in (2, 3, 5, 8, 64):
        path = tmp_path / f"t{rows}.json"
        path.write_text(json.dumps({f"2d_fp64_c{cls}_ns": {"rows": rows, "ny": 1, "ms": 0.0}}))
        g = fv.Grid(case)
        g.set_state(case.state_flat())
        g.tune(case.params, str(path))
        assert g.stats()["tile_rows"] == rows
        g.step(case.params, 7)
        outs.append(g.get_state())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])
    say(f"  {case.name}: 5 tile shapes bitwise equal after 7 viscous steps")


def test_ns_inlet_full(env):
    """The full inlet-like grid (4 x 512 x 256) with no-slip walls and
    viscosity: residual and 20 steps FP64 against the oracle; FP32-flux one
    step and 20 steps at their bars."""
    fv, O = env
    case = ns_inlet_full()
    _, dv = check_residual(fv, O, case)
    assert dv > 1e-4
    _, _, io, Uo = check_steps(fv, O, case, 20)
    check_fp32(fv, O, case, 20, Uo, io)


def test_ns_solve_stop_and_noalloc(env):
    """fv_solve stops a viscous run at the oracle's step; the allocation-free
    entry point gives the viscous state of fv_step bit for bit."""
    import torch
    fv, O = env
    case = curved_channel(Ni=90, Nj=21, icut=(40,), jcut=(11,))
    ref = O.OracleGrid(case)
    io = ref.run(case.params, 60)
    tol = io["drop"] * 1.000001
    ref2 = O.OracleGrid(case)
    io2 = ref2.run(case.params, 500, drop_tol=tol)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    si = g.solve(case.params, drop_tol=tol, max_steps=500)
    e = P.state_err(case, g.get_state(), ref2.get_state())
    say(f"  {case.name} solve: gpu {si['steps']} steps, oracle {io2['steps']}; e_U = {e:.3e}")
    assert si["steps"] == io2["steps"] and e <= P.FP64_TOL
    g2 = fv.Grid(case)
    g2.set_state(case.state_flat())
    g2.step(case.params, 9)
    U = torch.from_numpy(case.state_flat()).to("cuda")
    fv.step_noalloc(case, U, case.params, 9)
    assert np.array_equal(U.cpu().numpy(), g2.get_state())
