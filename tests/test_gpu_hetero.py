"""CPU-GPU heterogeneous stepping (the synchronous workflow of Sec. 4 with the
1D decomposition of Sec. 6) on the GPU machine, through the C ABI, against the
CPU reference run on the whole block: the GPU part and the host workers
together must reproduce the single-domain solution (FP64 <= 1e-12 relative,
the bar of Sec. 8 for its CPU and GPU solutions), for cuts next to either
end and in the middle, with 1 to several host workers, the three RK
schemes and a t_end landing; FP32-flux on the GPU part within its bars.
The Navier-Stokes solver (Sec. 8 runs it in this mode too) on curved and
uniform blocks with no-slip walls, moving and at rest, at every side the
host part touches.
"""
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


def channel(ni=150, nj=42, seed=31):
    """A uniform block: supersonic inflow at i-min, extrapolation at i-max,
    periodic in j, a seeded smooth state with noise (every face active)."""
    rng = np.random.default_rng(seed)
    h = 1.0 / nj
    xc = (np.arange(ni) + 0.5) * h
    yc = (np.arange(nj) + 0.5) * h
    X, Y = np.meshgrid(xc, yc)
    rho = 1.0 + 0.2 * np.sin(3 * X) * np.cos(2 * np.pi * Y) + 0.02 * rng.uniform(-1, 1, X.shape)
    u = 1.8 + 0.2 * np.cos(2 * np.pi * Y)
    v = 0.1 * np.sin(2 * X)
    p = 0.7 + 0.1 * np.cos(2 * X + 2 * np.pi * Y)
    U = CS.conserved(rho, [u, v], p)[:, None]
    prim = (1.0, 1.9, 0.0, 0.0, 0.7)
    bcs = [CS.BC(CS.INFLOW, prim=prim), CS.BC(CS.EXTRAP), CS.BC(CS.PERIODIC), CS.BC(CS.PERIODIC),
           CS.BC(CS.PERIODIC), CS.BC(CS.PERIODIC)]
    blk = CS.Block(ni, nj, 1, None, None, (0.0, 0.0, 0.0), (h, h, 1.0), bcs)
    return CS.Case("channel", 2, [blk], [U.copy()], CS.Params(qref=(1.0, 1.8, 1.0, 3.0, 1.0)), 1)


def inlet_block(Ni=300, Nj=60, seed=32):
    """The inlet-like curvilinear mesh as one block (curved slip walls in j,
    inflow and extrapolation in i) with seeded noise on the free stream."""
    c = CS.inlet_case(Ni, Nj, 1, name="inlet_block")
    rng = np.random.default_rng(seed)
    U = c.U0[0]
    U *= 1.0 + 0.01 * rng.uniform(-1, 1, U.shape)
    return c


def hetero_run(fv, case, split, workers, nsteps, params=None):
    h = fv.Hetero(case, split, workers)
    h.set_state(case.state_flat())
    info = h.step(params or case.params, nsteps)
    return h, info


def check(fv, O, case, split, workers, nsteps, params=None, tol=P.FP64_TOL):
    params = params or case.params
    h, info = hetero_run(fv, case, split, workers, nsteps, params)
    Ug = h.get_state()
    ref = O.OracleGrid(case)
    io = ref.run(with_(params, precision=CS.FP64), nsteps)
    Uo = ref.get_state()
    e = P.state_err(case, Ug, Uo)
    tm = info["times_ms"]
    say(f"  {case.name} split {split}/{case.blocks[0].ni} workers {workers} rk {params.rk} "
        f"prec {params.precision}: {nsteps} steps e_U = {e:.3e}, t {info['t']:.12g} ref "
        f"{io['t']:.12g}, norm {info['norm']:.9g} ref {io['norm']:.9g}; ms gpu {tm[0]:.2f} "
        f"host {tm[1]:.2f} exchange {tm[2]:.2f} total {tm[3]:.2f}")
    assert info["steps"] == io["steps"] == nsteps
    assert e <= tol
    if tol <= P.FP64_TOL:
        assert abs(info["t"] - io["t"]) <= 1e-11 * abs(io["t"])
        assert abs(info["norm"] - io["norm"]) <= 1e-10 * io["norm"]
        assert abs(info["drop"] - io["drop"]) <= 1e-10
        assert np.allclose(info["norms"][:4], io["norms"][:4], rtol=1e-10, atol=0)
    return h, info, Ug, Uo


@pytest.mark.parametrize("split", [2, 75, 148])
def test_channel_splits(env, split):
    fv, O = env
    check(fv, O, channel(), split, 3, 15)


@pytest.mark.parametrize("split,workers", [(2, 1), (150, 4), (298, 2)])
def test_inlet_block_splits(env, split, workers):
    fv, O = env
    check(fv, O, inlet_block(), split, workers, 15)


@pytest.mark.parametrize("rk", [2, 4])
def test_rk_schemes(env, rk):
    fv, O = env
    case = inlet_block()
    check(fv, O, case, 120, 3, 10, with_(case.params, rk=rk))


def test_workers_do_not_change_results(env):
    """Rows are dealt to the workers but summed in row order: 1 and 5 host
    workers give bitwise the same state and norms."""
    fv, _ = env
    case = inlet_block()
    h1, i1 = hetero_run(fv, case, 200, 1, 12)
    h5, i5 = hetero_run(fv, case, 200, 5, 12)
    assert np.array_equal(h1.get_state(), h5.get_state())
    assert i1["norm"] == i5["norm"] and i1["t"] == i5["t"]


def test_t_end_landing(env):
    """The last step is clamped so that t lands on t_end, as fv_step does."""
    fv, O = env
    case = channel()
    t_end = 0.0123
    prm = with_(case.params, t_end=t_end)
    h = fv.Hetero(case, 60, 2)
    h.set_state(case.state_flat())
    info = h.step(prm, 1000)
    ref = O.OracleGrid(case)
    io = ref.run(prm, 1000)
    e = P.state_err(case, h.get_state(), ref.get_state())
    say(f"  t_end {t_end}: {info['steps']} steps (ref {io['steps']}), t {info['t']!r}, e_U {e:.2e}")
    assert info["t"] == t_end and info["steps"] == io["steps"]
    assert info["flags"] & 4
    assert e <= P.FP64_TOL


def test_fp32_flux_gpu_part(env):
    fv, O = env
    case = inlet_block()
    p32 = with_(case.params, precision=CS.FP32_FLUX)
    h, _ = hetero_run(fv, case, 150, 3, 1, p32)
    ref = O.OracleGrid(case)
    ref.run(case.params, 1)
    e1 = P.state_err(case, h.get_state(), ref.get_state())
    h.step(p32, 19)
    ref.run(case.params, 19)
    eN = P.state_err(case, h.get_state(), ref.get_state())
    say(f"  fp32-flux GPU part: 1 step {e1:.2e}, 20 steps {eN:.2e}")
    assert e1 <= P.FP32_STEP_TOL and eN <= P.FP32_RUN_TOL


def test_inlet_full_size_split(env):
    """The inlet-like grid at its full 2048 x 256 size as one block, 32 host
    columns: 10 steps against the reference."""
    fv, O = env
    case = CS.inlet_case(2048, 256, 1, name="inlet_2d_1block")
    check(fv, O, case, 2048 - 32, 8, 10)


# ---------------------------------------------------------------------------
# Navier-Stokes
# ---------------------------------------------------------------------------
def ns_curved(imax=None, Ni=150, Nj=37):
    """The curved channel of the Navier-Stokes tests as one block: no-slip
    wall at rest below, a moving no-slip wall above, inflow at i-min and
    extrapolation (or the given rule) at i-max; mu = 2e-3."""
    from tests.test_gpu_ns import curved_channel
    c = curved_channel(Ni=Ni, Nj=Nj, icut=(), jcut=())
    if imax is not None:
        c.blocks[0].bc[1] = imax
    c.name = "ns_curved" + ("" if imax is None else f"_imax{imax.kind}")
    return c


def ns_uniform():
    """The uniform channel (periodic in j) with a viscosity."""
    c = channel()
    c.params = with_(c.params, mu=4e-3, prandtl=0.72)
    c.name = "ns_uniform"
    return c


@pytest.mark.parametrize("split,workers", [(2, 1), (77, 4), (148, 3)])
def test_ns_curved_splits(env, split, workers):
    fv, O = env
    check(fv, O, ns_curved(), split, workers, 12)


@pytest.mark.parametrize("imax", [CS.BC(CS.NOSLIP, prim=(0.0, 0.0, -0.2, 0.0, 0.0)),
                                  CS.BC(CS.SLIPWALL)])
def test_ns_walls_at_imax(env, imax):
    """A wall closing the host part's far end: its corner ghosts (the i-face
    rule, then the j-face rule) and reflected ghost centres."""
    fv, O = env
    check(fv, O, ns_curved(imax), 100, 3, 12)


@pytest.mark.parametrize("split", [3, 90])
def test_ns_uniform_periodic(env, split):
    fv, O = env
    check(fv, O, ns_uniform(), split, 2, 12)


@pytest.mark.parametrize("rk", [2, 4])
def test_ns_rk_schemes(env, rk):
    fv, O = env
    case = ns_curved()
    check(fv, O, case, 60, 3, 8, with_(case.params, rk=rk))


def test_ns_noslip_without_viscosity(env):
    """mu = 0 with no-slip walls: the Navier-Stokes kernel's inviscid path on
    the GPU part, the no-slip ghosts on both."""
    fv, O = env
    case = ns_curved()
    check(fv, O, case, 70, 2, 10, with_(case.params, mu=0.0))


def test_ns_fp32_flux_gpu_part(env):
    fv, O = env
    case = ns_curved()
    p32 = with_(case.params, precision=CS.FP32_FLUX)
    h, _ = hetero_run(fv, case, 75, 3, 1, p32)
    ref = O.OracleGrid(case)
    ref.run(case.params, 1)
    e1 = P.state_err(case, h.get_state(), ref.get_state())
    h.step(p32, 19)
    ref.run(case.params, 19)
    eN = P.state_err(case, h.get_state(), ref.get_state())
    say(f"  NS fp32-flux GPU part: 1 step {e1:.2e}, 20 steps {eN:.2e}")
    assert e1 <= P.FP32_STEP_TOL and eN <= P.FP32_RUN_TOL


def test_ns_inlet_full_size_split(env):
    """The viscous inlet grid (no-slip walls, mu = 1.5e-2) at its full
    2048 x 256 size as one block, 32 host columns: 6 steps."""
    fv, O = env
    case = CS.inlet_case(2048, 256, 1, name="inlet_2d_ns_1block")
    for f in (2, 3):
        case.blocks[0].bc[f] = CS.BC(CS.NOSLIP)
    case.params = with_(case.params, mu=1.5e-2, prandtl=0.72)
    check(fv, O, case, 2048 - 32, 8, 6)


def test_ns_workers_do_not_change_results(env):
    """The viscous host part too: 1 and 5 host workers give bitwise the same
    state and norms (rows are dealt out, summed in row order)."""
    fv, _ = env
    case = ns_curved()
    h1, i1 = hetero_run(fv, case, 60, 1, 8)
    h5, i5 = hetero_run(fv, case, 60, 5, 8)
    assert np.array_equal(h1.get_state(), h5.get_state())
    assert i1["norm"] == i5["norm"] and i1["t"] == i5["t"]
