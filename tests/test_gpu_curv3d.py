"""General 3D path on the GPU (through the C ABI) against the CPU reference,
element by element: curvilinear 3D blocks (face area vectors and volumes from
the nodes, slip walls about curved wall faces), blocks in rotated index
frames joined face to face by oriented links, the source term of
Eq. (residual) in 3D (general kernel) and 2D (the Navier-Stokes kernel's
route), and the manufactured-solution order.

FP64: relative error <= 1e-12 (U metric; R on the flux scale, see parity.py).
FP32-flux: <= 1e-5 for one step from the same FP64 state, <= 1e-4 after N.
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


# ---------------------------------------------------------------------------
# cases
# ---------------------------------------------------------------------------
def curv_periodic():
    """Deformed periodic box, 144 x 10 x 9 cells in two blocks of 72 columns
    (a 64-column tile and a ragged 8-column one), rows 4 + 4 + 2."""
    return CS.curv3d_case(ni=144, nj=10, nk=9, nblocks=2, amp=0.05, state="random", seed=21)


def curv_walls():
    """The same box with its curved k-faces as slip walls, inflow at i-min and
    extrapolation at i-max: every slip-wall ghost is mirrored about a tilted
    wall normal."""
    c = CS.curv3d_case(ni=100, nj=9, nk=11, nblocks=2, amp=0.06, state="random", seed=22)
    prim = (1.1, 0.7, 0.2, -0.1, 0.8)
    c.blocks[0].bc[0] = CS.BC(CS.INFLOW, prim=prim)
    c.blocks[-1].bc[1] = CS.BC(CS.EXTRAP)
    for b in c.blocks:
        b.bc[4] = CS.BC(CS.SLIPWALL)
        b.bc[5] = CS.BC(CS.SLIPWALL)
    c.name = "curv_walls"
    return c


def curv_walls_ij():
    """Curved slip walls on the j-faces and the i-max face (the halo path of
    the general kernel), inflow at i-min, periodic in k; two blocks."""
    c = CS.curv3d_case(ni=90, nj=11, nk=10, nblocks=2, amp=0.06, state="random", seed=23)
    prim = (1.05, 0.3, 0.1, 0.05, 0.75)
    c.blocks[0].bc[0] = CS.BC(CS.INFLOW, prim=prim)
    c.blocks[-1].bc[1] = CS.BC(CS.SLIPWALL)
    for b in c.blocks:
        b.bc[2] = CS.BC(CS.SLIPWALL)
        b.bc[3] = CS.BC(CS.SLIPWALL)
    c.name = "curv_walls_ij"
    return c


def curv_mms(n=24):
    c = CS.curv3d_case(ni=2 * n, nj=n, nk=n, nblocks=2, amp=0.04, state="mms",
                       L=(2.0, 1.0, 1.0))
    c.name = f"curv_mms_{n}"
    return c


ROT_CUTS = {"swapped": [70, 110], "reversed": [70, 100, 125]}


def rotated(which, walls=False, state="random"):
    """A deformed 150 x 20 x 12 box cut along i into pieces with rotated and
    reflected index frames (the first piece 70 columns wide: a 64-column
    tile and a ragged one), joined by oriented links: inflow at i-min,
    extrapolation at i-max, periodic in k and in j, or slip walls on the
    j-faces (which fall on i-, j- or k-faces of the pieces)."""
    c = CS.curv3d_case(ni=150, nj=20, nk=12, nblocks=1, amp=0.05, state=state, seed=24)
    c.blocks[0].bc[0] = CS.BC(CS.INFLOW, prim=(1.0, 0.8, 0.1, 0.05, 0.7))
    c.blocks[0].bc[1] = CS.BC(CS.EXTRAP)
    if walls:
        c.blocks[0].bc[2] = CS.BC(CS.SLIPWALL)
        c.blocks[0].bc[3] = CS.BC(CS.SLIPWALL)
    r, _ = CS.reindex_3d(c, ROT_CUTS[which], CS.ROTATED_FRAMES[which],
                         name=f"rot_{which}{'_walls' if walls else ''}_{state}")
    return r


def uniform_with_source():
    """A uniform 3D block (exact axis metrics in the general kernel) with a
    seeded source."""
    c = CS.blobs_case(24, nblobs=2, seed=5)
    rng = np.random.default_rng(9)
    c.source = [0.05 * rng.standard_normal(u.shape) for u in c.U0]
    c.name = "blobs_source"
    return c


def vortex_with_source():
    c = CS.vortex_2d(96, 40, seed=3)
    rng = np.random.default_rng(10)
    c.source = [0.02 * rng.standard_normal(u.shape) for u in c.U0]
    c.name = "vortex_source"
    return c


def inlet_with_source():
    c = CS.inlet_case(130, 36, 2)
    rng = np.random.default_rng(11)
    c.source = [0.01 * rng.standard_normal(u.shape) * np.abs(u).max(axis=(1, 2, 3), keepdims=True)
                for u in c.U0]
    c.name = "inlet_source"
    return c


# ---------------------------------------------------------------------------
# checks
# ---------------------------------------------------------------------------
def check_residual(fv, O, case, params=None, tol=P.FP64_TOL):
    params = params or case.params
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Rg, ng = g.residual(params)
    ref = O.OracleGrid(case)
    Ro, no, scale = ref.residual(params, with_scale=True)
    e = P.residual_err(case, Rg, Ro, scale)
    say(f"  residual {case.name} lim={params.limiter}: e_R = {e:.3e}")
    assert e <= tol
    nv = case.nv
    vol = P.cell_volumes(case, ref)
    sv = P.per_var(scale, case)
    snorm = np.array([np.sqrt(np.mean((sv[v] / vol) ** 2)) for v in range(nv)])
    assert np.all(np.abs(ng[:nv] - no[:nv]) <= 1e-11 * np.abs(no[:nv]) + 1e-12 * snorm), (ng, no)
    return g, ref


def check_steps(fv, O, case, nsteps, params=None):
    params = params or case.params
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    info = g.step(params, nsteps)
    ref = O.OracleGrid(case)
    io = ref.run(params, nsteps)
    Uo = ref.get_state()
    e = P.state_err(case, g.get_state(), Uo)
    say(f"  {nsteps} steps {case.name} rk={params.rk}: e_U = {e:.3e} "
        f"(per component {P.component_errs(case, g.get_state(), Uo)}), t gpu {info['t']:.12g} "
        f"ref {io['t']:.12g}")
    assert info["steps"] == io["steps"] == nsteps
    assert e <= P.FP64_TOL
    assert abs(info["t"] - io["t"]) <= 1e-11 * abs(io["t"])
    assert abs(info["norm"] - io["norm"]) <= 1e-10 * io["norm"]
    return g, info, io, Uo


# ---------------------------------------------------------------------------
# tests
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("maker", [curv_walls, curv_walls_ij])
def test_curv3d_ghosts_with_curved_slip_walls(env, maker):
    fv, O = env
    case = maker()
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Gg = g.ghosts()
    ref = O.OracleGrid(case)
    Go = ref.ghosts()
    e = float(np.max(np.abs(Gg - Go)) / np.max(np.abs(Go)))
    say(f"  ghosts {case.name}: max rel {e:.2e}")
    assert e <= 1e-14


@pytest.mark.parametrize("maker", [curv_periodic, curv_walls, curv_walls_ij])
@pytest.mark.parametrize("limiter", [CS.MINMOD, CS.UNLIMITED])
def test_curv3d_residual(env, maker, limiter):
    fv, O = env
    case = maker()
    check_residual(fv, O, case, with_(case.params, limiter=limiter))


@pytest.mark.parametrize("maker", [curv_periodic, curv_walls, curv_walls_ij])
def test_curv3d_steps(env, maker):
    fv, O = env
    check_steps(fv, O, maker(), 12)


@pytest.mark.parametrize("rk", [2, 4])
def test_curv3d_rk_schemes(env, rk):
    fv, O = env
    case = curv_periodic()
    check_steps(fv, O, case, 8, with_(case.params, rk=rk))


def test_curv3d_fp32_flux(env):
    fv, O = env
    case = curv_walls()
    p32 = with_(case.params, precision=CS.FP32_FLUX)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    g.step(p32, 1)
    ref = O.OracleGrid(case)
    ref.run(case.params, 1)
    e1 = P.state_err(case, g.get_state(), ref.get_state())
    g.step(p32, 19)
    io = ref.run(case.params, 19)
    eN = P.state_err(case, g.get_state(), ref.get_state())
    say(f"  fp32-flux {case.name}: 1 step {e1:.2e}, 20 steps {eN:.2e}")
    assert 1e-12 < e1 <= P.FP32_STEP_TOL
    assert eN <= P.FP32_RUN_TOL


def test_curv3d_free_stream_stays(env):
    """A uniform stream on the deformed periodic box: the face vectors of each
    cell close, so the state stays uniform (a property at any size)."""
    fv, O = env
    case = CS.curv3d_case(ni=128, nj=40, nk=36, nblocks=2, amp=0.06, state="uniform")
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    R, _ = g.residual()
    info = g.step(case.params, 10)
    d = np.max(np.abs(g.get_state() - case.state_flat())) / np.max(np.abs(case.state_flat()))
    say(f"  free stream {case.ncells} cells: max |R| {np.max(np.abs(R)):.2e}, 10 steps drift {d:.2e}")
    assert np.max(np.abs(R)) <= 1e-13
    assert d <= 1e-13 and info["steps"] == 10


def test_mms_source_parity(env):
    fv, O = env
    case = curv_mms(24)
    for lim in (CS.MINMOD, CS.UNLIMITED):
        check_residual(fv, O, case, with_(case.params, limiter=lim))
    check_steps(fv, O, case, 10)


def test_mms_truncation_order_on_gpu(env):
    """The GPU residual of the manufactured state with its source falls at
    second order (unlimited MUSCL) from 24 to 48 cells per unit length."""
    fv, O = env
    errs = []
    for n in (24, 48):
        case = curv_mms(n)
        prm = with_(case.params, limiter=CS.UNLIMITED)
        g = fv.Grid(case)
        g.set_state(case.state_flat())
        R, _ = g.residual(prm)
        ref = O.OracleGrid(case)
        vol = np.concatenate([np.tile(ref.metrics_3d(b)[1].ravel(), case.nv)
                              for b in range(len(case.blocks))])
        e = R / vol
        errs.append((np.sqrt(np.mean(e * e)), np.max(np.abs(e))))
    o2, oi = (np.log2(errs[0][a] / errs[1][a]) for a in range(2))
    say(f"  MMS truncation 24 -> 48: RMS {errs[0][0]:.3e} -> {errs[1][0]:.3e} (order {o2:.3f}), "
        f"max order {oi:.3f}")
    assert o2 > 1.9 and oi > 1.9


def test_uniform_3d_with_source(env):
    fv, O = env
    case = uniform_with_source()
    check_residual(fv, O, case)
    check_steps(fv, O, case, 10)


@pytest.mark.parametrize("maker", [vortex_with_source, inlet_with_source])
def test_2d_with_source(env, maker):
    fv, O = env
    case = maker()
    check_residual(fv, O, case)
    check_steps(fv, O, case, 10)


def test_set_source_on_device_and_zero(env):
    """fv_set_source from a device tensor gives the host-copy result; NULL
    returns the grid to the sourceless residual."""
    import torch
    fv, O = env
    case = curv_mms(16)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    R1, _ = g.residual()
    g.set_source(torch.tensor(case.source_flat(), device="cuda"))
    R2, _ = g.residual()
    assert np.array_equal(R1, R2)
    g.set_source(None)
    R0, _ = g.residual()
    ref = O.OracleGrid(case)
    ref.set_source(None)
    Ro, _, scale = ref.residual(case.params, with_scale=True)
    e = P.residual_err(case, R0, Ro, scale)
    say(f"  source cleared: e_R = {e:.2e}")
    assert e <= P.FP64_TOL


def test_curv3d_mms_full_size(env):
    """The 192^3 manufactured-solution workload (the size the benchmark
    times): residual and one step element by element against the oracle."""
    fv, O = env
    case = CS.curv3d_mms(192)
    say(f"  curv3d_mms 192^3: {case.ncells} cells")
    check_residual(fv, O, case)
    check_steps(fv, O, case, 1)


# ---------------------------------------------------------------------------
# oriented block links
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("which", sorted(CS.ROTATED_FRAMES))
def test_oriented_links_ghosts(env, which):
    fv, O = env
    case = rotated(which, walls=True)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    Gg = g.ghosts()
    Go = O.OracleGrid(case).ghosts()
    e = float(np.max(np.abs(Gg - Go)) / np.max(np.abs(Go)))
    say(f"  ghosts {case.name}: max rel {e:.2e}")
    assert e <= 1e-14


@pytest.mark.parametrize("which", sorted(CS.ROTATED_FRAMES))
@pytest.mark.parametrize("walls", [False, True])
@pytest.mark.parametrize("limiter", [CS.MINMOD, CS.UNLIMITED])
def test_oriented_links_residual(env, which, walls, limiter):
    fv, O = env
    case = rotated(which, walls)
    check_residual(fv, O, case, with_(case.params, limiter=limiter))


@pytest.mark.parametrize("which", sorted(CS.ROTATED_FRAMES))
def test_oriented_links_steps(env, which):
    fv, O = env
    check_steps(fv, O, rotated(which, walls=True), 10)


def test_oriented_links_mms_source(env):
    fv, O = env
    case = rotated("reversed", state="mms")
    check_residual(fv, O, case)
    check_steps(fv, O, case, 8)


def test_oriented_links_fp32_flux(env):
    fv, O = env
    case = rotated("reversed", walls=True)
    p32 = with_(case.params, precision=CS.FP32_FLUX)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    g.step(p32, 1)
    ref = O.OracleGrid(case)
    ref.run(case.params, 1)
    e1 = P.state_err(case, g.get_state(), ref.get_state())
    g.step(p32, 11)
    ref.run(case.params, 11)
    eN = P.state_err(case, g.get_state(), ref.get_state())
    say(f"  fp32-flux {case.name}: 1 step {e1:.2e}, 12 steps {eN:.2e}")
    assert e1 <= P.FP32_STEP_TOL and eN <= P.FP32_RUN_TOL


def test_twisted_uniform_box(env):
    """Uniform blocks whose links are oriented run the general kernel too
    (the uniform 3D kernel reads opposite faces unoriented): a 70^3 box
    joined to itself with reversed and swapped transverse indices."""
    fv, O = env
    case = CS.twisted_box_3d(70)
    check_residual(fv, O, case)
    check_steps(fv, O, case, 6)
