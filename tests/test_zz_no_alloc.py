"""fv_step_noalloc (every buffer beyond the caller's state in the library's
static device array) against fv_step on a grid with its own workspace.  Both
run the same kernels, so the states and the step info agree bitwise.  Each
test makes two calls in a row, the second on a smaller grid, so the second
call runs over what the first left in the shared array."""
import numpy as np
import pytest

from paper_2305_18057_amd import cases as CS

pytestmark = pytest.mark.gpu


def _perturbed(case, seed=11, amp=0.01):
    rng = np.random.default_rng(seed)
    for U in case.U0:
        U[0] *= 1.0 + amp * rng.uniform(-1.0, 1.0, size=U[0].shape)
    return case


def _with(params, **kw):
    return CS.Params(**{**params.__dict__, **kw})


def _run_pair(case, params, nsteps):
    import torch
    from paper_2305_18057_amd import fv
    print(f"  noalloc case {case.name}: {case.ncells} cells, prec={params.precision}, "
          f"rk={params.rk}, {nsteps} steps", flush=True)
    g = fv.Grid(case)
    g.set_state(case.state_flat())
    ref = g.step(params, nsteps)
    Uref = g.get_state()
    g.close()
    U = torch.from_numpy(case.state_flat()).to("cuda")
    got = fv.step_noalloc(case, U, params, nsteps)
    torch.cuda.synchronize()
    Ug = U.cpu().numpy()
    assert got["steps"] == ref["steps"] == nsteps
    assert got["t"] == ref["t"] and got["dt_last"] == ref["dt_last"]
    assert np.array_equal(got["norms"], ref["norms"]) and got["drop"] == ref["drop"]
    assert got["flags"] == ref["flags"]
    assert np.array_equal(Ug, Uref), np.max(np.abs(Ug - Uref))
    return Ug


def test_noalloc_2d_then_smaller():
    from paper_2305_18057_amd import fv
    fv.lib()
    big = _perturbed(CS.inlet_case(4 * 128, 64, 4, angle_deg=3.0))
    _run_pair(big, big.params, 13)
    small = CS.vortex_2d(64, 32)
    _run_pair(small, small.params, 7)


def test_noalloc_3d_fp32_flux_then_smaller():
    from paper_2305_18057_amd import fv
    fv.lib()
    big = CS.blobs_case(32, nblobs=4)
    _run_pair(big, _with(big.params, precision=CS.FP32_FLUX), 6)
    small = _perturbed(CS.blobs_case(16, nblobs=2, seed=7))
    _run_pair(small, _with(small.params, rk=4), 5)


def test_noalloc_3d_curvilinear_then_smaller():
    """3D curvilinear grids run the general 3D stage kernel, here too."""
    from paper_2305_18057_amd import fv
    fv.lib()
    big = CS.curv3d_case(ni=96, nj=20, nk=18, nblocks=2, amp=0.05, state="random", seed=12)
    _run_pair(big, big.params, 6)
    small = CS.curv3d_case(ni=40, nj=9, nk=8, nblocks=1, amp=0.04, state="random", seed=13,
                           walls_k=True)
    _run_pair(small, _with(small.params, precision=CS.FP32_FLUX), 4)


def test_noalloc_oriented_links_then_smaller():
    """Oriented block links (the general 3D kernel's signed plane strides)."""
    from paper_2305_18057_amd import fv
    fv.lib()
    big = CS.twisted_box_3d(40)
    _run_pair(big, big.params, 5)
    c = CS.curv3d_case(ni=24, nj=10, nk=8, nblocks=1, amp=0.05, state="random", seed=3)
    c.blocks[0].bc[0] = CS.BC(CS.INFLOW, prim=(1.0, 0.8, 0.1, 0.05, 0.7))
    c.blocks[0].bc[1] = CS.BC(CS.EXTRAP)
    small, _ = CS.reindex_3d(c, [6, 12, 18], CS.ROTATED_FRAMES["reversed"], name="rot_small")
    _run_pair(small, small.params, 4)


def test_noalloc_rejects_grid_beyond_scratch():
    import torch
    from paper_2305_18057_amd import fv
    L = fv.lib()
    cap = int(L.fv_noalloc_scratch_bytes())
    n = int(np.ceil(np.sqrt(cap / (2 * 4 * 8)))) + 8
    bcs = [CS.BC(CS.PERIODIC)] * 6
    case = CS.uniform_2d(n, n, (1.0, 0.5, 0.0, 0.0, 1.0), bcs)
    U = torch.from_numpy(case.state_flat()).to("cuda")
    before = U.clone()
    d = fv.step_noalloc(case, U, case.params, 1, check=False)
    assert d["status"] == fv.FV_E_NOMEM
    assert b"static scratch" in L.fv_last_error()
    assert torch.equal(U, before)
