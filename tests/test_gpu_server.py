"""Batched execution and the serving loop on the GPU.

Each served instance must give the same state alone and in any mix (bitwise:
its arithmetic and its reductions use only its own tiles, in a fixed order),
stop at exactly its own stop step, and match the CPU reference like a grid
solved on its own.
"""
import time

import numpy as np
import pytest

from paper_2305_18057_amd import cases as CS
from tests import parity as P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    from paper_2305_18057_amd import fv
    from oracle import oracle as O
    fv.lib()
    return fv, O


def drain(srv, tickets, timeout=120.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets):
        assert time.time() - t0 < timeout, "server did not finish in time"
        for t in tickets:
            if t not in out:
                r = srv.poll(t)
                if r is not None:
                    out[t] = r
        time.sleep(0.0005)
    return out


def mixed_cases():
    cs = [CS.inlet_case(192, 48, 3, mach=2.5, angle_deg=4.0, name="m0"),
          CS.inlet_case(64, 64, 1, mach=3.0, name="m1"),
          CS.blobs_case(24, nblobs=3, seed=11, name="m2"),
          CS.inlet_case(320, 40, 2, mach=1.8, angle_deg=8.0, name="m3"),
          CS.vortex_2d(96, 48, seed=3),
          CS.blobs_case(40, nblobs=2, seed=12, mach=2.5, name="m5")]
    return cs


@pytest.mark.parametrize("prec", [CS.FP64, CS.FP32_FLUX])
def test_alone_equals_in_mix(env, prec):
    fv, O = env
    cs = mixed_cases()
    steps = [37, 23, 41, 19, 30, 26]  # not multiples of the launch length
    alone = []
    for c, n in zip(cs, steps):
        srv = fv.Server(arena_bytes=256 << 20, max_instances=4, precision=prec, steps_per_launch=7)
        t = srv.submit(c, drop_tol=0.0, max_steps=n)
        alone.append(drain(srv, [t])[t])
        srv.close()
    srv = fv.Server(arena_bytes=256 << 20, max_instances=3, precision=prec, steps_per_launch=7)
    ts = [srv.submit(c, drop_tol=0.0, max_steps=n) for c, n in zip(cs, steps)]
    mix = drain(srv, ts)
    tol = P.FP64_TOL if prec == CS.FP64 else P.FP32_RUN_TOL
    for k, t in enumerate(ts):
        st, U, info = mix[t]
        st0, U0, info0 = alone[k]
        assert st == fv.FV_OK and st0 == fv.FV_OK
        assert info["steps"] == steps[k] and info0["steps"] == steps[k]
        assert np.array_equal(U, U0), f"instance {k} differs alone vs in mix"
        assert info["t"] == info0["t"] and info["norm"] == info0["norm"]
        # and each instance of the mix against the oracle (FP64)
        ref = O.OracleGrid(cs[k])
        io = ref.run(cs[k].params, steps[k])
        e = P.state_err(cs[k], U, ref.get_state())
        P.report("test_alone_equals_in_mix",
                 f"prec={prec} in-mix {cs[k].name} ({cs[k].ndim}D, {len(cs[k].blocks)} blocks) "
                 f"{steps[k]} steps: e_U = {e:.3e}")
        assert io["steps"] == steps[k] and e <= tol, (cs[k].name, e)
        assert abs(info["t"] - io["t"]) <= (1e-11 if prec == CS.FP64 else 1e-4) * io["t"]
    s = srv.stats()
    assert s["completed"] == len(cs) and s["arena_used"] == 0
    srv.close()


def test_served_equals_grid_and_reference(env):
    fv, O = env
    for c in (CS.inlet_case(256, 64, 4, angle_deg=5.0), CS.blobs_case(32, nblobs=4)):
        srv = fv.Server(arena_bytes=256 << 20, max_instances=2, precision=CS.FP64, steps_per_launch=10)
        t = srv.submit(c, drop_tol=0.0, max_steps=25)
        st, U, info = drain(srv, [t])[t]
        srv.close()
        g = fv.Grid(c)
        g.set_state(c.state_flat())
        gi = g.step(c.params, 25)
        assert np.array_equal(U, g.get_state())
        ref = O.OracleGrid(c)
        io = ref.run(c.params, 25)
        e = P.state_err(c, U, ref.get_state())
        P.report("test_served_equals_grid_and_reference", f"served {c.name} 25 steps: e_U = {e:.3e}")
        assert info["steps"] == io["steps"] == 25 and e <= P.FP64_TOL, e


def batch_subset():
    """A seeded subset of the 64-instance batch (the same generator and seed):
    the two smallest instances of each block count 1..4."""
    cs = CS.batch_2d(64)
    out = []
    for nb in (1, 2, 3, 4):
        sel = sorted([c for c in cs if len(c.blocks) == nb], key=lambda c: c.ncells)[:2]
        out += sel
    return out


def test_served_fp32_batch_against_oracle_and_grid(env):
    """Instances of the batched workload (1-4 blocks, Mach 1.5-4, sheared
    inlet mesh), served in FP32-flux with four resident at a time: each
    within the after-N bar of the FP64 oracle and bitwise equal to the same
    instance stepped alone on its own grid."""
    fv, O = env
    cs = batch_subset()
    assert sorted({len(c.blocks) for c in cs}) == [1, 2, 3, 4]
    steps = [23 + 4 * k for k in range(len(cs))]  # not multiples of the launch length
    srv = fv.Server(arena_bytes=512 << 20, max_instances=4, precision=CS.FP32_FLUX,
                    steps_per_launch=10)
    ts = [srv.submit(c, drop_tol=0.0, max_steps=n) for c, n in zip(cs, steps)]
    res = drain(srv, ts, timeout=300.0)
    stats = srv.stats()
    srv.close()
    p32 = lambda c: CS.Params(**{**c.params.__dict__, "precision": CS.FP32_FLUX})
    for c, n, t in zip(cs, steps, ts):
        st, U, info = res[t]
        assert st == fv.FV_OK and info["steps"] == n
        g = fv.Grid(c)
        g.set_state(c.state_flat())
        g.step(p32(c), n)
        assert np.array_equal(U, g.get_state()), f"{c.name} served differs from its own grid"
        g.close()
        ref = O.OracleGrid(c)
        ref.run(c.params, n)
        e = P.state_err(c, U, ref.get_state())
        P.report("test_served_fp32_batch_against_oracle_and_grid",
                 f"served fp32-flux {c.name} ({c.blocks[0].ni * len(c.blocks)}x{c.blocks[0].nj}, "
                 f"{len(c.blocks)} blocks) {n} steps: e_U = {e:.3e}")
        print(f"  {c.name}: {len(c.blocks)} blocks, {c.ncells} cells, {n} steps, e_U = {e:.3e}",
              flush=True)
        assert 1e-12 < e <= P.FP32_RUN_TOL, (c.name, e)
    assert stats["completed"] == len(cs) and stats["arena_used"] == 0


def test_drop_tolerance_stop_matches_solve(env):
    fv, O = env
    c = CS.inlet_case(128, 32, 2, angle_deg=6.0)
    g = fv.Grid(c)
    g.set_state(c.state_flat())
    gi = g.step(c.params, 60)
    # a tolerance the drop crosses inside the run
    tol = gi["drop"] * 1.000001
    g2 = fv.Grid(c)
    g2.set_state(c.state_flat())
    si = g2.solve(c.params, drop_tol=tol, max_steps=500)
    srv = fv.Server(arena_bytes=128 << 20, max_instances=2, precision=CS.FP64, steps_per_launch=9)
    t = srv.submit(c, drop_tol=tol, max_steps=500)
    st, U, info = drain(srv, [t])[t]
    srv.close()
    assert info["steps"] == si["steps"] and info["flags"] & fv.FLAG_CONVERGED
    assert np.array_equal(U, g2.get_state())


def test_failure_isolated(env):
    fv, O = env
    good = CS.inlet_case(128, 32, 2)
    bad = CS.sod_2d(n=64, nj=4, t_end=0.0)
    bad_p = CS.Params(**{**bad.params.__dict__, "dt_fixed": 0.2})  # far past the CFL limit
    srv = fv.Server(arena_bytes=128 << 20, max_instances=4, precision=CS.FP64, steps_per_launch=5)
    tg = srv.submit(good, drop_tol=0.0, max_steps=20)
    tb = srv.submit(bad, drop_tol=0.0, max_steps=20, params=bad_p)
    res = drain(srv, [tg, tb])
    srv.close()
    assert res[tb][0] == fv.FV_E_NONPHYSICAL and res[tb][2]["steps"] < 20
    assert res[tg][0] == fv.FV_OK and res[tg][2]["steps"] == 20
    g = fv.Grid(good)
    g.set_state(good.state_flat())
    g.step(good.params, 20)
    assert np.array_equal(res[tg][1], g.get_state())


def test_continuous_admission_under_load(env):
    """More requests than slots and arena: later ones are admitted as earlier
    ones retire, while the others keep running."""
    fv, O = env
    cs = [CS.inlet_case(64 * (1 + k % 4), 32 + 16 * (k % 3), 1 + k % 3, mach=1.5 + 0.2 * k,
                        name=f"q{k}") for k in range(12)]
    srv = fv.Server(arena_bytes=48 << 20, max_instances=4, precision=CS.FP32_FLUX, steps_per_launch=5)
    ts = [srv.submit(c, drop_tol=0.0, max_steps=15 + 3 * k) for k, c in enumerate(cs)]
    res = drain(srv, ts)
    s = srv.stats()
    srv.close()
    assert all(res[t][0] == fv.FV_OK for t in ts)
    assert [res[t][2]["steps"] for t in ts] == [15 + 3 * k for k in range(12)]
    assert s["admitted"] == 12 and s["launches"] > 0 and s["arena_used"] == 0


def test_served_viscous_and_general_3d_mixed(env):
    """Navier-Stokes instances (a viscosity and no-slip walls, six linked
    blocks), a 3D curvilinear grid and blocks in rotated frames joined by
    oriented links, served together with an Euler instance (four tile lists
    in each batched launch): each bitwise equal to the same grid stepped
    alone, and within the FP64 bar of the oracle."""
    fv, O = env
    from tests.test_gpu_ns import curved_channel
    from tests.test_gpu_curv3d import rotated
    c3 = CS.curv3d_case(ni=100, nj=9, nk=11, nblocks=2, amp=0.06, state="random", seed=22)
    jobs = [(curved_channel(), 17), (c3, 13), (rotated("reversed", walls=True), 11),
            (CS.inlet_case(256, 64, 4, angle_deg=5.0), 15)]
    srv = fv.Server(arena_bytes=512 << 20, max_instances=4, precision=CS.FP64, steps_per_launch=10)
    ts = [srv.submit(c, params=c.params, drop_tol=0.0, max_steps=n) for c, n in jobs]
    res = drain(srv, ts, timeout=300.0)
    srv.close()
    for (c, n), t in zip(jobs, ts):
        st, U, info = res[t]
        assert st == fv.FV_OK and info["steps"] == n, (c.name, st, info["steps"])
        g = fv.Grid(c)
        g.set_state(c.state_flat())
        g.step(c.params, n)
        Ug = g.get_state()
        g.close()
        ref = O.OracleGrid(c)
        ref.run(c.params, n)
        e = P.state_err(c, U, ref.get_state())
        P.report("test_served_viscous_and_general_3d_mixed",
                 f"served {c.name} {n} steps: e_U = {e:.3e}, bitwise = grid: {np.array_equal(U, Ug)}")
        assert np.array_equal(U, Ug), c.name
        assert e <= P.FP64_TOL, (c.name, e)


def test_served_sources(env):
    """Grids with a source S_h (fv_submit_with_source): the manufactured
    solution on a 3D curvilinear box and a 2D vortex with a seeded source,
    served with an Euler instance; each bitwise equal to the same grid with
    its source stepped alone, and within the FP64 bar of the oracle."""
    fv, O = env
    from tests.test_gpu_curv3d import curv_mms, vortex_with_source
    jobs = [(curv_mms(16), 9), (vortex_with_source(), 14), (CS.blobs_case(24, nblobs=2), 7)]
    srv = fv.Server(arena_bytes=256 << 20, max_instances=3, precision=CS.FP64, steps_per_launch=4)
    ts = [srv.submit(c, drop_tol=0.0, max_steps=n) for c, n in jobs]
    res = drain(srv, ts, timeout=300.0)
    srv.close()
    for (c, n), t in zip(jobs, ts):
        st, U, info = res[t]
        assert st == fv.FV_OK and info["steps"] == n, (c.name, st)
        g = fv.Grid(c)
        g.set_state(c.state_flat())
        g.step(c.params, n)
        Ug = g.get_state()
        g.close()
        ref = O.OracleGrid(c)
        ref.run(c.params, n)
        e = P.state_err(c, U, ref.get_state())
        P.report("test_served_sources", f"served {c.name} {n} steps: e_U = {e:.3e}, bitwise = grid: "
                 f"{np.array_equal(U, Ug)}")
        assert np.array_equal(U, Ug), c.name
        assert e <= P.FP64_TOL, (c.name, e)
