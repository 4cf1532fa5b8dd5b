"""Scheduling logic of the serving loop, run without a device (dry-run mode:
each resident request takes one step per step slot and returns its initial
state).  Admission by arena footprint, slots, cancellation, oversize
rejection, completion of every request and the arena accounting."""
import time

import numpy as np
import pytest

from paper_2305_18057_amd import cases as CS


@pytest.fixture(scope="module")
def fvb():
    import os
    from paper_2305_18057_amd import fv
    if not os.path.exists(fv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    fv.lib()
    return fv


def wait_all(srv, tickets, timeout=20.0):
    out = {}
    t0 = time.time()
    while len(out) < len(tickets) and time.time() - t0 < timeout:
        for t in tickets:
            if t in out:
                continue
            r = srv.poll(t)
            if r is not None:
                out[t] = r
        time.sleep(0.001)
    return out


def test_dry_run_completes_every_request(fvb):
    srv = fvb.Server(arena_bytes=64 << 20, max_instances=3, steps_per_launch=7, dry_run=True)
    cases = [CS.inlet_case(64 * (1 + k % 3), 32, 1 + k % 2) for k in range(10)]
    tickets = [srv.submit(c, drop_tol=0.0, max_steps=20 + 5 * k) for k, c in enumerate(cases)]
    res = wait_all(srv, tickets)
    assert len(res) == 10
    for k, t in enumerate(tickets):
        st, U, info = res[t]
        assert st == fvb.FV_OK
        assert info["steps"] == 20 + 5 * k          # exact stop, not a multiple of the launch
        assert np.array_equal(U, cases[k].state_flat())
    s = srv.stats()
    assert s["submitted"] == 10 and s["admitted"] == 10 and s["completed"] == 10
    assert s["arena_used"] == 0 and s["resident"] == 0 and s["queued"] == 0
    assert s["arena_peak"] > 0
    srv.close()


def test_admission_bounded_by_arena_and_slots(fvb):
    big = CS.inlet_case(512, 256, 4)
    foot = fvb.workspace_bytes(big)
    # room for two of them (the arena header is well under half a footprint)
    srv = fvb.Server(arena_bytes=int(2.5 * foot), max_instances=8, steps_per_launch=5,
                     dry_run=True)
    tickets = [srv.submit(big, drop_tol=0.0, max_steps=400) for _ in range(5)]
    peak_resident = 0
    t0 = time.time()
    done = {}
    while len(done) < 5 and time.time() - t0 < 20:
        peak_resident = max(peak_resident, srv.stats()["resident"])
        for t in tickets:
            if t not in done:
                r = srv.poll(t)
                if r is not None:
                    done[t] = r
        time.sleep(0.0005)
    assert len(done) == 5
    assert peak_resident == 2
    assert srv.stats()["arena_peak"] <= 2.5 * foot
    srv.close()


def test_oversize_request_rejected(fvb):
    srv = fvb.Server(arena_bytes=32 << 20, max_instances=4, dry_run=True)
    with pytest.raises(fvb.FVError) as e:
        srv.submit(CS.inlet_case(2048, 1024, 4), max_steps=10)
    assert e.value.status == fvb.FV_E_NOMEM
    assert "arena bytes" in str(e.value)
    srv.close()


def test_server_takes_ssp_rk3_only(fvb):
    """Resident instances share one stage sequence: the 2- and 4-stage
    schemes are for grids, and the server says so."""
    srv = fvb.Server(arena_bytes=32 << 20, max_instances=4, dry_run=True)
    case = CS.inlet_case(64, 64, 1)
    for rk in (2, 4):
        prm = CS.Params(**{**case.params.__dict__, "rk": rk})
        with pytest.raises(fvb.FVError) as e:
            srv.submit(case, params=prm, max_steps=10)
        assert e.value.status == fvb.FV_E_UNSUPPORTED
    prm = CS.Params(**{**case.params.__dict__, "rk": 5})
    with pytest.raises(fvb.FVError) as e:
        srv.submit(case, params=prm, max_steps=10)
    assert e.value.status == fvb.FV_E_UNSUPPORTED
    srv.close()


def test_cancel_queued_and_resident(fvb):
    srv = fvb.Server(arena_bytes=64 << 20, max_instances=1, steps_per_launch=1, dry_run=True)
    c = CS.inlet_case(128, 64, 2)
    a = srv.submit(c, drop_tol=0.0, max_steps=10 ** 7)   # occupies the only slot
    b = srv.submit(c, drop_tol=0.0, max_steps=5)          # waits in the queue
    time.sleep(0.05)
    assert srv.cancel(b) == fvb.FV_OK
    assert srv.cancel(a) == fvb.FV_OK
    res = wait_all(srv, [a, b])
    assert res[a][0] == fvb.FV_E_CANCELLED and res[b][0] == fvb.FV_E_CANCELLED
    s = srv.stats()
    assert s["cancelled"] == 2 and s["arena_used"] == 0
    with pytest.raises(fvb.FVError):
        srv.poll(a)  # collected tickets are gone
    srv.close()


def test_request_times_and_unknown_ticket(fvb):
    srv = fvb.Server(arena_bytes=64 << 20, max_instances=2, dry_run=True)
    t = srv.submit(CS.vortex_2d(64, 32), drop_tol=0.0, max_steps=3)
    time.sleep(0.05)
    sub, adm, done = srv.times(t)
    assert 0.0 <= sub <= adm <= done <= srv.clock()
    assert srv.poll(t)[0] == fvb.FV_OK
    assert srv.cancel(t) == fvb.FV_E_NOTFOUND
    srv.close()


def test_server_takes_viscous_and_general_3d_grids(fvb):
    """Viscous 2D solves, no-slip walls, 3D curvilinear grids and oriented
    block links are served (the Navier-Stokes and the general 3D stage
    kernels run their own tile lists); every request completes in the dry
    run with its exact step count."""
    srv = fvb.Server(arena_bytes=64 << 20, max_instances=4, steps_per_launch=5, dry_run=True)
    visc = CS.inlet_case(64, 64, 1)
    prm = CS.Params(**{**visc.params.__dict__, "mu": 1e-3})
    wall = CS.inlet_case(64, 32, 2)
    wall.blocks[0].bc[2] = CS.BC(CS.NOSLIP)
    jobs = [(visc, prm, 12), (wall, None, 9),
            (CS.curv3d_case(ni=16, nj=8, nk=8, nblocks=2, state="random"), None, 7),
            (CS.twisted_box_3d(12), None, 11), (CS.inlet_case(64, 32, 1), None, 6)]
    tickets = [srv.submit(c, params=p, max_steps=n) for c, p, n in jobs]
    res = wait_all(srv, tickets)
    for (c, p, n), t in zip(jobs, tickets):
        st, U, info = res[t]
        assert st == fvb.FV_OK and info["steps"] == n
    srv.close()


def test_server_sources_and_3d_viscosity(fvb):
    """A grid with a source is served through fv_submit_with_source (the
    binding passes the case's source); fv_submit refuses such a descriptor
    and fv_submit_with_source one without it (FV_E_INVAL); a viscosity on a
    3D grid is FV_E_UNSUPPORTED."""
    import ctypes as C
    L = fvb.lib()
    srv = fvb.Server(arena_bytes=64 << 20, max_instances=4, steps_per_launch=4, dry_run=True)
    c2 = CS.inlet_case(64, 64, 1)
    c2.source = [np.zeros_like(u) for u in c2.U0]
    c3 = CS.curv3d_case(ni=16, nj=8, nk=8, nblocks=2, state="mms")
    ts = [srv.submit(c2, max_steps=9), srv.submit(c3, max_steps=6)]
    res = wait_all(srv, ts)
    assert [res[t][2]["steps"] for t in ts] == [9, 6]
    gd = fvb.GridDesc(c3)
    U = np.ascontiguousarray(c3.state_flat())
    p = fvb.make_params(c3.params)
    t = C.c_ulonglong()
    dp = C.POINTER(C.c_double)
    assert L.fv_submit(srv._h, C.byref(gd.desc), U.ctypes.data_as(dp), C.byref(p), 0.0, 5,
                       C.byref(t)) == fvb.FV_E_INVAL
    assert b"fv_submit_with_source" in L.fv_last_error()
    c0 = CS.inlet_case(64, 32, 1)
    g0 = fvb.GridDesc(c0)
    U0 = np.ascontiguousarray(c0.state_flat())
    assert L.fv_submit_with_source(srv._h, C.byref(g0.desc), U0.ctypes.data_as(dp),
                                   U0.ctypes.data_as(dp), C.byref(p), 0.0, 5,
                                   C.byref(t)) == fvb.FV_E_INVAL
    c3v = CS.blobs_case(8, nblobs=1)
    p3 = CS.Params(**{**c3v.params.__dict__, "mu": 1e-3})
    with pytest.raises(fvb.FVError) as e:
        srv.submit(c3v, params=p3, max_steps=10)
    assert e.value.status == fvb.FV_E_UNSUPPORTED
    srv.close()
