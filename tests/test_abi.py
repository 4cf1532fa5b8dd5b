"""The C-ABI library loads, exports every symbol include/fv.h declares, and its
host-side logic (descriptor validation, workspace sizing, status strings)
behaves.  No device call is made here."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2305_18057_amd import cases as CS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(fv_[a-z_0-9]+)\s*\(", src)
    return sorted(set(names))


@pytest.fixture(scope="module")
def fvb():
    from paper_2305_18057_amd import fv
    if not os.path.exists(fv.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    fv.lib()
    return fv


def test_every_declared_symbol_exported(fvb):
    L = fvb.lib()
    names = declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(fvb.EXPORTS)


def test_status_strings_and_defaults(fvb):
    L = fvb.lib()
    assert L.fv_strerror(0) == b"ok"
    assert L.fv_strerror(-4) == b"non-physical state"
    p = fvb.fv_params()
    L.fv_default_params(C.byref(p))
    assert p.cfl == 0.5 and p.limiter == 0 and p.eps == 1.0 and p.kappa == -1.0 and p.rk == 3


def test_workspace_bytes_and_validation(fvb):
    L = fvb.lib()
    case = CS.inlet_case(128, 32, 2)
    gd = fvb.GridDesc(case)
    n = L.fv_grid_workspace_bytes(C.byref(gd.desc), 0)
    # three FP64 state buffers plus node coordinates at least
    assert n >= 3 * 8 * case.nv * case.ncells + 2 * 8 * 2 * 65 * 33
    # bad neighbour face -> rejected (0 bytes, error string set)
    case.blocks[0].bc[1] = CS.BC(CS.BLOCK, 1, CS.IMAX)
    gd = fvb.GridDesc(case)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"opposite face" in L.fv_last_error()
    # mismatched neighbour size -> rejected
    c2 = CS.inlet_case(128, 32, 2)
    c2.blocks[1] = CS.Block(64, 16, 1, None, None, (0, 0, 0), (1, 1, 1), c2.blocks[1].bc)
    gd = fvb.GridDesc(c2)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    # a periodic direction one cell deep has no second ghost source
    c1 = CS.vortex_2d(1, 4, noise=0.0)
    gd = fvb.GridDesc(c1)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"at least 2 cells" in L.fv_last_error()
    # a 3D curvilinear block needs x, y and z
    c3 = CS.blobs_case(8, nblobs=1)
    c3.blocks[0].x = np.zeros((9, 9, 9))
    c3.blocks[0].y = np.zeros((9, 9, 9))
    gd = fvb.GridDesc(c3)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"x, y and z" in L.fv_last_error()


def test_curvilinear_3d_and_source_descriptors(fvb):
    """3D node coordinates and the source buffer enter the workspace size;
    a 2D z, non-finite nodes or a bad with_source flag are refused; the
    allocation-free path refuses a source before any device work."""
    L = fvb.lib()
    c = CS.curv3d_case(ni=16, nj=8, nk=8, nblocks=2, state="random")
    gd = fvb.GridDesc(c)
    n_curv = L.fv_grid_workspace_bytes(C.byref(gd.desc), 0)
    nodes = sum(3 * 8 * (b.ni + 1) * (b.nj + 1) * (b.nk + 1) for b in c.blocks)
    assert n_curv >= 3 * 8 * c.nv * c.ncells + nodes
    cs = CS.curv3d_case(ni=16, nj=8, nk=8, nblocks=2, state="mms")
    gds = fvb.GridDesc(cs)
    assert gds.desc.with_source == 1
    n_src = L.fv_grid_workspace_bytes(C.byref(gds.desc), 0)
    assert n_src >= n_curv + 8 * c.nv * c.ncells
    gds.desc.with_source = 2
    assert L.fv_grid_workspace_bytes(C.byref(gds.desc), 0) == 0
    assert b"with_source" in L.fv_last_error()
    bad = CS.curv3d_case(ni=16, nj=8, nk=8, nblocks=1, state="random")
    bad.blocks[0].z[1, 2, 3] = np.nan
    g_bad = fvb.GridDesc(bad)
    assert L.fv_grid_workspace_bytes(C.byref(g_bad.desc), 0) == 0
    assert b"non-finite node" in L.fv_last_error()
    c2 = CS.inlet_case(64, 16, 1)
    c2.blocks[0].z = np.zeros((17, 65))
    g2 = fvb.GridDesc(c2)
    assert L.fv_grid_workspace_bytes(C.byref(g2.desc), 0) == 0
    assert b"z must be NULL" in L.fv_last_error()
    info = fvb.fv_step_info()
    p = fvb.make_params(cs.params)
    assert L.fv_step_noalloc(C.byref(gds.desc), C.c_void_p(256), C.byref(p), 1, None,
                             C.byref(info)) == fvb.FV_E_INVAL  # with_source = 2
    gds.desc.with_source = 1
    assert L.fv_step_noalloc(C.byref(gds.desc), C.c_void_p(256), C.byref(p), 1, None,
                             C.byref(info)) == fvb.FV_E_UNSUPPORTED
    assert b"source" in L.fv_last_error()


def test_oriented_block_links_validation(fvb):
    """3D links may join any two faces with any of the 8 orientations when the
    transverse sizes agree under it; 2D links stay opposite-face and
    unoriented; out-of-range faces and codes are refused."""
    L = fvb.lib()
    c = CS.curv3d_case(ni=24, nj=10, nk=8, nblocks=1, amp=0.05, state="random", seed=3)
    c.blocks[0].bc[0] = CS.BC(CS.INFLOW, prim=(1.0, 0.8, 0.1, 0.05, 0.7))
    c.blocks[0].bc[1] = CS.BC(CS.EXTRAP)
    r, _ = CS.reindex_3d(c, [6, 12, 18], CS.ROTATED_FRAMES["reversed"])
    gd = fvb.GridDesc(r)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) > 0
    b, f = next((b, f) for b, blk in enumerate(r.blocks) for f, bc in enumerate(blk.bc)
                if bc.kind == CS.BLOCK and bc.orient & 1)
    for field, value, msg in (("orient", lambda o: o ^ 1, b"transverse size"),
                              ("orient", lambda o: 8, b"orient"),
                              ("nbr_face", lambda o: 6, b"neighbour face")):
        gd = fvb.GridDesc(r)
        fc = gd.arr[b].face[f]
        setattr(fc, field, value(getattr(fc, field)))
        assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0, (field, value)
        assert msg in L.fv_last_error()
    gd = fvb.GridDesc(CS.twisted_box_3d(12))
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) > 0
    c2 = CS.inlet_case(64, 16, 2)
    for fld, val in (("orient", 2), ("nbr_face", 2)):
        gd = fvb.GridDesc(c2)
        setattr(gd.arr[0].face[1], fld, val)
        assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
        assert b"2D links join opposite faces" in L.fv_last_error()


def test_degenerate_grids_rejected(fvb):
    """Empty and degenerate descriptors are errors (0 bytes and a message),
    never a grid."""
    L = fvb.lib()
    for ni, nj in ((0, 8), (8, 0), (-4, 8)):
        c = CS.vortex_2d(8, 8, noise=0.0)
        b = c.blocks[0]
        c.blocks[0] = CS.Block(ni, nj, 1, None, None, b.origin, b.h, b.bc)
        gd = fvb.GridDesc(c)
        assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
        assert b"bad extents" in L.fv_last_error()
    c = CS.vortex_2d(8, 8, noise=0.0)
    gd = fvb.GridDesc(c)
    gd.desc.nblocks = 0
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"no blocks" in L.fv_last_error()
    gd = fvb.GridDesc(c)
    gd.desc.gamma = 1.0
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    gd = fvb.GridDesc(c)
    gd.desc.ndim = 4
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    c = CS.vortex_2d(8, 8, noise=0.0)
    b = c.blocks[0]
    c.blocks[0] = CS.Block(8, 8, 1, None, None, b.origin, (0.0, b.h[1], b.h[2]), b.bc)
    gd = fvb.GridDesc(c)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"spacing" in L.fv_last_error()


def test_create_grid_rejects_small_workspace(fvb):
    L = fvb.lib()
    case = CS.vortex_2d(16, 8)
    gd = fvb.GridDesc(case)
    h = C.c_void_p()
    st = L.fv_create_grid(C.byref(gd.desc), C.c_void_p(256), C.c_size_t(16), None, C.byref(h))
    assert st == fvb.FV_E_NOMEM and not h.value


def test_3d_plane_beyond_32bit_offsets_rejected(fvb):
    """The 3D kernels address a cell within a k-plane by a 32-bit byte offset,
    so a plane of 2^29 or more cells is refused, with the reason."""
    L = fvb.lib()
    bc = [CS.BC(CS.PERIODIC)] * 6
    for ni, nj, ok in ((32768, 16384, False), (16384, 32767, True)):
        blk = CS.Block(ni, nj, 4, None, None, (0, 0, 0), (1.0, 1.0, 1.0), bc)
        case = CS.Case("big_plane", 3, [blk], [], CS.Params(), 1)
        gd = fvb.GridDesc(case)
        n = L.fv_grid_workspace_bytes(C.byref(gd.desc), 0)
        if ok:
            assert n > 0
        else:
            assert n == 0 and b"32-bit" in L.fv_last_error()


def test_noalloc_rejects_grid_beyond_scratch_before_device_work(fvb):
    """The allocation-free step refuses a grid whose buffers exceed its static
    array, with the reason, before any device work (the pointer given is never
    dereferenced), and checks its arguments like fv_step."""
    L = fvb.lib()
    cap = int(L.fv_noalloc_scratch_bytes())
    assert cap == 64 << 20
    n = int(np.ceil(np.sqrt(cap / (2 * 4 * 8)))) + 8
    blk = CS.Block(n, n, 1, None, None, (0, 0, 0), (1.0, 1.0, 1.0), [CS.BC(CS.PERIODIC)] * 6)
    case = CS.Case("beyond_scratch", 2, [blk], [], CS.Params(), 1)
    gd = fvb.GridDesc(case)
    p = fvb.make_params(case.params)
    info = fvb.fv_step_info()
    st = L.fv_step_noalloc(C.byref(gd.desc), C.c_void_p(256), C.byref(p), 1, None, C.byref(info))
    assert st == fvb.FV_E_NOMEM and b"static scratch" in L.fv_last_error()
    small = CS.vortex_2d(16, 8)
    gd = fvb.GridDesc(small)
    p = fvb.make_params(small.params)
    assert L.fv_step_noalloc(C.byref(gd.desc), None, C.byref(p), 1, None, C.byref(info)) == fvb.FV_E_INVAL
    assert L.fv_step_noalloc(C.byref(gd.desc), C.c_void_p(256), C.byref(p), -1, None,
                             C.byref(info)) == fvb.FV_E_INVAL
    p.rk = 5
    assert L.fv_step_noalloc(C.byref(gd.desc), C.c_void_p(256), C.byref(p), 1, None,
                             C.byref(info)) == fvb.FV_E_UNSUPPORTED


def test_viscous_parameters_and_noslip_validation(fvb):
    """Defaults give an inviscid run with Pr 0.72; no-slip walls are 2D only
    and need two cells across; a negative viscosity or a viscous run without
    a Prandtl number is refused before any device work."""
    L = fvb.lib()
    p = fvb.fv_params()
    L.fv_default_params(C.byref(p))
    assert p.mu == 0.0 and p.prandtl == 0.72
    c = CS.inlet_case(64, 16, 1)
    c.blocks[0].bc[2] = CS.BC(CS.NOSLIP, prim=(0, 0.5, 0, 0, 0))
    gd = fvb.GridDesc(c)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) > 0
    c3 = CS.blobs_case(8, nblobs=1)
    c3.blocks[0].bc[2] = CS.BC(CS.NOSLIP)
    gd = fvb.GridDesc(c3)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"2D only" in L.fv_last_error()
    c1 = CS.vortex_2d(8, 1, noise=0.0)
    c1.blocks[0].bc[2] = CS.BC(CS.NOSLIP)
    gd = fvb.GridDesc(c1)
    assert L.fv_grid_workspace_bytes(C.byref(gd.desc), 0) == 0
    assert b"at least 2 cells" in L.fv_last_error()
    # parameter checks run before the device: the no-alloc entry shows them
    small = CS.vortex_2d(16, 8)
    gd = fvb.GridDesc(small)
    info = fvb.fv_step_info()
    for mu, pr in ((-1.0, 0.72), (1e-3, 0.0), (float("nan"), 0.72)):
        q = fvb.make_params(CS.Params(mu=mu, prandtl=pr))
        assert L.fv_step_noalloc(C.byref(gd.desc), C.c_void_p(256), C.byref(q), 1, None,
                                 C.byref(info)) == fvb.FV_E_INVAL
    q = fvb.make_params(CS.Params(mu=1e-3))
    g3 = fvb.GridDesc(CS.blobs_case(8, nblobs=1))
    assert L.fv_step_noalloc(C.byref(g3.desc), C.c_void_p(256), C.byref(q), 1, None,
                             C.byref(info)) == fvb.FV_E_UNSUPPORTED


def test_hetero_split_validation(fvb):
    """The CPU-GPU split takes one 2D block (Euler or Navier-Stokes, no
    source) cut along i with both parts at least 2 columns wide; everything
    else is refused before any device work (workspace size 0 and the
    reason)."""
    L = fvb.lib()
    c = CS.inlet_case(64, 16, 1)
    gd = fvb.GridDesc(c)
    n = L.fv_hetero_workspace_bytes(C.byref(gd.desc), 40)
    # the GPU part (40 columns and a 2-column halo block) in three state buffers
    assert n >= 3 * 8 * 4 * 16 * 42
    assert n < L.fv_grid_workspace_bytes(C.byref(gd.desc), 0)
    for split in (1, 63, 0, 64):
        assert L.fv_hetero_workspace_bytes(C.byref(gd.desc), split) == 0
        assert b"at least 2 columns" in L.fv_last_error()
    assert L.fv_hetero_workspace_bytes(C.byref(gd.desc), 2) > 0
    assert L.fv_hetero_workspace_bytes(C.byref(gd.desc), 62) > 0
    cases = [
        (CS.inlet_case(128, 16, 2), b"one 2D block"),
        (CS.blobs_case(8, nblobs=1), b"one 2D block"),
        (CS.vortex_2d(32, 16), b"may not be periodic"),
    ]
    c_ns = CS.inlet_case(64, 16, 1)
    c_ns.blocks[0].bc[2] = CS.BC(CS.NOSLIP)
    c_ns.blocks[0].bc[1] = CS.BC(CS.NOSLIP)
    g_ns = fvb.GridDesc(c_ns)
    assert L.fv_hetero_workspace_bytes(C.byref(g_ns.desc), 8) > 0
    c_src = CS.inlet_case(64, 16, 1)
    c_src.source = [np.zeros_like(u) for u in c_src.U0]
    cases.append((c_src, b"no source"))
    for case, msg in cases:
        g = fvb.GridDesc(case)
        assert L.fv_hetero_workspace_bytes(C.byref(g.desc), 8) == 0, case.name
        assert msg in L.fv_last_error(), (case.name, L.fv_last_error())
