"""Solution-level pins of the CPU reference: exact Riemann solution of the
Sod tube and second-order convergence on an advected isentropic vortex."""
import math

import numpy as np
import pytest

from paper_2305_18057_amd import cases as C
from tests import exact_riemann as ER

G = 1.4
SOD_L = (1.0, 0.0, 1.0)
SOD_R = (0.125, 0.0, 0.1)


# ---------------------------------------------------------------------------
# the exact solver is pinned by the jump conditions it must satisfy
# ---------------------------------------------------------------------------
def test_exact_riemann_jump_conditions():
    ps, us, rsl, rsr = ER.star_state(SOD_L, SOD_R, G)
    # right shock: mass, momentum and energy fluxes equal in the shock frame
    S = ER.right_shock_speed(SOD_L, SOD_R, G)
    rr, ur, pr = SOD_R

    def fluxes(rho, u, p):
        E = p / (G - 1) + 0.5 * rho * u * u
        return np.array([rho * (u - S), rho * u * (u - S) + p, E * (u - S) + p * u])

    assert np.allclose(fluxes(rsr, us, ps), fluxes(rr, ur, pr), rtol=1e-12, atol=1e-12)
    # left rarefaction: isentropic, left Riemann invariant u + 2c/(g-1) kept
    rl, ul, pl = SOD_L
    assert ps / rsl ** G == pytest.approx(pl / rl ** G, rel=1e-12)
    cl, csl = math.sqrt(G * pl / rl), math.sqrt(G * ps / rsl)
    assert us + 2 * csl / (G - 1) == pytest.approx(ul + 2 * cl / (G - 1), rel=1e-12)
    # star state of the Sod data lies where the textbook puts it
    assert 0.30 < ps < 0.31 and 0.92 < us < 0.93


def _sod_run(orc, n, limiter=C.MINMOD):
    case = C.sod_2d(n=n, nj=4, t_end=0.2, limiter=limiter)
    g = orc.OracleGrid(case)
    info = g.run(case.params, 100000)
    assert info["status"] == 0 and info["t"] == 0.2
    U = g.get_state().reshape(4, 4, n)
    h = 1.0 / n
    xc = (np.arange(n) + 0.5) * h
    rho_e, u_e, p_e = ER.sample(SOD_L, SOD_R, (xc - 0.5) / 0.2, G)
    return U, rho_e, h, xc


def test_sod_against_exact(orc):
    U4, re4, h4, x4 = _sod_run(orc, 400)
    U2, re2, h2, _ = _sod_run(orc, 200)
    e4 = np.sum(np.abs(U4[0, 0] - re4)) * h4
    e2 = np.sum(np.abs(U2[0, 0] - re2)) * h2
    assert e4 <= 4e-3
    assert math.log(e2 / e4, 2) >= 0.5
    # rows identical, no transverse momentum
    assert all(np.array_equal(U4[:, j], U4[:, 0]) for j in range(4))
    assert np.all(U4[2] == 0.0)
    # shock position within 2 cells: where rho crosses the mid value between
    # the post-shock and the right state
    ps, us, rsl, rsr = ER.star_state(SOD_L, SOD_R, G)
    xs = 0.5 + 0.2 * ER.right_shock_speed(SOD_L, SOD_R, G)
    mid = 0.5 * (rsr + SOD_R[0])
    rho = U4[0, 0]
    idx = np.where((x4 > 0.75) & (rho < mid))[0][0]
    assert abs(x4[idx] - xs) <= 2 * h4


# ---------------------------------------------------------------------------
# isentropic vortex advected for t = 1 on a periodic box: exact solution is the
# initial vortex translated by u_inf * t
# ---------------------------------------------------------------------------
def _vortex_err(orc, ni, limiter, t_end=1.0):
    nj = ni // 2
    case = C.vortex_2d(ni, nj, noise=0.0, limiter=limiter)
    hx = case.blocks[0].h[0]
    uinf = case.meta["uinf"]
    c = math.sqrt(G)
    dt = 0.4 * hx / (uinf + 2 * c)
    nsteps = int(math.ceil(t_end / dt))
    dt = t_end / nsteps
    prm = C.Params(dt_fixed=dt, limiter=limiter, qref=case.params.qref)
    g = orc.OracleGrid(case)
    info = g.run(prm, nsteps)
    assert info["status"] == 0
    rho = g.get_state().reshape(4, nj, ni)[0]
    h = case.blocks[0].h
    X, Y = np.meshgrid((np.arange(ni) + 0.5) * h[0], (np.arange(nj) + 0.5) * h[1])
    re, _, _, _ = C.vortex_fields(10.0 + uinf * t_end, 5.0, X, Y)
    d = rho - re
    return math.sqrt(np.mean(d * d)), np.mean(np.abs(d))


def test_vortex_second_order_unlimited(orc):
    e1 = _vortex_err(orc, 64, C.UNLIMITED)[0]
    e2 = _vortex_err(orc, 128, C.UNLIMITED)[0]
    e3 = _vortex_err(orc, 256, C.UNLIMITED)[0]
    order = math.log(e2 / e3, 2)
    assert math.log(e1 / e2, 2) > 1.5
    assert order >= 1.8, (e1, e2, e3)


def test_vortex_order_minmod(orc):
    e2 = _vortex_err(orc, 128, C.MINMOD)[1]
    e3 = _vortex_err(orc, 256, C.MINMOD)[1]
    assert math.log(e2 / e3, 2) >= 1.4, (e2, e3)
