"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas).

Written from the textbook construction (E. F. Toro, "Riemann Solvers and
Numerical Methods for Fluid Dynamics", ch. 4): the star pressure is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock (Rankine-Hugoniot)
branch for p > p_K and the rarefaction (isentropic) branch otherwise, found by
Newton iteration; the solution is then sampled along x/t.  Used only as a pin
of the CPU reference; it is itself pinned in the tests by the jump conditions.
"""
import math

import numpy as np


def _fK(p, rho, pK, g):
    c = math.sqrt(g * pK / rho)
    if p > pK:
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        s = math.sqrt(A / (p + B))
        f = (p - pK) * s
        df = s * (1.0 - 0.5 * (p - pK) / (p + B))
    else:
        r = p / pK
        f = 2.0 * c / (g - 1.0) * (r ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * c) * r ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(L, R, g=1.4, tol=1e-15, itmax=100):
    """L, R = (rho, u, p).  Returns p*, u*, rho*_L, rho*_R."""
    rl, ul, pl = L
    rr, ur, pr = R
    p = max(1e-12, 0.5 * (pl + pr))
    for _ in range(itmax):
        fl, dfl = _fK(p, rl, pl, g)
        fr, dfr = _fK(p, rr, pr, g)
        f = fl + fr + (ur - ul)
        pn = p - f / (dfl + dfr)
        pn = max(pn, 1e-14)
        if abs(pn - p) <= tol * 0.5 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _fK(p, rl, pl, g)
    fr, _ = _fK(p, rr, pr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)

    def rho_star(rho, pK):
        if p > pK:
            q = (g - 1.0) / (g + 1.0)
            return rho * (p / pK + q) / (q * p / pK + 1.0)
        return rho * (p / pK) ** (1.0 / g)

    return p, u, rho_star(rl, pl), rho_star(rr, pr)


def sample(L, R, xi, g=1.4):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    rl, ul, pl = L
    rr, ur, pr = R
    ps, us, rsl, rsr = star_state(L, R, g)
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi.ravel()):
        if s <= us:  # left of the contact
            if ps > pl:  # left shock
                S = ul - cl * math.sqrt((g + 1) / (2 * g) * ps / pl + (g - 1) / (2 * g))
                val = (rl, ul, pl) if s <= S else (rsl, us, ps)
            else:  # left rarefaction
                csl = cl * (ps / pl) ** ((g - 1) / (2 * g))
                head, tail = ul - cl, us - csl
                if s <= head:
                    val = (rl, ul, pl)
                elif s >= tail:
                    val = (rsl, us, ps)
                else:
                    uu = 2.0 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    cc = 2.0 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    rr_ = rl * (cc / cl) ** (2 / (g - 1))
                    val = (rr_, uu, pl * (cc / cl) ** (2 * g / (g - 1)))
        else:
            if ps > pr:  # right shock
                S = ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
                val = (rr, ur, pr) if s >= S else (rsr, us, ps)
            else:
                csr = cr * (ps / pr) ** ((g - 1) / (2 * g))
                head, tail = ur + cr, us + csr
                if s >= head:
                    val = (rr, ur, pr)
                elif s <= tail:
                    val = (rsr, us, ps)
                else:
                    uu = 2.0 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    cc = 2.0 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    rr_ = rr * (cc / cr) ** (2 / (g - 1))
                    val = (rr_, uu, pr * (cc / cr) ** (2 * g / (g - 1)))
        rho.flat[n], u.flat[n], p.flat[n] = val
    return rho, u, p


def right_shock_speed(L, R, g=1.4):
    ps, us, rsl, rsr = star_state(L, R, g)
    rr, ur, pr = R
    cr = math.sqrt(g * pr / rr)
    return ur + cr * math.sqrt((g + 1) / (2 * g) * ps / pr + (g - 1) / (2 * g))
