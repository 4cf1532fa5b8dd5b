"""Error metrics of the GPU path against the CPU reference.

U: e = max_v max_cells |dU_v| / s_v  (relative per variable, the worst
   variable), s_v = max_cells |U_v| for rho and rho e_t and the largest
   momentum magnitude max_cells |rho u| for each momentum component.  The paper compares the solutions of its CPU and GPU runs
   to a relative difference below 1e-12 (Sec. 8); the same bound is used here.
R: the residual is a sum of face fluxes that largely cancel, so its round-off
   is relative to the size of those fluxes, not to R itself:
   e_R = max_v max_cells |dR_v| / max_cells (sum over faces |F_v| ds).
"""
import numpy as np

FP64_TOL = 1e-12
FP32_STEP_TOL = 1e-5
FP32_RUN_TOL = 1e-4


def per_var(flat, case):
    """Split a flat [block][var][k][j][i] array into nv arrays (all blocks)."""
    nv = case.nv
    parts = [[] for _ in range(nv)]
    o = 0
    for b in case.blocks:
        n = b.ncells
        for v in range(nv):
            parts[v].append(np.asarray(flat[o:o + n]))
            o += n
    return [np.concatenate(p) for p in parts]


def state_scales(case, Uo):
    """Scale of each variable: max |rho| and max |rho e_t| for the scalars, and
    for every momentum component the largest momentum magnitude |rho u| (a
    component that is zero everywhere, e.g. rho v of a flow along x, would
    otherwise turn round-off into an O(1) relative error)."""
    o = per_var(Uo, case)
    nd = case.ndim
    mom = np.sqrt(sum(o[1 + a] ** 2 for a in range(nd)))
    sc = [np.max(np.abs(o[0]))] + [np.max(mom)] * nd + [np.max(np.abs(o[nd + 1]))]
    return [max(s, 1e-300) for s in sc]


def state_err(case, Ug, Uo):
    g, o = per_var(Ug, case), per_var(Uo, case)
    sc = state_scales(case, Uo)
    return max(float(np.max(np.abs(gv - ov)) / s) for gv, ov, s in zip(g, o, sc))


def component_errs(case, Ug, Uo):
    """Per-variable errors, each relative to that variable's own max |U_v|,
    reported beside state_err.  A momentum component whose own maximum is
    below 1e-6 of the largest momentum magnitude (zero up to round-off, e.g.
    the transverse momentum of a flow along x) has no scale of its own: it is
    reported as "abs=" its absolute error."""
    g, o = per_var(Ug, case), per_var(Uo, case)
    nd = case.ndim
    mom = float(np.max(np.sqrt(sum(o[1 + a] ** 2 for a in range(nd)))))
    out = []
    for v, (gv, ov) in enumerate(zip(g, o)):
        s = float(np.max(np.abs(ov)))
        d = float(np.max(np.abs(gv - ov)))
        if 1 <= v <= nd and s < 1e-6 * mom:
            out.append(f"abs={d:.2e}")
        else:
            out.append(f"{d / s:.2e}" if s > 0 else f"abs={d:.2e}")
    return out


def residual_err(case, Rg, Ro, scale):
    g, o, s = per_var(Rg, case), per_var(Ro, case), per_var(scale, case)
    return max(float(np.max(np.abs(gv - ov)) / np.max(sv)) for gv, ov, sv in zip(g, o, s))


def cell_volumes(case, ref=None):
    """Cell volumes in the state order of one variable (all blocks); 3D
    curvilinear blocks take theirs from the oracle grid ref."""
    out = []
    for n, b in enumerate(case.blocks):
        if case.ndim == 3 and getattr(b, "z", None) is not None:
            out.append(ref.metrics_3d(n)[1].ravel())
        elif b.x is not None:
            X, Y = b.x, b.y
            a = (X[1:, 1:] - X[:-1, :-1]) * (Y[1:, :-1] - Y[:-1, 1:])
            c = (X[1:, :-1] - X[:-1, 1:]) * (Y[1:, 1:] - Y[:-1, :-1])
            out.append((0.5 * (a - c)).ravel())
        else:
            v = b.h[0] * b.h[1] * (b.h[2] if case.ndim == 3 else 1.0)
            out.append(np.full(b.ncells, v))
    return np.concatenate(out)


# every measured error of the GPU tests, written out at the end of the session
REPORT = []


def report(test, msg):
    REPORT.append(f"{test}: {msg}")
