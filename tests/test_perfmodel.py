"""Pins of the Sec. 6 performance model against the relations the paper
states between its equations, and of the ratio form and its fit."""
import math

import numpy as np
import pytest

from paper_2305_18057_amd import perfmodel as PM

Nl, Nw = 2048, 256
tI, tB = 7e-7, 2.1e-7
x = dict(tDH=3e-6, tHH=1e-6, tHD=2e-6, tS=4e-6)


def test_sequential_counts_cells_and_faces():
    # a 1-cell domain: one interior cell and six boundary cells
    assert PM.time_seq(1, 1, 1, tI, tB) == pytest.approx(tI + 6 * tB)
    # 3D counting: N^3 interior and 6 N^2 boundary cells
    assert PM.time_seq(10, 10, 10, 1.0, 1.0) == 1000 + 600


def test_cpu_gpu_hete_reduce_to_each_other():
    # C = 0 CPUs: the heterogeneous time is the GPU time
    assert PM.time_hete(Nl, Nw, 2, 0, 40.0, tI, tB, **x) == pytest.approx(
        PM.time_gpu(Nl, Nw, 2, 40.0, tI, tB, **x))
    # G = 0 GPUs: the C-CPU time
    assert PM.time_hete(Nl, Nw, 0, 16, 40.0, tI, tB, **x) == pytest.approx(
        PM.time_cpu(Nl, Nw, 16, tI, tB, **x))
    # a GPU with r_gc = 1 counts as one more CPU
    assert PM.time_hete(Nl, Nw, 1, 7, 1.0, tI, tB) == pytest.approx(PM.time_cpu(Nl, Nw, 8, tI, tB))


def test_alpha_and_beta_substitutions():
    G, C, r = 1, 8, 40.0
    Tb = PM.boundary_cells(Nl, Nw, G, C, r) * tB
    alpha = (x["tDH"] + x["tHH"] + x["tHD"] + 5 * x["tS"]) / Tb
    # t_f = alpha T_b turns Eq. (hete) into Eq. (alpha)
    assert PM.time_alpha(Nl, Nw, G, C, r, tI, tB, alpha) == pytest.approx(
        PM.time_hete(Nl, Nw, G, C, r, tI, tB, **x))
    # t_B = beta t_I turns Eq. (alpha) into Eq. (beta)
    beta = tB / tI
    assert PM.time_beta(Nl, Nw, G, C, r, tI, alpha, beta) == pytest.approx(
        PM.time_alpha(Nl, Nw, G, C, r, tI, tB, alpha))


def test_ratio_form_is_eq_beta_at_balance_and_has_its_optimum_there():
    G, C, r_gc, alpha, beta = 1, 8, 45.0, 0.5, 0.3
    kappa = (1 + alpha) * beta
    assert PM.time_ratio(Nl, Nw, G, C, r_gc, r_gc, tI, kappa) == pytest.approx(
        PM.time_beta(Nl, Nw, G, C, r_gc, tI, alpha, beta))
    rs = np.linspace(5, 200, 400)
    T = [PM.time_ratio(Nl, Nw, G, C, r, r_gc, tI, kappa) for r in rs]
    assert abs(rs[int(np.argmin(T))] - r_gc) < 1.0
    # below the balance the CPU workers set the pace, above it the GPU
    assert PM.time_ratio(Nl, Nw, G, C, 10, r_gc, tI, 0.0) == pytest.approx(Nl * Nw / (10 + C) * tI)
    assert PM.time_ratio(Nl, Nw, G, C, 100, r_gc, tI, 0.0) == pytest.approx(
        100 * Nl * Nw / (100 + C) * tI / r_gc)


def test_fit_recovers_kappa():
    G, C, r_gc, kappa = 1, 16, 3000.0, 4.2
    rs = [200, 500, 1000, 2000, 4000, 8000]
    T = [PM.time_ratio(Nl, Nw, G, C, r, r_gc, tI, kappa) for r in rs]
    f = PM.fit_kappa(Nl, Nw, G, C, rs, T, r_gc, tI)
    assert f.kappa == pytest.approx(kappa, rel=1e-12)
    assert f.rms_rel < 1e-12
    assert f.alpha(0.3) == pytest.approx(kappa / 0.3 - 1)
    assert PM.best_ratio(Nl, Nw, G, C, r_gc, tI, kappa, rs) == rs[int(np.argmin(T))]
    # with no boundary cost the balance point wins
    assert PM.best_ratio(Nl, Nw, G, C, r_gc, tI, 0.0, rs + [r_gc]) == r_gc


def test_worker_rate_and_fit_from_a_sweep():
    """The bench's procedure on a sweep the model itself generates: the
    workers' t_I is the slope of the host time over cells per worker (a
    fixed pool cost is the intercept), and kappa comes back exactly."""
    C, tI_w, r_gc, kappa, fixed = 16, 7.9e-7, 5900.0, 0.49, 8.6e-5
    cols = [2, 4, 8, 16, 32, 64, 128]
    tI, icpt = PM.worker_tI([c * Nw / C for c in cols], [c * Nw / C * tI_w + fixed for c in cols])
    assert tI == pytest.approx(tI_w, rel=1e-12) and icpt == pytest.approx(fixed, rel=1e-9)
    ratios = [(Nl - c) * C / c for c in cols]
    T = [PM.time_ratio(Nl, Nw, 1, C, r, r_gc, tI_w, kappa) for r in ratios]
    f = PM.fit_kappa(Nl, Nw, 1, C, ratios, T, r_gc, tI)
    assert f.kappa == pytest.approx(kappa, rel=1e-9) and f.rms_rel < 1e-9
