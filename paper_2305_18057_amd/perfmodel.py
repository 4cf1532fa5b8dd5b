"""The performance model of CPU-GPU heterogeneous computing (Sec. 6).

Times per iteration (one step) of a domain of N_l x N_w x N_d interior cells:

  Eq. (sequential): one CPU,
      N_l N_w N_d t_I + (2 N_l N_w + 2 N_l N_d + 2 N_w N_d) t_B
      + t_DH + t_HH + t_HD + 5 t_S
  Eq. (cpu): C CPUs, 2D, 1D decomposition along N_l,
      N_l N_w / C t_I + (2 N_w + 2 N_l / C) t_B + t_DH + t_HH + t_HD + 5 t_S
  Eq. (gpu): G GPUs, each r_gc times one CPU,
      N_l N_w / (G r_gc) t_I + (2 N_w + 2 N_l / (G r_gc)) t_B + ...
  Eq. (hete): G GPUs and C CPUs together,
      N_l N_w / (G r_gc + C) t_I + (2 N_w + 2 N_l / (G r_gc + C)) t_B + ...
  Eq. (alpha): transfers and synchronizations t_f = alpha T_b, T_b the
      boundary-enforcement time,
      N_l N_w / (G r_gc + C) t_I + (2 N_w + 2 N_l / (G r_gc + C)) t_B (1 + alpha)
  Eq. (beta): t_B = beta t_I,
      [N_l N_w / (G r_gc + C) + (2 N_w + 2 N_l / (G r_gc + C)) (1 + alpha) beta] t_I

t_I and t_B are one CPU's times per interior and per boundary cell.  The
paper's Eq. (cpu) is printed with the name time_gpu; it is the C-CPU time.

For a workload ratio r that is not the balance point (the paper sweeps r,
the cells of one GPU over the cells of one CPU), each worker's interior part
takes its own time and the slower one sets the pace:

  time_ratio(r) = max(r n_c t_I / r_gc, n_c t_I)
                  + (2 N_w + 2 N_l / (G r + C)) (1 + alpha) beta t_I,
  n_c = N_l N_w / (G r + C)  (cells of one CPU worker),

which is Eq. (beta) at r = r_gc.  This is the reading the measured ratio
sweeps are compared with; t_I there is the rate of one worker as the C
workers run together (worker_tI), and r_gc the GPU's speed over it.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Iterable, Sequence

import numpy as np


def time_seq(Nl, Nw, Nd, tI, tB, tDH=0.0, tHH=0.0, tHD=0.0, tS=0.0):
    """Eq. (sequential)."""
    return Nl * Nw * Nd * tI + (2 * Nl * Nw + 2 * Nl * Nd + 2 * Nw * Nd) * tB + tDH + tHH + tHD + 5 * tS


def time_cpu(Nl, Nw, C, tI, tB, tDH=0.0, tHH=0.0, tHD=0.0, tS=0.0):
    """Eq. (cpu): C CPU workers, 1D decomposition along N_l."""
    return Nl * Nw / C * tI + (2 * Nw + 2 * Nl / C) * tB + tDH + tHH + tHD + 5 * tS


def time_gpu(Nl, Nw, G, r_gc, tI, tB, tDH=0.0, tHH=0.0, tHD=0.0, tS=0.0):
    """Eq. (gpu): G GPUs, each r_gc times as fast as one CPU."""
    w = G * r_gc
    return Nl * Nw / w * tI + (2 * Nw + 2 * Nl / w) * tB + tDH + tHH + tHD + 5 * tS


def time_hete(Nl, Nw, G, C, r_gc, tI, tB, tDH=0.0, tHH=0.0, tHD=0.0, tS=0.0):
    """Eq. (hete): G GPUs and C CPUs share the domain."""
    w = G * r_gc + C
    return Nl * Nw / w * tI + (2 * Nw + 2 * Nl / w) * tB + tDH + tHH + tHD + 5 * tS


def boundary_cells(Nl, Nw, G, C, r):
    """The boundary-cell count of Eqs. (hete)-(beta) at workload ratio r."""
    return 2 * Nw + 2 * Nl / (G * r + C)


def time_alpha(Nl, Nw, G, C, r_gc, tI, tB, alpha):
    """Eq. (alpha): transfers and synchronizations as alpha times T_b."""
    w = G * r_gc + C
    return Nl * Nw / w * tI + boundary_cells(Nl, Nw, G, C, r_gc) * tB * (1 + alpha)


def time_beta(Nl, Nw, G, C, r_gc, tI, alpha, beta):
    """Eq. (beta): t_B = beta t_I."""
    w = G * r_gc + C
    return (Nl * Nw / w + boundary_cells(Nl, Nw, G, C, r_gc) * (1 + alpha) * beta) * tI


def time_ratio(Nl, Nw, G, C, r, r_gc, tI, kappa):
    """Time per step at workload ratio r (module docstring); kappa is the
    lumped boundary coefficient (1 + alpha) beta."""
    nc = Nl * Nw / (G * r + C)
    return max(r * nc * tI / r_gc, nc * tI) + boundary_cells(Nl, Nw, G, C, r) * kappa * tI


@dataclass
class Fit:
    tI: float        # one CPU's time per cell and step, s
    r_gc: float      # one GPU's speed over one CPU's
    kappa: float     # (1 + alpha) beta
    rms_rel: float   # RMS relative misfit over the sweep

    def alpha(self, beta: float) -> float:
        """alpha for an assumed beta (the paper quotes 0.2 .. 0.5)."""
        return self.kappa / beta - 1.0


def fit_kappa(Nl, Nw, G, C, ratios: Sequence[float], times: Sequence[float], r_gc: float,
              tI: float) -> Fit:
    """Least-squares kappa of time_ratio over measured (ratio, time) pairs,
    with t_I and r_gc from the pure-mode measurements.  time_ratio is linear
    in kappa: kappa = sum(b (T - a)) / sum(b^2) with a the interior part and
    b the boundary part per unit kappa."""
    a = np.array([time_ratio(Nl, Nw, G, C, r, r_gc, tI, 0.0) for r in ratios])
    b = np.array([boundary_cells(Nl, Nw, G, C, r) * tI for r in ratios])
    T = np.asarray(times, dtype=np.float64)
    kappa = float(np.dot(b, T - a) / np.dot(b, b))
    pred = a + kappa * b
    rms = float(np.sqrt(np.mean(((pred - T) / T) ** 2)))
    return Fit(tI=tI, r_gc=r_gc, kappa=kappa, rms_rel=rms)


def worker_tI(cells_per_worker: Sequence[float], host_times: Sequence[float]):
    """t_I of one CPU worker as the C workers run together, and the pool's
    fixed time per step: the least-squares line of the host part's time per
    step over its cells per worker (slope, intercept).  The model gives each
    of its C CPUs the rate t_I, so this is the rate it takes on a host whose
    workers do not keep one core's speed when they run together."""
    slope, icpt = np.polyfit(np.asarray(cells_per_worker, dtype=np.float64),
                             np.asarray(host_times, dtype=np.float64), 1)
    return float(slope), float(icpt)


def best_ratio(Nl, Nw, G, C, r_gc, tI, kappa, ratios: Iterable[float]):
    """The ratio of the given ones with the smallest predicted time."""
    return min(ratios, key=lambda r: time_ratio(Nl, Nw, G, C, r, r_gc, tI, kappa))
