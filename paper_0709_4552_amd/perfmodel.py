"""The single-device performance model of section 4.1, recast for one GPU.

Section 4.1 writes the time to integrate one N-body time unit as a sum over
the block steps,

    T_integrate = sum_i ( t_pred + t_force + t_corr ),
    t_pred  = tau_pred  * N,
    t_force = tau_force * n * N,
    t_corr  = tau_corr  * n,

with n the block size of step i, and gives the constants of five hosts in its
Table 3; section 3.2 takes the block size as n = 0.20 N^0.81.  On the GPU each
block step also costs a fixed t0 (kernel launches and their latency), and
tau_force depends on n (small blocks fill the chip poorly), so the model here
is

    T = sum_i ( t0 + tau_pred N + tau_force(n_i) n_i N + tau_corr n_i ),

with tau_force(n) interpolated log-log between measured block sizes.  With
t0 = 0 and a constant tau_force it is the paper's equation exactly.

Pure Python and numpy; nothing here touches the GPU.  The measurements that
feed it come from `bench.py --perfmodel` (or the default benchmark run).
"""
from __future__ import annotations

import math
from typing import Callable, Dict, Iterable, Sequence, Tuple, Union

import numpy as np

# Table 3 of the paper: host -> (Whetstone Mflops, tau_pred, tau_force,
# tau_corr), the times in seconds (the table gives microseconds).
PAPER_TABLE3: Dict[str, Tuple[float, float, float, float]] = {
    "vader": (377.0, 0.247e-6, 0.216e-6, 4.81e-6),
    "palpatine": (422.0, 0.273e-6, 0.193e-6, 2.39e-6),
    "yoda": (436.0, 0.131e-6, 0.110e-6, 1.29e-6),
    "skywalker": (436.0, 0.131e-6, 0.110e-6, 1.29e-6),
    "obi-wan": (1191.0, 0.098e-6, 0.148e-6, 1.14e-6),
}

# GRAPE-6Af time per pairwise force (section 4.4)
TAU_GFORCE = 4.3e-10

TauForce = Union[float, Callable[[float], float]]


def block_size_paper(N: float) -> float:
    """Average block size of section 3.2: n = 0.20 N^0.81."""
    return 0.20 * float(N) ** 0.81


def _tau(tau_force: TauForce, n: float) -> float:
    return float(tau_force(n)) if callable(tau_force) else float(tau_force)


def t_step(N: float, n: float, tau_pred: float, tau_force: TauForce, tau_corr: float,
           t0: float = 0.0) -> float:
    """Time of one block step with n active particles out of N."""
    return t0 + tau_pred * N + _tau(tau_force, n) * n * N + tau_corr * n


def t_step_parts(N: float, n: float, tau_pred: float, tau_force: TauForce,
                 tau_corr: float) -> Dict[str, float]:
    """The three terms of one step separately (t_pred, t_force, t_corr)."""
    return {"t_pred": tau_pred * N, "t_force": _tau(tau_force, n) * n * N,
            "t_corr": tau_corr * n}


def T_integrate(N: float, sizes: Iterable[float], tau_pred: float, tau_force: TauForce,
                tau_corr: float, t0: float = 0.0) -> float:
    """Sum of t_step over the block sizes of a run (the section 4.1 sum)."""
    return float(sum(t_step(N, n, tau_pred, tau_force, tau_corr, t0) for n in sizes))


def T_integrate_mean(N: float, steps: int, n_mean: float, tau_pred: float,
                     tau_force: TauForce, tau_corr: float, t0: float = 0.0) -> float:
    """The same with every step at one (mean) block size."""
    return steps * t_step(N, n_mean, tau_pred, tau_force, tau_corr, t0)


def tau_force_table(points: Dict[int, float]) -> Callable[[float], float]:
    """tau_force(n) from measured (n, tau) pairs: log-log linear in between,
    the end values held beyond the measured range."""
    ns = np.array(sorted(points), dtype=np.float64)
    if ns.size == 0 or np.any(ns <= 0):
        raise ValueError("block sizes must be positive")
    lt = np.log(np.array([points[int(k)] for k in ns], dtype=np.float64))
    ln = np.log(ns)

    def tau(n: float) -> float:
        return float(np.exp(np.interp(math.log(max(float(n), 1.0)), ln, lt)))

    return tau


def fit_t0(T_measured: float, N: float, sizes: Sequence[float], tau_pred: float,
           tau_force: TauForce, tau_corr: float) -> float:
    """The fixed cost per step that makes the model match one measured run."""
    steps = len(sizes)
    if steps == 0:
        raise ValueError("no steps")
    rest = T_integrate(N, sizes, tau_pred, tau_force, tau_corr, 0.0)
    return (T_measured - rest) / steps


def paper_host_rate(host: str) -> float:
    """Pairwise force interactions per second of a Table 3 host."""
    return 1.0 / PAPER_TABLE3[host][2]
