"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds no arithmetic of the collision operator: it only draws
momentum grids, initial distributions and per-solve parameters from a seeded
generator (numpy PCG64), so that the oracle and the library see bit-identical
inputs.  The workload shapes follow the paper's own inputs:

* log-spaced momentum grids (Sec. 4.1, "logarithmic grid q_i in [q_min, q_max]");
* two log-normal bumps in momentum, the shape of the paper's validation input
  (Sec. 5, eq. benchmark_two_bump);
* Maxwell-Boltzmann shapes z*exp(-E/T), the thermal fixed point discussed in
  App. B (eq. app_log_interp) and App. C.

Draw order per solve is fixed: lambda, p_low, p_high, ratio, then (serving
only) N, t_end, inter-arrival time.  The default seed is 20261202.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

DEFAULT_SEED = 20261202


def rng(seed: int = DEFAULT_SEED) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def log_grid(n: int, pmin: float, pmax: float) -> np.ndarray:
    """n log-spaced momenta, endpoints included (the paper's log grid)."""
    if n < 2:
        raise ValueError("need at least two grid points")
    return np.exp(np.linspace(np.log(pmin), np.log(pmax), n))


def bump_pair(p: np.ndarray, p1: float, p2: float, a1: float, a2: float,
              w1: float, w2: float) -> np.ndarray:
    """Sum of two log-normal bumps, a_k*exp(-ln^2(p/p_k)/(2 w_k^2))."""
    l1 = np.log(p / p1)
    l2 = np.log(p / p2)
    return a1 * np.exp(-l1 * l1 / (2.0 * w1 * w1)) + a2 * np.exp(-l2 * l2 / (2.0 * w2 * w2))


def two_bump_benchmark(q: np.ndarray) -> np.ndarray:
    """The paper's validation input (Sec. 5, eq. benchmark_two_bump)."""
    return bump_pair(q, 0.3, 8.0, 1.0, 0.5, 0.18, 0.22)


def maxwell_boltzmann(p: np.ndarray, mass: float, temp: float, z: float = 1.0) -> np.ndarray:
    """z*exp(-E/T) with E = sqrt(p^2 + m^2) (thermal shape of App. B/C)."""
    return z * np.exp(-np.sqrt(p * p + mass * mass) / temp)


@dataclass
class Solve:
    """One solve of a parameter scan: coupling, bump positions, ratio."""
    lam: float
    p_low: float
    p_high: float
    ratio: float
    n: int = 0
    t_end: float = 0.0
    arrival: float = 0.0

    def f0(self, p: np.ndarray, width: float = 0.3) -> np.ndarray:
        return bump_pair(p, self.p_low, self.p_high, 1.0, self.ratio, width, width)


def _loguniform(g: np.random.Generator, lo: float, hi: float) -> float:
    return float(np.exp(g.uniform(np.log(lo), np.log(hi))))


def draw_solves(count: int, lam_range=(1e-3, 1e3), low_range=(0.05, 0.5),
                high_range=(1.0, 5.0), ratio_range=(0.1, 10.0),
                seed: int = DEFAULT_SEED) -> List[Solve]:
    """Batched-evaluation workload: lambda log-uniform, bump positions
    log-uniform in the two ranges, amplitude ratio uniform."""
    g = rng(seed)
    out = []
    for _ in range(count):
        lam = _loguniform(g, *lam_range)
        pl = _loguniform(g, *low_range)
        ph = _loguniform(g, *high_range)
        ratio = float(g.uniform(*ratio_range))
        out.append(Solve(lam, pl, ph, ratio))
    return out


# --- the five workloads -----------------------------------------------------

@dataclass
class Workload:
    name: str
    n: int
    pmin: float
    pmax: float
    batch: int
    solves: List[Solve] = field(default_factory=list)

    def grid(self) -> np.ndarray:
        return log_grid(self.n, self.pmin, self.pmax)

    def f0(self, count: Optional[int] = None) -> np.ndarray:
        p = self.grid()
        sel = self.solves if count is None else self.solves[:count]
        return np.stack([s.f0(p) for s in sel])


def single_fp64_n32() -> Workload:
    """FP64 single distribution, N=32 on p/m in [1e-2, 10]; bumps at 0.1 and
    2.0 (width 0.3 in ln p), amplitudes 1 : 0.5, lambda = 1."""
    return Workload("single_fp64_n32", 32, 1e-2, 10.0, 1,
                    [Solve(1.0, 0.1, 2.0, 0.5)])


def single_fp32_n128(seed: int = DEFAULT_SEED) -> Workload:
    """FP32 single distribution with radiation-era drift, N=128 on
    p/m in [1e-3, 20], lambda log-uniform in [1e-2, 1e2]."""
    s = draw_solves(1, lam_range=(1e-2, 1e2), seed=seed)
    return Workload("single_fp32_n128_drift", 128, 1e-3, 20.0, 1, s)


def batched_fp32_n256(batch: int = 512, seed: int = DEFAULT_SEED) -> Workload:
    """Batched evaluation, N=256 on p/m in [1e-3, 20], lambda log-uniform in
    [1e-3, 1e3]."""
    return Workload("batched_fp32_n256_b%d" % batch, 256, 1e-3, 20.0, batch,
                    draw_solves(batch, seed=seed))


def mixed_n256(batch: int = 4096, seed: int = DEFAULT_SEED) -> Workload:
    """Mixed-precision batch, N=256, B=4096, same draws as the FP32 batch."""
    return Workload("mixed_n256_b%d" % batch, 256, 1e-3, 20.0, batch,
                    draw_solves(batch, seed=seed))


SERVING_NS = (64, 128, 256, 384)
SERVING_WEIGHTS = (0.4, 0.3, 0.2, 0.1)
SERVING_PMIN, SERVING_PMAX = 1e-4, 20.0


def serving_requests(count: int, rate: float = 200.0, seed: int = DEFAULT_SEED,
                     t_end_range=(1e2, 1e4)) -> List[Solve]:
    """Poisson arrivals of parameter-scan solves: lambda log-uniform
    [1e-3, 1e3], N from {64,128,256,384} with weights 0.4/0.3/0.2/0.1,
    end time uniform in [1e2, 1e4] Hubble units, exponential inter-arrival
    times at `rate` per second."""
    g = rng(seed)
    t = 0.0
    out = []
    cum = np.cumsum(SERVING_WEIGHTS)
    for _ in range(count):
        lam = _loguniform(g, 1e-3, 1e3)
        pl = _loguniform(g, 0.05, 0.5)
        ph = _loguniform(g, 1.0, 5.0)
        ratio = float(g.uniform(0.1, 10.0))
        k = int(np.searchsorted(cum, g.uniform(0.0, 1.0), side="right"))
        n = SERVING_NS[min(k, len(SERVING_NS) - 1)]
        t_end = float(g.uniform(*t_end_range))
        t += float(g.exponential(1.0 / rate))
        out.append(Solve(lam, pl, ph, ratio, n=n, t_end=t_end, arrival=t))
    return out
