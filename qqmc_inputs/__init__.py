"""Seeded synthetic inputs shared by the oracle side and the GPU side.

This module holds no arithmetic of the method: it only draws the random
numbers the method consumes (the Korobov lattice multiplier and the random
shifts of randomised QMC) and spells out the workloads (dot parameters,
orders, lattice sizes, shift counts).  Both the oracle and the GPU library
receive these numbers as plain inputs.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), implemented here from its
published definition.
"""
from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64: a 64-bit state advanced by the golden-ratio increment and
    passed through a two-multiply finaliser."""

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """A double in [0, 1) with 53 random bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)

    def uniform_int(self, lo: int, hi: int) -> int:
        """An integer in [lo, hi] (modulo bias is irrelevant at these ranges)."""
        return lo + self.next_u64() % (hi - lo + 1)


def lattice_multiplier(rng: SplitMix64, log2_n: int) -> int:
    """Odd Korobov multiplier a in [3, N) for N = 2^log2_n."""
    half = 1 << (log2_n - 1)
    while True:
        a = 2 * (rng.next_u64() % half) + 1
        if a != 1:
            return a


def shifts(rng: SplitMix64, n_shifts: int, order: int) -> np.ndarray:
    """n_shifts x order uniform shifts in [0, 1), row-major."""
    out = np.empty((n_shifts, order), dtype=np.float64)
    for s in range(n_shifts):
        for j in range(order):
            out[s, j] = rng.uniform()
    return out


@dataclass
class Dot:
    """Anderson dot: level eps_d, coupling Gamma, inverse temperature beta,
    symmetric bias V, measurement time t, table grid; half_bandwidth D of
    semicircular leads (0: wide band); lead 1 or 2 also tabulates that lead's
    dot-lead functions for the current (0: none)."""
    eps_d: float = 0.0
    gamma: float = 1.0
    beta: float = 20.0
    bias_v: float = 0.0
    t_meas: float = 10.0
    n_grid: int = 8192
    t_half: float = 10.0
    half_bandwidth: float = 0.0
    lead: int = 0


@dataclass
class OrderJob:
    """One (parameter point, order) integration: N = 2^log2_n lattice points,
    the lattice multiplier, K random shifts, the model-function tau, and the
    interaction shift alpha (drawn from no random stream)."""
    order: int
    log2_n: int
    lattice_a: int
    shifts: np.ndarray
    model_tau: float = 1.0
    mode: int = 0
    alpha: float = 0.0
    sobol_v: Optional[np.ndarray] = None       # (order, 32) uint32, or None
    sobol_shifts: Optional[np.ndarray] = None  # (n_shifts, order) uint32


def order_job(seed: int, order: int, log2_n: int, n_shifts: int,
              model_tau: float = 1.0, mode: int = 0, alpha: float = 0.0) -> OrderJob:
    """Draw the multiplier, then the shifts, from one SplitMix64 stream whose
    seed mixes (seed, order) so that every order has its own stream."""
    rng = SplitMix64((seed * 1000003 + order) & _MASK)
    a = lattice_multiplier(rng, log2_n)
    sh = shifts(rng, n_shifts, order)
    return OrderJob(order, log2_n, a, sh, model_tau, mode, alpha)


def sobol_job(seed: int, order: int, log2_n: int, n_shifts: int, model_tau: float = 1.0,
              mode: int = 0, alpha: float = 0.0) -> OrderJob:
    """The first 2^log2_n Sobol' points (App. B) with n_shifts random digital
    shifts from one SplitMix64 stream seeded by (seed, order); direction
    numbers as derived in qqmc_inputs.sobol."""
    from . import sobol
    V = sobol.direction_numbers(order)
    ds = sobol.digital_shifts((seed * 1000003 + order + 77) & _MASK, n_shifts, order)
    return OrderJob(order, log2_n, 0, np.zeros((n_shifts, order)), model_tau, mode, alpha,
                    V, ds)


# ---------------------------------------------------------------------------
# Workloads.  The paper's own runs (Anderson dot benchmark, Coulomb-diamond
# sweep) are replaced by these synthetic wide-band dots.
# ---------------------------------------------------------------------------
TINY_DOT = Dot(eps_d=0.0, gamma=1.0, beta=20.0, bias_v=0.0)


def tiny_jobs(seed: int = 1) -> List[OrderJob]:
    """Orders 1..3, N = 2^14, 16 shifts, tau = 1."""
    return [order_job(seed, n, 14, 16) for n in (1, 2, 3)]


def plain_jobs(seed: int = 1, orders=range(1, 9)) -> List[OrderJob]:
    """Orders 1..8, N = 2^20, 32 shifts, tau = 1 (the n = 8 job is the
    throughput workload)."""
    return [order_job(seed, n, 20, 32) for n in orders]


STRESS_DOT = Dot(eps_d=-0.5, gamma=1.0, beta=20.0, bias_v=0.2)

# The paper's own benchmark configuration (main text, "Benchmark"): T = 0,
# eps_d = 0, wide band, Gamma = 1, measurement at t = 30, where the printed
# Bethe-ansatz coefficients apply; a finer grid on [-30, 30].
BETHE_DOT = Dot(eps_d=0.0, gamma=1.0, beta=float("inf"), bias_v=0.0, t_meas=30.0,
                n_grid=65536, t_half=30.0)


def stress_jobs(seed: int = 4, orders=range(11, 15)) -> List[OrderJob]:
    """Orders 11..14, N = 2^18, 16 shifts."""
    return [order_job(seed, n, 18, 16) for n in orders]


def batched_log2_n(order: int) -> int:
    """Uneven per-order sizes from 2^16 at n = 1 to 2^22 at n = 10."""
    return 16 + (2 * (order - 1)) // 3


def batched_dots(seed: int = 2, count: int = 64) -> List[Dot]:
    """64 parameter points: eps_d ~ U[-3, 3], V in {0, 0.5, 1},
    Gamma in {0.5, 1}, beta = 20."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        eps = -3.0 + 6.0 * rng.uniform()
        v = (0.0, 0.5, 1.0)[rng.next_u64() % 3]
        g = (0.5, 1.0)[rng.next_u64() % 2]
        out.append(Dot(eps_d=eps, gamma=g, beta=20.0, bias_v=v))
    return out


def batched_jobs(seed: int = 2, count: int = 64, orders=range(1, 11),
                 log2_offset: int = 0) -> List[Tuple[int, OrderJob]]:
    """(parameter index, job) for every parameter point and order."""
    out = []
    for p in range(count):
        for n in orders:
            out.append((p, order_job(seed * 7919 + p, n,
                                     batched_log2_n(n) - log2_offset, 16)))
    return out


@dataclass
class Request:
    arrival_s: float
    dot: Dot
    job: OrderJob


def serving_trace(seed: int = 3, n_requests: int = 512, rate_hz: float = 200.0,
                  k_min: int = 14, k_max: int = 22, n_min: int = 2,
                  n_max: int = 12) -> List[Request]:
    """Poisson arrivals of sweep requests: eps_d ~ U[-3, 3],
    Gamma ~ U[0.5, 2], V ~ U[0, 1], n ~ U{2..12}, N = 2^k with
    k ~ U{14..22}, 16 shifts, beta = 20, t = 10, tau = 1."""
    rng = SplitMix64(seed)
    t = 0.0
    out = []
    for r in range(n_requests):
        # exponential inter-arrival time by inversion of a uniform
        t += -np.log1p(-rng.uniform()) / rate_hz
        eps = -3.0 + 6.0 * rng.uniform()
        g = 0.5 + 1.5 * rng.uniform()
        v = rng.uniform()
        n = rng.uniform_int(n_min, n_max)
        k = rng.uniform_int(k_min, k_max)
        job = order_job(seed * 104729 + r, n, k, 16)
        out.append(Request(t, Dot(eps_d=eps, gamma=g, beta=20.0, bias_v=v), job))
    return out
