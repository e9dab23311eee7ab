"""Seeded synthetic workloads (instance lists only; none of the sampler's
arithmetic lives here).  Shared by the tests, the benchmark and the oracle
comparisons so that both sides see the same Hamiltonian points.

Random draws use SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), so the
lists do not depend on any library's generator.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

MASK = (1 << 64) - 1


class SplitMix64:
    def __init__(self, seed: int):
        self.x = seed & MASK

    def next(self) -> int:
        self.x = (self.x + 0x9E3779B97F4A7C15) & MASK
        z = self.x
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        """Uniform in [0, 1) with 53 random bits."""
        return (self.next() >> 11) * (1.0 / (1 << 53))

    def normal(self) -> float:
        """Standard normal by Box-Muller."""
        u1 = max(self.uniform(), 1e-300)
        u2 = self.uniform()
        return math.sqrt(-2.0 * math.log(u1)) * math.cos(2.0 * math.pi * u2)


@dataclass
class Point:
    L: int
    J1: float
    J2: float
    h: float
    T0: float
    T1: float
    sched: str
    n_chains: int
    id: int


SEED_BATCHED = 0x5EED000000000003
SEED_SCALE = 0x5EED000000000005


def batched_uneven(n_instances: int = 2048, chains: int = 256, seed: int = SEED_BATCHED):
    """Uneven batch: L drawn from {6, 12, 18, 24, 36, 48}, J2/J1 ~ U[0.2, 2.5],
    h/J1 ~ U[0, 3], T ~ logU[0.05, 5] fixed per instance, `chains` chains each."""
    rng = SplitMix64(seed)
    sizes = (6, 12, 18, 24, 36, 48)
    out = []
    for k in range(n_instances):
        L = sizes[rng.next() % len(sizes)]
        J2 = 0.2 + 2.3 * rng.uniform()
        h = 3.0 * rng.uniform()
        T = math.exp(math.log(0.05) + (math.log(5.0) - math.log(0.05)) * rng.uniform())
        out.append(Point(L, 1.0, J2, h, T, T, "const", chains, k))
    return out


def scale_points(L: int, n_points: int = 64, chains: int = 512, seed: int = SEED_SCALE):
    """Points clustered near the T = 0 phase boundaries of the SS Ising model
    (J1 = 1): Neel|1/3 at h = 4 - 2 J2 (J2 in [0.3, 1.9]), 1/3|FM at h = 4 + J2
    (J2 in [0.3, 2.5]), dimer|1/3 at h = J2 - 2 (J2 in [2.1, 3]) and Neel|dimer at
    J2 = 2 (h in [0, 0.5]); each offset by N(0, 0.1) in h (or J2 for the last
    line); T ~ logU[0.1, 1]; one quarter of the points on each line."""
    rng = SplitMix64(seed ^ L)
    out = []
    per = n_points // 4
    for line in range(4):
        for q in range(per):
            u = (q + 0.5) / per
            if line == 0:
                J2 = 0.3 + 1.6 * u
                h = 4.0 - 2.0 * J2 + 0.1 * rng.normal()
            elif line == 1:
                J2 = 0.3 + 2.2 * u
                h = 4.0 + J2 + 0.1 * rng.normal()
            elif line == 2:
                J2 = 2.1 + 0.9 * u
                h = J2 - 2.0 + 0.1 * rng.normal()
            else:
                h = 0.5 * u
                J2 = 2.0 + 0.1 * rng.normal()
            T = math.exp(math.log(0.1) + (math.log(1.0) - math.log(0.1)) * rng.uniform())
            out.append(Point(L, 1.0, J2, h, T, T, "const", chains, len(out)))
    return out
