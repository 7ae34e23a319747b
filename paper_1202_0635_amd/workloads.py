"""Seeded synthetic workloads: the lattice configurations the benchmarks and
tests run, and seeded random spin states.

This module holds none of the method's arithmetic; it only names parameters
(sizes, temperatures, seeds, mixes) and draws arbitrary starting states with
numpy, so both the GPU library and the CPU oracle can be fed the same input.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

TC_POTTS = {q: 1.0 / math.log(1.0 + math.sqrt(q)) for q in (2, 3, 4)}
T_CLOCK6 = 0.9  # upper KT temperature of the q = 6 clock model quoted in Sec. 4


@dataclass(frozen=True)
class LatticeConfig:
    name: str
    L: int
    q: int
    model: str
    T: float
    J: float = 1.0
    seed: int = 0
    therm: int = 0
    sweeps: int = 0


# Ising (q = 2 Potts) at T_c, L = 64, 1000 sweeps from the random start.
ISING_L64 = LatticeConfig("potts2_L64_Tc", 64, 2, "potts", TC_POTTS[2], seed=1, therm=0, sweeps=1000)
# Ising at T_c, L = 4096: 200 thermalisation + 1000 timed sweeps (Table 1, L = 4096 column).
ISING_L4096 = LatticeConfig("potts2_L4096_Tc", 4096, 2, "potts", TC_POTTS[2], seed=2, therm=200, sweeps=1000)
# q = 6 clock at T = 0.9, L = 4096 (Table 3, L = 4096 column).
CLOCK6_L4096 = LatticeConfig("clock6_L4096_T0.9", 4096, 6, "clock", T_CLOCK6, seed=3, therm=200, sweeps=1000)

CONFIGS = {c.name: c for c in (ISING_L64, ISING_L4096, CLOCK6_L4096)}


def replica_mix_q3(n: int = 256):
    """n q = 3 Potts replicas: L cycling over {64, 128, 256, 512}, T spread
    linearly over [0.9, 1.1] T_c, seeds 0x4000 + r."""
    sizes = (64, 128, 256, 512)
    tc = TC_POTTS[3]
    return [LatticeConfig(f"rep{r}", sizes[r % 4], 3, "potts", tc * (0.9 + 0.2 * r / max(1, n - 1)),
                          seed=0x4000 + r, sweeps=500) for r in range(n)]


def request_trace(n: int = 2000, seed: int = 20120203):
    """Serving trace: L log-uniform in [128, 2048], model/q uniform over
    {Potts 2, 3, 4; clock 6}, T uniform in [0.8, 1.2] T_c(q), sweeps uniform in
    [100, 1000], per-request seeds 0x50000 + i.  Arrival times are assigned by
    the caller from a Poisson rate."""
    rng = np.random.default_rng(seed)
    kinds = [("potts", 2), ("potts", 3), ("potts", 4), ("clock", 6)]
    out = []
    for i in range(n):
        L = int(math.floor(128 * 16 ** rng.random()))
        model, q = kinds[int(rng.integers(0, 4))]
        tc = TC_POTTS[q] if model == "potts" else T_CLOCK6
        T = tc * (0.8 + 0.4 * rng.random())
        sweeps = int(rng.integers(100, 1001))
        out.append(LatticeConfig(f"req{i}", L, q, model, T, seed=0x50000 + i, sweeps=sweeps))
    return out


def random_spins(L: int, q: int, seed: int) -> np.ndarray:
    """An arbitrary (not Philox) starting state for tests, values in [0, q)."""
    return np.random.default_rng(seed).integers(0, q, size=(L, L), dtype=np.int8)


def striped_spins(L: int, q: int, width: int = 3) -> np.ndarray:
    """Horizontal stripes of equal spins (long wrapped clusters at low T)."""
    rows = (np.arange(L) // width) % q
    return np.repeat(rows[:, None], L, axis=1).astype(np.int8)
