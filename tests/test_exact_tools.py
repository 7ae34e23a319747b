"""The exact-result helpers that pin the oracle, pinned themselves.

Kaufman's finite-torus partition function (used for the exact Ising energy at
T_c that the oracle's chain must reproduce) is checked against brute-force
enumeration of the 4 x 4 torus (2^16 states), at several couplings; the
energy it gives is checked against the enumerated Potts energy.
"""
import itertools
import math

import numpy as np
import pytest

import exact_tools as et

TC2 = 1.0 / math.log(1.0 + math.sqrt(2.0))


def _ising_logz_enumerated(L, K):
    edges = et.torus_edges(L)
    a = np.array([i for i, _ in edges])
    b = np.array([j for _, j in edges])
    N = L * L
    idx = np.arange(2**N, dtype=np.int64)
    spins = 1 - 2 * ((idx[:, None] >> np.arange(N)[None, :]) & 1)  # +-1
    bond_sum = (spins[:, a] * spins[:, b]).sum(axis=1).astype(np.float64)
    x = K * bond_sum
    mx = x.max()
    return mx + math.log(np.exp(x - mx).sum())


@pytest.mark.parametrize("T", [0.8, TC2, 2.0])
def test_kaufman_logz_equals_enumeration_4x4(T):
    K = 1.0 / (2.0 * T)  # Potts J = 1 at temperature T is the Ising model with K = J / (2T)
    assert abs(et.kaufman_logz(4, K) - _ising_logz_enumerated(4, K)) < 1e-9


@pytest.mark.parametrize("T", [0.8, TC2, 2.0])
def test_kaufman_energy_equals_enumeration_4x4(T):
    e_enum, _, _ = et.exact_averages(4, 2, "potts", T)
    assert abs(et.ising_potts_energy(4, T) - e_enum) < 1e-8


def test_kaufman_logz_small_coupling_limit():
    # K -> 0: Z -> 2^N
    assert abs(et.kaufman_logz(4, 1e-7) - 16 * math.log(2.0)) < 1e-5
