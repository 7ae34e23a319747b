"""Pins of the oracle's correlation function (Sec. 4: G(r) = <S_i^x S_{i+r}^x +
S_i^y S_{i+r}^y> of the clock model, at r = L/4 and L/2, and their ratio R).

The counts histogram (s_{i+r} - s_i) mod q over both lattice directions; G is
their cos-weighted mean.  Pinned by the definition written with the spin
vectors themselves, by the nearest-neighbour pair counts (r = 1 is the same set
of pairs, counted by another function), by closed forms for uniform and
striped states, and by the mirror symmetry r <-> L - r."""
import math

import numpy as np
import pytest


def _random_state(L, q, seed):
    return np.random.default_rng(seed).integers(0, q, size=(L, L)).astype(np.int8)


@pytest.mark.parametrize("L,q", [(5, 6), (12, 6), (13, 3), (16, 4), (9, 32), (6, 2)])
def test_r1_equals_pair_counts(orc, L, q):
    s = _random_state(L, q, 100 + L)
    ch = orc.Chain(L, q, "clock", T=1.0, spins=s)
    _, pair = ch.counts()
    assert np.array_equal(orc.corr_counts(L, q, s, 1), pair)


@pytest.mark.parametrize("L,q,r", [(8, 6, 2), (12, 6, 3), (12, 6, 6), (11, 5, 2), (7, 32, 3), (10, 4, 0)])
def test_g_equals_vector_definition(orc, L, q, r):
    # G written out with the spin vectors S = (cos theta, sin theta), theta = 2 pi s / q
    s = _random_state(L, q, 7 * L + r)
    th = 2.0 * math.pi * s.astype(np.float64) / q
    sx, sy = np.cos(th), np.sin(th)
    g = 0.0
    for axis in (1, 0):
        tx, ty = np.roll(sx, -r, axis=axis), np.roll(sy, -r, axis=axis)
        g += float(np.sum(sx * tx + sy * ty))
    g /= 2.0 * L * L
    h = orc.corr_counts(L, q, s, r)
    assert int(h.sum()) == 2 * L * L
    assert abs(orc.corr_g(L, q, h) - g) < 1e-12


@pytest.mark.parametrize("q", [2, 3, 6, 8])
def test_uniform_and_striped_states(orc, q):
    L = 4 * q
    # uniform state: every pair has difference 0 and G = 1
    s = np.full((L, L), q - 1, np.int8)
    h = orc.corr_counts(L, q, s, L // 4)
    assert h[0] == 2 * L * L and h[1:].sum() == 0
    assert orc.corr_g(L, q, h) == 1.0
    # stripes s = x mod q: along x every pair differs by r mod q, along y by 0
    s = np.tile(np.arange(L) % q, (L, 1)).astype(np.int8)
    for r in (L // 4, L // 2, 1, 3):
        h = orc.corr_counts(L, q, s, r)
        want = np.zeros(q, np.int64)
        want[0] += L * L
        want[r % q] += L * L
        assert np.array_equal(h, want), r
        assert abs(orc.corr_g(L, q, h) - 0.5 * (1.0 + math.cos(2.0 * math.pi * r / q))) < 1e-12


@pytest.mark.parametrize("L,q,r", [(10, 6, 3), (9, 4, 2), (12, 32, 5)])
def test_mirror_symmetry(orc, L, q, r):
    # the pairs at distance L - r are those at distance r, taken the other way
    s = _random_state(L, q, 3 * L)
    h = orc.corr_counts(L, q, s, r)
    hm = orc.corr_counts(L, q, s, L - r)
    assert np.array_equal(hm, h[(-np.arange(q)) % q])


def test_chain_corr_counts_use_quarter_and_half(orc):
    L, q = 20, 6
    ch = orc.Chain(L, q, "clock", T=0.9, seed=4).sweep(3)
    c1, c2 = ch.corr_counts()
    assert np.array_equal(c1, orc.corr_counts(L, q, ch.spins, 5))
    assert np.array_equal(c2, orc.corr_counts(L, q, ch.spins, 10))
