"""Pins of the oracle's bond activation (Sec. 2 steps (i)-(iii)) and flip
(Sec. 2 steps (v)-(vii); Sec. 4 embedded cluster), by statistics and by the
special cases the method has."""
import math

import numpy as np
import pytest
from scipy import stats


def test_bond_frequency_equals_cutoff(orc):
    # Among equal-spin pairs the fraction of active bonds is c / 2^32
    # (binomial z-test); unequal pairs never bond (Potts).
    L, q = 256, 3
    T = 1.0 / math.log(1.0 + math.sqrt(3.0))
    ch = orc.Chain(L, q, "potts", T=T, seed=5)
    c = int(ch.table[0])
    n_eq = n_act = 0
    for _ in range(4):
        s = ch.spins.reshape(L, L).copy()
        ch.sweep(1)
        br = ch.bond_r.reshape(L, L).astype(bool)
        bd = ch.bond_d.reshape(L, L).astype(bool)
        eq_r = s == np.roll(s, -1, axis=1)
        eq_d = s == np.roll(s, -1, axis=0)
        assert not np.any(br & ~eq_r) and not np.any(bd & ~eq_d)
        n_eq += int(eq_r.sum() + eq_d.sum())
        n_act += int(br.sum() + bd.sum())
    p = c / 2**32
    z = (n_act - n_eq * p) / math.sqrt(n_eq * p * (1 - p))
    assert abs(z) < 4.5, z


def test_bonds_right_and_down_are_independent(orc):
    # The right and down bond of one site use different 32-bit uniforms: with
    # all spins equal, the joint frequency factorises.
    L, q = 128, 2
    T = 1.0 / math.log(2.0)  # p = 1/2
    tab = orc.cutoffs("potts", q, T, 1.0)
    s = np.zeros((L, L), np.int8)
    both = 0
    n = 0
    for t in range(8):
        br, bd = orc.bonds(L, q, "potts", tab, 3, t, s)
        both += int((br & bd).sum())
        n += L * L
    p = int(tab[0]) / 2**32
    z = (both - n * p * p) / math.sqrt(n * p * p * (1 - p * p))
    assert abs(z) < 4.5


def test_extreme_temperatures(orc):
    L, q = 32, 2
    s = orc.init(L, q, 1)
    hot = orc.cutoffs("potts", q, 1e12, 1.0)
    br, bd = orc.bonds(L, q, "potts", hot, 1, 0, s)
    assert br.sum() == 0 and bd.sum() == 0
    cold = orc.cutoffs("potts", q, 1e-3, 1.0)
    br, bd = orc.bonds(L, q, "potts", cold, 1, 0, s)
    assert np.array_equal(br.astype(bool), s == np.roll(s, -1, axis=1))
    assert np.array_equal(bd.astype(bool), s == np.roll(s, -1, axis=0))


@pytest.mark.parametrize("q", [2, 3, 4, 7])
def test_potts_new_values_uniform(orc, q):
    # Step (vi): every cluster takes one of the q values with probability 1/q,
    # the old value included.  With no bonds every site is its own cluster.
    L = 128
    tab = orc.cutoffs("potts", q, 1e12, 1.0)
    s = orc.init(L, q, 2)
    counts = np.zeros(q)
    kept = 0
    for t in range(6):
        br, bd = orc.bonds(L, q, "potts", tab, 2, t, s)
        lab = orc.label(L, br, bd)
        s2 = orc.flip(L, q, "potts", 2, t, lab, s)
        counts += np.bincount(s2.reshape(-1), minlength=q)
        kept += int((s2 == s).sum())
        s = s2
    chi2, pval = stats.chisquare(counts)
    assert pval > 1e-4
    n = 6 * L * L
    z = (kept - n / q) / math.sqrt(n * (1 / q) * (1 - 1 / q))
    assert abs(z) < 4.5


def test_two_outcome_draws_independent_within_and_across_groups(orc):
    # R6: a two-outcome cluster takes one bit of the draw of its 128-site
    # group.  Each cluster's outcome must be fair and independent of every
    # other cluster's: pairs of canonical labels in the same group (next
    # site, the same bit of the next word), across a group boundary and in
    # the same bit position of the next group give four equally likely joint
    # outcomes.  A shared bit, a single word or a shared draw per group would
    # fail one of them.
    base = 128 * np.arange(0, 4000, 7, dtype=np.int64)
    pairs = {"next site": (5, 6), "next word": (9, 41), "group boundary": (127, 128), "next group": (3, 131)}
    for name, (da, db) in pairs.items():
        joint = np.zeros(4)
        for t in range(8):
            roots = np.concatenate([base + da, base + db])
            out = orc.flip_at(2, "potts", 77, t, roots, np.zeros(roots.size, dtype=np.int8))
            a, b = out[: base.size].astype(int), out[base.size:].astype(int)
            joint += np.bincount(2 * a + b, minlength=4)
        chi2, pval = stats.chisquare(joint)
        assert pval > 1e-4, (name, joint)


def test_flip_is_constant_on_clusters(orc):
    L, q = 64, 3
    T = 1.0 / math.log(1.0 + math.sqrt(3.0))
    ch = orc.Chain(L, q, "potts", T=T, seed=9)
    ch.sweep(3)
    lab = ch.labels.reshape(-1)
    s = ch.spins.reshape(-1)
    for root in np.unique(lab):
        assert len(np.unique(s[lab == root])) == 1


def test_clock_flip_half_and_mirror_map(orc):
    L, q = 96, 6
    T = 0.9
    ch = orc.Chain(L, q, "clock", T=T, seed=4)
    ch.sweep(2)
    flipped = 0
    total = 0
    for _ in range(5):
        s_old = ch.spins.copy()
        t = ch.t
        m = orc.mirror(q, ch.seed, t)
        ch.sweep(1)
        lab = ch.labels
        s_new = ch.spins
        for root in np.unique(lab):
            mem = lab == root
            same = np.all(s_new[mem] == s_old[mem])
            refl = np.all(s_new[mem] == (m - s_old[mem]) % q)
            assert same or refl
            if not np.all(s_old[mem] == (m - s_old[mem]) % q):  # reflection changes it
                total += 1
                flipped += int(refl)
    # clusters whose reflection changes them flip with probability 1/2
    z = (flipped - total / 2) / math.sqrt(total / 4)
    assert abs(z) < 4.5


def test_clock_bonds_only_for_positive_projection(orc):
    L, q = 64, 6
    tab = orc.cutoffs("clock", q, 0.01, 1.0)  # p ~ 1 for every P > 0
    s = orc.init(L, q, 8)
    for t in range(3):
        m = orc.mirror(q, 8, t)
        br, bd = orc.bonds(L, q, "clock", tab, 8, t, s)
        sr = np.roll(s, -1, axis=1)
        sd = np.roll(s, -1, axis=0)
        Pr = np.vectorize(lambda a, b: orc.clock_projection(q, int(a), int(b), m))(s, sr)
        Pd = np.vectorize(lambda a, b: orc.clock_projection(q, int(a), int(b), m))(s, sd)
        assert np.array_equal(br.astype(bool), Pr > 1e-12)
        assert np.array_equal(bd.astype(bool), Pd > 1e-12)


def test_mirror_uniform(orc):
    q = 6
    ms = [orc.mirror(q, 123, t) for t in range(6000)]
    chi2, pval = stats.chisquare(np.bincount(ms, minlength=q))
    assert pval > 1e-4


def test_random_start_uniform(orc):
    for q in (2, 3, 6):
        s = orc.init(200, q, 77)
        chi2, pval = stats.chisquare(np.bincount(s.reshape(-1), minlength=q))
        assert pval > 1e-4


def test_counts_and_energy_identities(orc):
    L = 37
    for q, model in [(2, "potts"), (3, "potts"), (6, "clock")]:
        ch = orc.Chain(L, q, model, T=1.0, seed=3)
        ch.sweep(2)
        h, p = ch.counts()
        assert h.sum() == L * L and p.sum() == 2 * L * L
        s = ch.spins.reshape(L, L).astype(np.int64)
        sr = np.roll(s, -1, axis=1)
        sd = np.roll(s, -1, axis=0)
        e, m2 = ch.observables()
        if model == "potts":
            # Eq. 1: H = -J sum (delta - 1)
            H = -1.0 * (((s == sr).astype(int) - 1).sum() + ((s == sd).astype(int) - 1).sum())
            n = np.bincount(s.reshape(-1), minlength=q)
            M2 = (q * (n.astype(float) ** 2).sum() - (L * L) ** 2) / (q - 1)
        else:
            th = 2 * np.pi * s / q
            H = -(np.cos(th - np.roll(th, -1, 1)).sum() + np.cos(th - np.roll(th, -1, 0)).sum())
            M2 = np.cos(th).sum() ** 2 + np.sin(th).sum() ** 2
        assert abs(e - H / (L * L)) < 1e-12
        assert abs(m2 - M2 / (L * L) ** 2) < 1e-12


@pytest.mark.parametrize("model,q,T", [("potts", 3, 0.9), ("clock", 6, 0.9), ("potts", 2, 1.1)])
def test_single_site_entry_points_match_whole_lattice(orc, model, q, T):
    # The single-site bond and flip entry points (used to check sampled sites
    # of lattices too large for a whole oracle sweep) give the whole-lattice
    # functions' results at every site of a ragged lattice, in shuffled order.
    L, seed, t = 37, 5, 3
    tab = orc.cutoffs(model, q, T)
    s = orc.init(L, q, seed)
    br, bd = orc.bonds(L, q, model, tab, seed, t, s)
    idx = np.random.default_rng(1).permutation(L * L)
    b2, d2 = orc.bonds_at(L, q, model, tab, seed, t, s, idx)
    assert np.array_equal(br.reshape(-1)[idx], b2) and np.array_equal(bd.reshape(-1)[idx], d2)
    lab = orc.label(L, br, bd).reshape(-1)
    f = orc.flip(L, q, model, seed, t, lab, s).reshape(-1)
    assert np.array_equal(f[idx], orc.flip_at(q, model, seed, t, lab[idx], s.reshape(-1)[idx]))
