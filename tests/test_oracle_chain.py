"""Whole-chain pins of the oracle against exact physics.

* Exact enumeration of the Boltzmann distribution on 3x3 and 4x4 tori: the
  oracle's Monte Carlo averages of E, M^2 and M^4 agree within statistical error.
* Detailed balance by brute force: the exact one-sweep SW kernel on the 2x2
  torus is reversible with respect to exp(-H/T) (Potts, Sec. 2; clock with the
  mirror reading of Sec. 4), while the other mirror reading is not; the
  oracle's empirical one-sweep transitions match the exact kernel (chi-square).
* The exact Ising energy: Kaufman's finite-torus value at T_c (Sec. 4 gives
  T_c = 1/ln(1+sqrt 2)) for L = 16, 32, 64, and the infinite-lattice value
  1 - 1/sqrt(2) as L grows.
"""
import math

import numpy as np
import pytest
from scipy import stats

import exact_tools as et

TC2 = 1.0 / math.log(1.0 + math.sqrt(2.0))
TC3 = 1.0 / math.log(1.0 + math.sqrt(3.0))


def _check_mc(orc, L, q, model, T, n_meas, seed, nsig=4.5):
    ex_e, ex_m2, ex_m4 = et.exact_averages(L, q, model, T)
    e, m2, _ = orc.run(L, q, model, T, 1.0, seed, 1000, n_meas)
    for name, series, exact in (("e", e, ex_e), ("m2", m2, ex_m2), ("m4", m2 * m2, ex_m4)):
        mean, err = et.binned_mean(series)
        assert abs(mean - exact) < nsig * err + 1e-9, (name, mean, exact, err)


@pytest.mark.parametrize(
    "q,model,T",
    [(2, "potts", TC2), (2, "potts", 0.7), (3, "potts", TC3), (4, "potts", 1.3),
     (6, "clock", 0.9), (6, "clock", 0.5), (4, "clock", 1.1), (3, "clock", 0.8)],
)
def test_enumeration_3x3(orc, q, model, T):
    _check_mc(orc, 3, q, model, T, 200_000, seed=1000 + q)


@pytest.mark.parametrize("q,model,T", [(2, "potts", TC2), (2, "clock", 1.5)])
def test_enumeration_4x4(orc, q, model, T):
    _check_mc(orc, 4, q, model, T, 200_000, seed=77)


def _potts_prob(orc, q, T):
    c = int(orc.cutoffs("potts", q, T, 1.0)[0])
    p = c / 2**32
    return (lambda a, b, m: p if a == b else 0.0), -math.log1p(-p)


def _clock_prob_from_table(orc, q, T):
    tab = orc.cutoffs("clock", q, T, 1.0).reshape(q, q, q)
    return lambda a, b, m: int(tab[m, a, b]) / 2**32


def _clock_prob_geometric(q, T, phi_of_m):
    def f(a, b, m):
        phi = phi_of_m(m)
        P = math.cos(2 * math.pi * a / q - phi) * math.cos(2 * math.pi * b / q - phi)
        return -math.expm1(-2 * P / T) if P > 1e-12 else 0.0

    return f


def _reversibility_defect(P, pi):
    F = pi[:, None] * P
    return np.abs(F - F.T).max() / pi.max()


@pytest.mark.parametrize("q,T", [(2, TC2), (3, TC3), (4, 0.8)])
def test_detailed_balance_potts_2x2(orc, q, T):
    prob, beta_eff = _potts_prob(orc, q, T)
    P = et.sw_transition_matrix(2, q, "potts", prob)
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-12)
    pi = et.boltzmann(2, q, "potts", 1.0 / beta_eff)
    assert _reversibility_defect(P, pi) < 1e-12
    assert np.allclose(pi @ P, pi, atol=1e-12)


@pytest.mark.parametrize("q,T", [(4, 0.9), (6, 0.9)])
def test_detailed_balance_clock_2x2_and_negative_control(q, T):
    good = et.sw_transition_matrix(2, q, "clock",
                                   _clock_prob_geometric(q, T, lambda m: math.pi * m / q + math.pi / 2))
    pi = et.boltzmann(2, q, "clock", T)
    assert np.allclose(good.sum(axis=1), 1.0, atol=1e-12)
    assert _reversibility_defect(good, pi) < 1e-10
    # the other reading of the mirror direction, phi = pi m / q, breaks detailed balance
    bad = et.sw_transition_matrix(2, q, "clock", _clock_prob_geometric(q, T, lambda m: math.pi * m / q))
    assert _reversibility_defect(bad, pi) > 1e-3


def _chi2_rows(orc, L, q, model, T, prob, rows, nseeds=60_000):
    P = et.sw_transition_matrix(L, q, model, prob)
    pw = q ** np.arange(L * L)
    for r, idx in enumerate(rows):
        s0 = ((idx // pw) % q).astype(np.int8)
        counts = orc.transition_counts(L, q, model, T, 1.0, s0, t=3 + r, seed0=1000 * (r + 1),
                                       nseeds=nseeds)
        expect = P[idx] * nseeds
        keep = expect > 5
        assert counts[~keep].sum() <= max(10, 3 * expect[~keep].sum() + 10)
        obs = counts[keep].astype(float)
        exp = expect[keep]
        exp *= obs.sum() / exp.sum()
        _, pval = stats.chisquare(obs, exp)
        assert pval > 1e-4, (idx, pval)


@pytest.mark.parametrize("q,T", [(2, TC2), (3, 0.8)])
def test_oracle_transitions_match_exact_kernel_potts(orc, q, T):
    prob, _ = _potts_prob(orc, q, T)
    n = q**4
    _chi2_rows(orc, 2, q, "potts", T, prob, rows=[0, 1, n // 3, n - 2])


def test_oracle_transitions_match_exact_kernel_clock(orc):
    q, T = 4, 0.9
    prob = _clock_prob_from_table(orc, q, T)
    _chi2_rows(orc, 2, q, "clock", T, prob, rows=[0, 5, 27, 200])


@pytest.mark.parametrize("L,n_meas", [(16, 40_000), (32, 20_000), (64, 12_000)])
def test_ising_energy_kaufman_at_tc(orc, L, n_meas):
    exact = et.ising_potts_energy(L, TC2)
    e, _, _ = orc.run(L, 2, "potts", TC2, 1.0, 4242 + L, 500, n_meas)
    mean, err = et.binned_mean(e)
    assert abs(mean - exact) < 4.5 * err, (mean, exact, err)


def test_ising_energy_infinite_lattice_limit(orc):
    # e_inf = 1 - 1/sqrt(2) at T_c (Onsager); the L = 256 torus is within the
    # finite-size bias bounded by Kaufman's L = 256 value plus statistical error.
    L = 256
    e_inf = 1.0 - 1.0 / math.sqrt(2.0)
    bias = abs(et.ising_potts_energy(L, TC2) - e_inf)
    e, _, _ = orc.run(L, 2, "potts", TC2, 1.0, 5, 100, 600)
    mean, err = et.binned_mean(e, nbins=20)
    assert abs(mean - e_inf) < bias + 4.5 * err
    assert bias < 0.002


def test_potts_self_dual_energy_loose(orc):
    # At the self-dual point the infinite-lattice energy per site of
    # H = -J sum (delta - 1) is 1 - 1/sqrt(q); finite size corrections at
    # L = 64 are a few 1e-2 for q = 3, 4.
    for q in (3, 4):
        Tc = 1.0 / math.log(1.0 + math.sqrt(q))
        e, _, _ = orc.run(64, q, "potts", Tc, 1.0, 17, 200, 2000)
        assert abs(e.mean() - (1.0 - 1.0 / math.sqrt(q))) < 0.05


def test_binder_ratio_ising_tc_loose(orc):
    # U = <M^4>/<M^2>^2 (Sec. 4).  At T_c of the periodic square Ising model U
    # tends to about 1.168 (Binder cumulant 0.6107, Salas & Sokal 2000).
    e, m2, _ = orc.run(32, 2, "potts", TC2, 1.0, 23, 500, 30_000)
    U = (m2 * m2).mean() / m2.mean() ** 2
    assert abs(U - 1.168) < 0.03
