"""Pins of the oracle's bond cutoff tables (Sec. 2 step (ii); Sec. 4 embedded cluster).

The oracle evaluates p = -expm1(-x) in FP64 and takes floor(2^32 p).  These
tests rebuild every entry from closed forms in 60-digit decimal arithmetic:
at the Potts critical point T = 1/ln(1+sqrt q) the bond probability is exactly
sqrt(q)/(1+sqrt(q)); the clock projection P is recomputed from plane geometry
(cos(theta_a - phi) cos(theta_b - phi) with phi = pi m/q + pi/2), and the mirror
is checked to reflect spin a onto spin (m - a) mod q.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

getcontext().prec = 60
TWO32 = Decimal(2) ** 32


def dec_floor_cutoff(p: Decimal) -> int:
    c = int((p * TWO32).to_integral_value(rounding="ROUND_FLOOR"))
    return min(c, 2**32 - 1)


def dec_one_minus_exp(x: Decimal) -> Decimal:
    return Decimal(1) - (-x).exp()


@pytest.mark.parametrize("q", [2, 3, 4])
def test_potts_cutoff_at_critical_point(orc, q):
    # Sec. 4: T_c/J = 1/ln(1+sqrt q) (q = 2, 3 printed; q = 4 by the same
    # self-dual formula).  There p = 1 - 1/(1+sqrt q) = sqrt q / (1 + sqrt q).
    Tc = 1.0 / math.log(1.0 + math.sqrt(q))
    tab = orc.cutoffs("potts", q, Tc, 1.0).reshape(q, q)
    sq = Decimal(q).sqrt()
    expect = dec_floor_cutoff(sq / (1 + sq))
    # FP64 Tc differs from the exact Tc by at most ~1 ulp, which moves
    # 2^32 p by ~1e-6: assert the floor is not that close to an integer.
    frac = (sq / (1 + sq)) * TWO32 - expect
    assert Decimal("1e-5") < frac < 1 - Decimal("1e-5")
    for a in range(q):
        for b in range(q):
            assert tab[a, b] == (expect if a == b else 0)


@pytest.mark.parametrize("T", [0.05, 0.3, 0.9, 1.1345926, 2.0, 7.5, 1e3, 1e8])
@pytest.mark.parametrize("J", [1.0, 0.5, 2.5])
def test_potts_cutoff_general(orc, T, J):
    tab = orc.cutoffs("potts", 3, T, J).reshape(3, 3)
    x = Decimal(J) / Decimal(T)
    exact = dec_one_minus_exp(x) * TWO32
    c = int(tab[0, 0])
    # floor(2^32 p) up to FP64 rounding of p (relative 1e-15 -> < 1e-5 absolute)
    assert abs(Decimal(c) - exact.to_integral_value(rounding="ROUND_FLOOR")) <= 1
    if min(exact - int(exact), int(exact) + 1 - exact) > Decimal("1e-4") and exact < TWO32 - 1:
        assert c == min(int(exact), 2**32 - 1)
    assert tab[0, 1] == 0 and tab[1, 2] == 0


def test_potts_cutoff_extremes(orc):
    # Very low T: p -> 1, clamped to the largest u32.  Very high T: p -> 0.
    assert orc.cutoffs("potts", 2, 1e-3, 1.0)[0] == 2**32 - 1
    assert orc.cutoffs("potts", 2, 1e12, 1.0)[0] == 0


@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 8, 12])
def test_clock_projection_is_plane_geometry(orc, q):
    for m in range(q):
        phi = math.pi * m / q + math.pi / 2
        for a in range(q):
            for b in range(q):
                ta, tb = 2 * math.pi * a / q, 2 * math.pi * b / q
                geo = math.cos(ta - phi) * math.cos(tb - phi)
                assert abs(orc.clock_projection(q, a, b, m) - geo) < 1e-12


@pytest.mark.parametrize("q", [2, 3, 4, 5, 6, 8, 12])
def test_clock_mirror_maps_a_to_m_minus_a(orc, q):
    # Reflection S -> S - 2 (S.r) r with r = (cos phi, sin phi) maps the clock
    # state a onto (m - a) mod q.
    for m in range(q):
        phi = math.pi * m / q + math.pi / 2
        r = np.array([math.cos(phi), math.sin(phi)])
        for a in range(q):
            S = np.array([math.cos(2 * math.pi * a / q), math.sin(2 * math.pi * a / q)])
            R = S - 2 * S.dot(r) * r
            k = (m - a) % q
            T = np.array([math.cos(2 * math.pi * k / q), math.sin(2 * math.pi * k / q)])
            assert np.allclose(R, T, atol=1e-12)


def test_clock_wrong_mirror_direction_is_not_a_reflection_onto_m_minus_a():
    # The other reading, phi = pi m / q, preserves the projected component:
    # the map k -> (m - k) is then not the reflection along r (negative control).
    q, m, a = 6, 1, 0
    phi = math.pi * m / q
    r = np.array([math.cos(phi), math.sin(phi)])
    S = np.array([1.0, 0.0])
    R = S - 2 * S.dot(r) * r
    k = (m - a) % q
    T = np.array([math.cos(2 * math.pi * k / q), math.sin(2 * math.pi * k / q)])
    assert not np.allclose(R, T, atol=1e-6)


@pytest.mark.parametrize("T,J", [(0.9, 1.0), (0.7, 1.0), (1.3, 0.5)])
def test_clock6_cutoffs_exact(orc, T, J):
    q = 6
    tab = orc.cutoffs("clock", q, T, J).reshape(q, q, q)
    for m in range(q):
        phi = math.pi * m / q + math.pi / 2
        for a in range(q):
            for b in range(q):
                geo = math.cos(2 * math.pi * a / q - phi) * math.cos(2 * math.pi * b / q - phi)
                quarter = round(geo * 4)
                assert abs(geo * 4 - quarter) < 1e-9  # q = 6: P in {0, +-1/4, ..., +-1}
                if quarter <= 0:
                    assert tab[m, a, b] == 0
                else:
                    P = Decimal(quarter) / 4
                    exact = dec_one_minus_exp(2 * Decimal(J) * P / Decimal(T)) * TWO32
                    assert tab[m, a, b] == min(int(exact), 2**32 - 1)
                assert tab[m, a, b] == tab[m, b, a]


def test_clock6_projection_values(orc):
    vals = {round(orc.clock_projection(6, a, b, m) * 4) for a in range(6) for b in range(6) for m in range(6)}
    assert vals == {-4, -3, -2, -1, 0, 1, 2, 3, 4}


@pytest.mark.parametrize("q", [5, 7, 12])
def test_clock_cutoffs_general_q(orc, q):
    T = 0.8
    tab = orc.cutoffs("clock", q, T, 1.0).reshape(q, q, q)
    for m in range(q):
        for a in range(q):
            for b in range(q):
                P = orc.clock_projection(q, a, b, m)
                if P <= 1e-12:
                    assert tab[m, a, b] == 0 or P > 0
                else:
                    exact = dec_one_minus_exp(2 * Decimal(P) / Decimal(T)) * TWO32
                    assert abs(int(tab[m, a, b]) - int(exact)) <= 1


def test_invalid_parameters(orc):
    for bad in [dict(q=1), dict(q=33)]:
        with pytest.raises(ValueError):
            orc.cutoffs("potts", bad["q"], 1.0, 1.0)
    with pytest.raises(ValueError):
        orc.cutoffs("potts", 2, 0.0, 1.0)
    with pytest.raises(ValueError):
        orc.cutoffs("potts", 2, 1.0, -1.0)
