"""GPU: equilibrium physics of the chain, checked against exact results that
owe nothing to the oracle (Sec. 4, Figs. 4 and 6).

The moment ratio U(T) = <M^4>/<M^2>^2 of two sizes crosses near the exact
critical temperature T_c = 1/ln(1 + sqrt q) (q = 2, 3 Potts).  At L = 16 and 32
the finite-size shift of the crossing is a few tenths of a per cent and the
statistical error of 20000 measured sweeps per point about as much, so the
crossing must fall within 1.5 % of T_c.  Far from T_c, U takes its limits:
1 in the ordered phase and (q + 1)/(q - 1) for the (q - 1)-component order
parameter of the disordered phase (Gaussian fluctuations).  The clock model's
correlation ratio R = G(L/2)/G(L/4) is 1 in the ordered limit and falls well
below it once the correlation length is short against L/4 (T = 1.5, above the
upper KT temperature near 0.9)."""
import sys

import pytest

import bench

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def swmc():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    import paper_1202_0635_amd as swmc

    swmc._lib.lib()
    return swmc


def _scan(swmc, q, model, temps, sizes, therm, meas, key):
    specs = [(L, q, model, T, 1.0, 0x700000 + 1000 * L + k) for L in sizes for k, T in enumerate(temps)]
    b = swmc.Batch(specs)
    b.sweep(therm)
    b.sweep(meas, measure=True)
    obs = [b.measure(r)[key] for r in range(len(specs))]
    b.close()
    return {L: obs[i * len(temps):(i + 1) * len(temps)] for i, L in enumerate(sizes)}


@pytest.mark.parametrize("q", [2, 3])
def test_moment_ratio_crosses_at_tc(swmc, q):
    tc = swmc.critical_temperature("potts", q)
    temps = [tc * (0.96 + 0.01 * k) for k in range(9)]
    _say(f"[physics] Potts q={q}: U(T) at L = 16, 32")
    curves = _scan(swmc, q, "potts", temps, [16, 32], 1000, 20000, "binder_u")
    cr = bench.crossings(temps, curves)
    _say(f"[physics] q={q} crossings {[round(c['T'] / tc, 5) for c in cr]} (in units of T_c)")
    assert len(cr) == 1, cr
    assert abs(cr[0]["T"] / tc - 1.0) < 0.015


@pytest.mark.parametrize("q", [2, 3])
def test_moment_ratio_limits(swmc, q):
    tc = swmc.critical_temperature("potts", q)
    curves = _scan(swmc, q, "potts", [0.5 * tc, 3.0 * tc], [32], 200, 4000, "binder_u")
    low, high = curves[32]
    _say(f"[physics] q={q}: U(T_c/2) = {low:.5f}, U(3 T_c) = {high:.5f}")
    assert abs(low - 1.0) < 1e-3
    assert abs(high - (q + 1) / (q - 1)) < 0.05 * (q + 1) / (q - 1)


def test_clock_correlation_ratio_limits(swmc):
    curves = _scan(swmc, 6, "clock", [0.2, 1.5], [32], 200, 4000, "corr_ratio")
    low, high = curves[32]
    _say(f"[physics] clock q=6: R(0.2) = {low:.5f}, R(1.5) = {high:.5f}")
    assert abs(low - 1.0) < 1e-3
    assert high < 0.5
