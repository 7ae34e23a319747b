"""GPU parity: the HIP sweep against the CPU oracle, element by element.

Bonds, canonical labels and spins must be bit-identical after every sweep
(the chain is a pure function of parameters and seed); counts are integers
and must be identical; E, M^2, M^4 and the moment ratio agree to 1e-12
relative (they are computed from identical integer counts).
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TC2 = 1.0 / math.log(1.0 + math.sqrt(2.0))
TC3 = 1.0 / math.log(1.0 + math.sqrt(3.0))
TC4 = 1.0 / math.log(3.0)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def swmc():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    import paper_1202_0635_amd as swmc

    swmc._lib.lib()  # fail loudly if the HIP library was not built
    return swmc


CASES = [
    # L, q, model, T, seed, sweeps
    (64, 2, "potts", TC2, 1, 6),       # Ising L = 64 at T_c
    (100, 3, "potts", TC3, 7, 5),      # ragged tiles
    (130, 6, "clock", 0.9, 3, 5),      # ragged clock
    (2, 2, "potts", TC2, 5, 8),        # multigraph torus
    (3, 3, "potts", 0.7, 9, 8),
    (5, 6, "clock", 0.6, 4, 8),
    (63, 4, "potts", TC4, 11, 4),
    (65, 2, "clock", 1.2, 12, 4),
    (127, 2, "potts", 0.5, 13, 4),     # ordered: wrapped spanning clusters
    (200, 2, "potts", 5.0, 14, 3),     # disordered: many small clusters
    (192, 32, "potts", 0.4, 15, 3),    # q at the upper limit
    (97, 32, "clock", 0.05, 16, 3),    # large q clock, cold
    (256, 6, "clock", 0.9, 17, 3),
]


@pytest.mark.parametrize("L,q,model,T,seed,nsw", CASES)
def test_sweep_parity(swmc, orc, L, q, model, T, seed, nsw):
    _say(f"[parity] L={L} q={q} {model} T={T:.4f} seed={seed}")
    lat = swmc.Lattice(L, q, model, T=T, seed=seed)
    ch = orc.Chain(L, q, model, T=T, seed=seed)
    assert np.array_equal(lat.spins().reshape(-1), ch.spins), "random start differs"
    for s in range(nsw):
        lat.sweep(1, verify=True)
        ch.sweep(1)
        br, bd = lat.bonds()
        assert np.array_equal(br.reshape(-1), ch.bond_r), f"right bonds differ at sweep {s}"
        assert np.array_equal(bd.reshape(-1), ch.bond_d), f"down bonds differ at sweep {s}"
        assert np.array_equal(lat.labels().reshape(-1), ch.labels), f"labels differ at sweep {s}"
        assert np.array_equal(lat.spins().reshape(-1), ch.spins), f"spins differ at sweep {s}"
    lat.close()


@pytest.mark.parametrize("L,q,model,T", [(96, 3, "potts", TC3), (77, 6, "clock", 0.9)])
def test_parity_from_arbitrary_state(swmc, orc, L, q, model, T):
    from paper_1202_0635_amd.workloads import random_spins, striped_spins

    for k, s0 in enumerate([random_spins(L, q, 5), striped_spins(L, q, 3)]):
        _say(f"[parity-state] L={L} q={q} {model} start={k}")
        t0 = 1000 + k
        lat = swmc.Lattice(L, q, model, T=T, seed=21).set_spins(s0, t=t0)
        ch = orc.Chain(L, q, model, T=T, seed=21, spins=s0, t=t0)
        for _ in range(3):
            lat.sweep(1, verify=True)
            ch.sweep(1)
            assert np.array_equal(lat.labels().reshape(-1), ch.labels)
            assert np.array_equal(lat.spins().reshape(-1), ch.spins)
        lat.close()


# Several sweeps in one call run the previous sweep's flip inside the next
# sweep's bond kernel (from the previous sweep's codes and node forest,
# alternating between two buffers); the state after every call, and the last
# sweep's bonds and labels, must be the oracle's.
@pytest.mark.parametrize("L,q,model,T,seed,calls", [
    (2, 2, "potts", TC2, 5, (4, 3)), (3, 3, "potts", 0.7, 9, (5,)), (5, 6, "clock", 0.6, 4, (2, 1, 3)),
    (64, 2, "potts", TC2, 1, (6,)), (70, 2, "clock", 1.2, 12, (3, 2)), (100, 3, "potts", TC3, 7, (5,)),
    (130, 6, "clock", 0.9, 3, (4, 1)), (127, 2, "potts", 0.5, 13, (4,)), (200, 2, "potts", 5.0, 14, (3,)),
    (192, 32, "potts", 0.4, 15, (3,)), (97, 32, "clock", 0.05, 16, (3,)),
])
@pytest.mark.parametrize("waves", [4, 8])  # 16 or 8 rows per wave of a tile
def test_multi_sweep_calls(swmc, orc, L, q, model, T, seed, calls, waves):
    _say(f"[fused] L={L} q={q} {model} calls={calls} waves={waves}")
    lat = swmc.Lattice(L, q, model, T=T, seed=seed).set_tile_waves(waves)
    ch = orc.Chain(L, q, model, T=T, seed=seed)
    for n in calls:
        lat.sweep(n, verify=True)
        ch.sweep(n)
        br, bd = lat.bonds()  # the last sweep's bonds (from the fused kernel when n > 1)
        assert np.array_equal(br.reshape(-1), ch.bond_r) and np.array_equal(bd.reshape(-1), ch.bond_d)
        assert np.array_equal(lat.spins().reshape(-1), ch.spins)
        assert np.array_equal(lat.labels().reshape(-1), ch.labels)
    assert lat.measure()["t"] == sum(calls)
    lat.close()


def test_many_sweeps_batch_call(swmc, orc):
    # 40 sweeps enqueued by one call; compare the end state and last labels.
    L, q, T = 160, 2, TC2
    _say("[parity-many] L=160 40 sweeps")
    lat = swmc.Lattice(L, q, "potts", T=T, seed=99)
    ch = orc.Chain(L, q, "potts", T=T, seed=99)
    lat.sweep(40, verify=True)
    ch.sweep(40)
    assert np.array_equal(lat.labels().reshape(-1), ch.labels)
    assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    assert lat.measure()["t"] == 40


# q <= 8: the counts of a sweep are taken by the next sweep's bond kernel (the
# last sweep of a call by the count kernel); q = 10: the count kernel every
# sweep.  1100 sweeps cross the 1024-row device ring; split calls hand the
# pending count over to the count kernel at every call boundary.
@pytest.mark.parametrize("q,model,T,L,calls", [
    (2, "potts", TC2, 48, (300,)), (3, "potts", TC3, 48, (300,)), (6, "clock", 0.9, 48, (300,)),
    (10, "potts", 1.0 / np.log(1.0 + np.sqrt(10.0)), 40, (300,)),
    (2, "potts", TC2, 24, (1100,)), (3, "potts", TC3, 40, (1, 7, 1, 291)),
    (3, "potts", TC3, 37, (120,)), (6, "clock", 0.9, 1030, (3,)),   # rows not a multiple of 4; > 1 step per row
    (2, "potts", TC2, 45, (60,)), (2, "clock", 1.2, 1030, (2,)), (8, "potts", 0.7, 50, (40,)),
])
def test_measurements(swmc, orc, q, model, T, L, calls):
    therm, nmeas = 20, sum(calls)
    _say(f"[measure] q={q} {model} L={L} calls={calls}")
    lat = swmc.Lattice(L, q, model, T=T, seed=31)
    lat.sweep(therm)
    for n in calls:
        lat.sweep(n, measure=True)
    ob = lat.measure()
    e, m2, s_final = orc.run(L, q, model, T, 1.0, 31, therm, nmeas)
    assert np.array_equal(lat.spins(), s_final)
    ch = orc.Chain(L, q, model, T=T, seed=31, spins=s_final)
    h, p = ch.counts()
    assert np.array_equal(ob["hist"], h) and np.array_equal(ob["pair_hist"], p)
    e_now, m2_now = ch.observables()
    rel = lambda a, b: abs(a - b) <= 1e-12 * max(1.0, abs(b))
    assert rel(ob["e"], e_now) and rel(ob["m2"], m2_now)
    assert ob["samples"] == nmeas
    assert rel(ob["mean_e"], e.mean()) and rel(ob["mean_m2"], m2.mean())
    assert rel(ob["mean_m4"], (m2 * m2).mean())
    U = (m2 * m2).mean() / m2.mean() ** 2
    assert rel(ob["binder_u"], U)
    if model == "potts":
        assert not ob["corr_hist"].any() and ob["mean_g_quarter"] == 0.0


# The clock model's correlation function (Sec. 4): exact correlation counts at
# r = L/4 and L/2 of the final state, G of that state, and the running means
# and their ratio R, against the oracle sweep by sweep.  q = 2 and 6 take the
# per-lane bin path, q = 10 the shared-bin path; L = 1030 and 37 give rows
# that are not a multiple of four sites and displacements that wrap inside a
# group of four.
@pytest.mark.parametrize("q,T,L,calls", [
    (6, 0.9, 48, (40,)), (6, 0.9, 1030, (3,)), (2, 1.2, 37, (20,)), (4, 0.8, 64, (1, 9)),
    (10, 0.6, 40, (12,)), (6, 1.1, 130, (5,)), (3, 0.7, 45, (8,)),
])
def test_clock_correlations(swmc, orc, q, T, L, calls):
    therm = 6
    _say(f"[corr] clock q={q} L={L} calls={calls}")
    lat = swmc.Lattice(L, q, "clock", T=T, seed=77)
    lat.sweep(therm)
    for n in calls:
        lat.sweep(n, measure=True)
    ob = lat.measure()
    ch = orc.Chain(L, q, "clock", T=T, seed=77).sweep(therm)
    g1s, g2s = [], []
    for _ in range(sum(calls)):
        ch.sweep(1)
        c1, c2 = ch.corr_counts()
        g1s.append(orc.corr_g(L, q, c1))
        g2s.append(orc.corr_g(L, q, c2))
    assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    c1, c2 = ch.corr_counts()
    assert np.array_equal(ob["corr_hist"][0], c1) and np.array_equal(ob["corr_hist"][1], c2)
    rel = lambda a, b: abs(a - b) <= 1e-12 * max(1.0, abs(b))
    assert rel(ob["g_quarter"], g1s[-1]) and rel(ob["g_half"], g2s[-1])
    m1, m2 = float(np.mean(g1s)), float(np.mean(g2s))
    assert rel(ob["mean_g_quarter"], m1) and rel(ob["mean_g_half"], m2)
    assert rel(ob["corr_ratio"], m2 / m1)
    # a batch replica measures the same
    b = swmc.Batch([(L, q, "clock", T, 1.0, 77)])
    b.sweep(therm)
    b.sweep(sum(calls), measure=True)
    obb = b.measure(0)
    assert np.array_equal(obb["corr_hist"], ob["corr_hist"])
    assert rel(obb["mean_g_quarter"], m1) and rel(obb["corr_ratio"], m2 / m1)
    b.close()
    lat.close()


@pytest.mark.parametrize("model,q,T,nsw", [("potts", 2, TC2, 3), ("clock", 6, 0.9, 2)])
def test_full_size_L4096(swmc, orc, model, q, T, nsw):
    # The benchmark lattice at full size: whole-state comparison after a few
    # sweeps (the oracle needs about a second per sweep here).
    L = 4096
    _say(f"[full] L=4096 {model} q={q}")
    lat = swmc.Lattice(L, q, model, T=T, seed=2)
    ch = orc.Chain(L, q, model, T=T, seed=2)
    for s in range(nsw):
        lat.sweep(1, verify=True)
        ch.sweep(1)
        assert np.array_equal(lat.labels().reshape(-1), ch.labels), f"labels differ at sweep {s}"
        assert np.array_equal(lat.spins().reshape(-1), ch.spins), f"spins differ at sweep {s}"
    lat.close()


@pytest.mark.parametrize("waves", [4, 8])  # the autotuner picks 4 at this size
@pytest.mark.parametrize("model,q,T", [("potts", 2, TC2), ("clock", 6, 0.9)])
def test_full_size_L4096_one_call(swmc, orc, model, q, T, waves):
    # The benchmark's launch configuration: several sweeps in one call, every
    # sweep after the first running the fused flip-and-bond kernel.  Whole
    # states are compared, with the counts of a measured call and the bonds and
    # canonical labels of a verified one.
    L = 4096
    _say(f"[full, one call] L=4096 {model} q={q} waves={waves}")
    lat = swmc.Lattice(L, q, model, T=T, seed=2).set_tile_waves(waves)
    ch = orc.Chain(L, q, model, T=T, seed=2)
    lat.sweep(3, measure=True)
    ch.sweep(3)
    assert np.array_equal(lat.spins().reshape(-1), ch.spins), "spins differ after a 3-sweep call"
    ob = lat.measure()
    hist, pair = ch.counts()
    assert ob["t"] == 3 and ob["samples"] == 3
    assert np.array_equal(ob["hist"], hist) and np.array_equal(ob["pair_hist"], pair)
    lat.sweep(2, verify=True)
    ch.sweep(2)
    br, bd = lat.bonds()
    assert np.array_equal(br.reshape(-1), ch.bond_r) and np.array_equal(bd.reshape(-1), ch.bond_d)
    assert np.array_equal(lat.labels().reshape(-1), ch.labels)
    assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    lat.close()


@pytest.mark.parametrize("L,q,model,T,seed", [
    (2, 2, "potts", TC2, 5), (70, 3, "potts", TC3, 6), (130, 6, "clock", 0.9, 3), (300, 2, "potts", TC2, 7),
    (127, 2, "potts", 0.5, 13),
])
@pytest.mark.parametrize("waves", [4, 8])
def test_tile_waves_do_not_change_results(swmc, orc, L, q, model, T, seed, waves):
    # 4 waves of 16 rows or 8 waves of 8 rows per tile: the same bonds, labels and spins
    _say(f"[tile waves] L={L} q={q} {model} waves={waves}")
    lat = swmc.Lattice(L, q, model, T=T, seed=seed).set_tile_waves(waves)
    ch = orc.Chain(L, q, model, T=T, seed=seed)
    for n in (1, 4):
        lat.sweep(n, verify=True)
        ch.sweep(n)
        br, bd = lat.bonds()
        assert np.array_equal(br.reshape(-1), ch.bond_r) and np.array_equal(bd.reshape(-1), ch.bond_d)
        assert np.array_equal(lat.labels().reshape(-1), ch.labels)
        assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    lat.close()


def test_zero_sweeps_change_nothing(swmc, orc):
    # a call with no sweeps (with or without measurement) leaves state, sweep
    # index and running averages as they were
    lat = swmc.Lattice(70, 3, "potts", T=TC3, seed=8)
    lat.sweep(3, measure=True)
    s0, ob0 = lat.spins().copy(), lat.measure()
    lat.sweep(0)
    lat.sweep(0, measure=True)
    ob1 = lat.measure()
    assert np.array_equal(lat.spins(), s0)
    assert ob1["t"] == ob0["t"] == 3 and ob1["samples"] == ob0["samples"] == 3
    assert ob1["mean_e"] == ob0["mean_e"]
    ch = orc.Chain(70, 3, "potts", T=TC3, seed=8).sweep(3)
    assert np.array_equal(s0.reshape(-1), ch.spins)
    lat.close()


def test_invalid_arguments_raise(swmc):
    with pytest.raises(swmc.SwError):
        swmc.Lattice(1, 2, "potts", T=1.0)
    with pytest.raises(swmc.SwError):
        swmc.Lattice(16, 33, "potts", T=1.0)
    lat = swmc.Lattice(16, 3, "potts", T=1.0)
    with pytest.raises(swmc.SwError):
        lat.set_spins(np.full((16, 16), 3, np.int8))
    with pytest.raises(swmc.SwError):
        lat.labels()  # no SW_VERIFY sweep yet
    with pytest.raises(swmc.SwError):
        lat.sweep(-1)
    for w in (0, 2, 5, 16):
        with pytest.raises(swmc.SwError):
            lat.set_tile_waves(w)
