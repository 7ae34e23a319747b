"""GPU: schedules, the autotuner and batches keep the chain bit-identical.

Canonical labels are unique, so the merge schedule cannot change any result;
a batch replica must follow exactly the chain of the same lattice swept alone
(and so the oracle's)."""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

TC2 = 1.0 / math.log(1.0 + math.sqrt(2.0))
TC3 = 1.0 / math.log(1.0 + math.sqrt(3.0))


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


@pytest.mark.parametrize("mt,L", [(1, 300), (2, 300), (4, 300), (4, 1100), (2, 1100)])
def test_schedule_does_not_change_results(swmc, orc, mt, L):
    # one replica under every merge schedule of the batched path
    q = 2
    _say(f"[schedule] L={L} merge_tiles={mt}")
    b = swmc.Batch([(L, q, "potts", TC2, 1.0, 41)]).set_schedule(mt)
    ch = orc.Chain(L, q, "potts", T=TC2, seed=41)
    for _ in range(3):
        b.sweep(1, verify=True)
        ch.sweep(1)
        assert np.array_equal(b.labels(0).reshape(-1), ch.labels)
        assert np.array_equal(b.spins(0).reshape(-1), ch.spins)
    b.close()


def test_tune_leaves_the_chain_unchanged(swmc, orc):
    L = 200
    _say("[tune] lattice")
    lat = swmc.Lattice(L, 3, "potts", T=TC3, seed=5)
    lat.sweep(4)
    chosen = lat.tune(3)
    assert chosen in (4, 8)  # waves per tile
    lat.sweep(2, verify=True)
    ch = orc.Chain(L, 3, "potts", T=TC3, seed=5).sweep(6)
    assert lat.measure()["t"] == 6
    assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    assert np.array_equal(lat.labels().reshape(-1), ch.labels)


MIX = [
    (64, 2, "potts", TC2, 1.0, 1),
    (100, 3, "potts", TC3, 1.0, 7),
    (130, 6, "clock", 0.9, 1.0, 3),
    (2, 2, "potts", TC2, 1.0, 5),
    (257, 4, "potts", 0.9, 1.0, 9),
    (65, 2, "clock", 1.2, 1.0, 12),
    (33, 32, "potts", 0.4, 1.0, 15),
    (128, 3, "potts", 1.1, 0.8, 0x4000),
]


@pytest.mark.parametrize("graph", [True, False])
def test_batch_replicas_follow_their_own_chains(swmc, orc, graph):
    _say(f"[batch] mix graph={graph}")
    b = swmc.Batch(MIX)
    b.sweep(4, graph=graph)
    b.sweep(1, verify=True, graph=graph)
    for r, (L, q, model, T, J, seed) in enumerate(MIX):
        ch = orc.Chain(L, q, model, T=T, J=J, seed=seed).sweep(5)
        assert np.array_equal(b.spins(r).reshape(-1), ch.spins), f"replica {r} spins"
        assert np.array_equal(b.labels(r).reshape(-1), ch.labels), f"replica {r} labels"
        assert b.measure(r)["t"] == 5
    b.close()


# Sides whose rows are not a multiple of four sites: the flip takes one
# column of sixteen rows per lane there (sixteen consecutive sites of a row
# per thread otherwise).  Sides below a tile, one or two sites past it, and
# every residue mod 4; the clock replicas read the old spins in that layout.
ODD_SIDES = [
    (3, 2, "potts", TC2, 1.0, 31),
    (5, 6, "clock", 0.9, 1.0, 32),
    (7, 3, "potts", TC3, 1.0, 33),
    (17, 4, "potts", 0.9, 1.0, 34),
    (63, 6, "clock", 0.8, 1.0, 35),
    (66, 2, "potts", TC2, 1.0, 36),
    (67, 6, "clock", 1.0, 1.0, 37),
    (129, 3, "potts", TC3, 1.0, 38),
    (131, 2, "clock", 1.1, 1.0, 39),
]


def test_batch_odd_sides_follow_the_oracle_every_sweep(swmc, orc):
    _say("[batch] odd sides, one sweep per call")
    b = swmc.Batch(ODD_SIDES)
    chains = [orc.Chain(L, q, model, T=T, J=J, seed=seed) for (L, q, model, T, J, seed) in ODD_SIDES]
    for t in range(1, 7):
        b.sweep(1, verify=(t % 3 == 0), graph=False)
        for r, ch in enumerate(chains):
            ch.sweep(1)
            assert np.array_equal(b.spins(r).reshape(-1), ch.spins), f"replica {r} (L={ODD_SIDES[r][0]}) spins, sweep {t}"
            if t % 3 == 0:
                assert np.array_equal(b.labels(r).reshape(-1), ch.labels), f"replica {r} labels, sweep {t}"
    b.close()


def test_batch_equals_alone_and_measures(swmc, orc):
    specs = [(96, 3, "potts", TC3 * (0.9 + 0.2 * r / 7), 1.0, 0x4000 + r) for r in range(8)]
    _say("[batch] measure")
    b = swmc.Batch(specs)
    b.sweep(10)
    b.sweep(20, measure=True)
    for r, (L, q, model, T, J, seed) in enumerate(specs):
        lat = swmc.Lattice(L, q, model, T=T, J=J, seed=seed)
        lat.sweep(10)
        lat.sweep(20, measure=True)
        ob, ol = b.measure(r), lat.measure()
        assert np.array_equal(b.spins(r), lat.spins())
        for k in ("t", "samples"):
            assert ob[k] == ol[k]
        assert np.array_equal(ob["hist"], ol["hist"]) and np.array_equal(ob["pair_hist"], ol["pair_hist"])
        for k in ("mean_e", "mean_m2", "mean_m4", "binder_u"):
            assert ob[k] == ol[k]
        lat.close()
    b.close()


def test_batch_schedules_and_tune(swmc, orc):
    specs = [(L, 3, "potts", TC3, 1.0, 100 + i) for i, L in enumerate((64, 128, 256, 512, 300, 70))]
    _say("[batch] schedules")
    ref = swmc.Batch(specs)
    ref.sweep(6)
    with pytest.raises(swmc.SwError):
        swmc.Batch(specs[:1]).set_schedule(8)
    with pytest.raises(swmc.SwError):
        swmc.Batch(specs[:1]).set_tile_waves(6)
    for mt, w in ((1, 4), (2, 4), (4, 8), (1, 8)):
        b = swmc.Batch(specs).set_schedule(mt).set_tile_waves(w)
        b.sweep(6)
        for r in range(len(specs)):
            assert np.array_equal(b.spins(r), ref.spins(r)), (mt, w, r)
        b.close()
    b = swmc.Batch(specs)
    b.sweep(3)
    mt, w = b.tune(2)
    assert mt in (1, 2, 4) and w in (4, 8)
    b.sweep(3)
    for r in range(len(specs)):
        assert np.array_equal(b.spins(r), ref.spins(r))
        assert b.measure(r)["t"] == 6


def test_profiles_name_every_launch(swmc):
    # per-launch timing with measurement: every kernel that ran is reported by name
    _say("[profile] batch and single lattice")
    b = swmc.Batch([(96, 3, "potts", TC3, 1.0, 1), (64, 6, "clock", 0.9, 1.0, 2)])
    b.sweep(3, measure=True, profile=True)
    prof = b.profile()
    for name in ("kb_bond_local<potts>", "kb_bond_local<clock>", "kb_border_merge", "kb_flatten", "kb_flip",
                 "kb_counts", "kb_count_sum"):
        assert prof[name][0] == 3, (name, prof)
        assert prof[name][1] > 0.0
    b.close()
    lat = swmc.Lattice(200, 2, "potts", T=TC2, seed=3)
    lat.sweep(4, measure=True, profile=True)
    prof = lat.profile()
    # a call: one bond kernel from the spins, then the bond kernel from the
    # previous codes (the flip fused in), a merge per sweep, one final flip
    expect = {"k_code_bond": 1, "k_code_flip_bond": 3, "k_node_merge": 4, "k_code_flip": 1, "k_counts": 4,
              "k_bond_local": 0, "k_border_merge": 0, "k_flatten": 0, "k_flip": 0}
    for name, n in expect.items():
        assert prof[name][0] == n, (name, prof)
    lat.close()


def test_batch_graph_runs_of_many_sweeps(swmc):
    # one call of n sweeps replays one captured run of n sweeps (up to 512, then
    # the remainder): the same states as sweeps taken one call at a time, with
    # and without the graph
    specs = [(L, q, m, T, 1.0, 300 + i) for i, (L, q, m, T) in
             enumerate([(64, 2, "potts", TC2), (130, 3, "potts", TC3), (70, 6, "clock", 0.9), (256, 2, "potts", 1.5)])]
    _say("[batch] graph runs")
    a = swmc.Batch(specs)
    a.sweep(700)  # a run of 512 and one of 188
    a.sweep(37)
    b = swmc.Batch(specs)
    for n in (1, 2, 5, 100, 3):
        b.sweep(n, graph=False)
    b.sweep(737 - 111)
    for r in range(len(specs)):
        assert np.array_equal(a.spins(r), b.spins(r)), r
        assert a.measure(r)["t"] == b.measure(r)["t"] == 737
    a.close()
    b.close()
