"""GPU: the paper's own labelers (Sec. 3; label equivalence after Hawick et al.
and after Kalentev et al.), kept as an ablation of the union-find path.

Canonical labels are unique, so every labeler must give the oracle's bonds,
canonical labels and spins bit for bit after every sweep, in single-sweep and
multi-sweep calls, with measurement, and when the labeler changes mid-chain."""
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


CASES = [
    # L, q, model, T, seed, sweeps
    (64, 2, "potts", TC2, 1, 4),
    (100, 3, "potts", TC3, 7, 3),     # ragged tiles
    (130, 6, "clock", 0.9, 3, 3),
    (2, 2, "potts", TC2, 5, 6),       # multigraph torus
    (127, 2, "potts", 0.5, 13, 3),    # ordered: clusters wrap around the torus
    (200, 2, "potts", 5.0, 14, 2),    # many small clusters
    (97, 32, "clock", 0.05, 16, 2),
]


@pytest.mark.parametrize("labeler", ["hawick", "kalentev"])
@pytest.mark.parametrize("L,q,model,T,seed,nsw", CASES)
def test_labeler_parity(swmc, orc, labeler, L, q, model, T, seed, nsw):
    _say(f"[labeler] {labeler} L={L} q={q} {model}")
    lat = swmc.Lattice(L, q, model, T=T, seed=seed).set_labeler(labeler)
    ch = orc.Chain(L, q, model, T=T, seed=seed)
    for s in range(nsw):
        lat.sweep(1, verify=True)
        ch.sweep(1)
        br, bd = lat.bonds()
        assert np.array_equal(br.reshape(-1), ch.bond_r) and np.array_equal(bd.reshape(-1), ch.bond_d), s
        assert np.array_equal(lat.labels().reshape(-1), ch.labels), f"labels differ at sweep {s}"
        assert np.array_equal(lat.spins().reshape(-1), ch.spins), f"spins differ at sweep {s}"
    stats = lat.labeler_stats()
    assert stats["sweeps"] == nsw and stats["iterations"] >= nsw
    lat.close()


@pytest.mark.parametrize("labeler", ["hawick", "kalentev"])
def test_labeler_multi_sweep_measured_and_switched(swmc, orc, labeler):
    L, q, model, T = 90, 3, "potts", TC3
    _say(f"[labeler] {labeler} multi-sweep")
    lat = swmc.Lattice(L, q, model, T=T, seed=21).set_labeler(labeler)
    lat.sweep(5, measure=True)
    lat.set_labeler("union_find").sweep(3)
    lat.set_labeler(labeler).sweep(4, verify=True)
    e, m2, s_final = orc.run(L, q, model, T, 1.0, 21, 0, 5)
    ch = orc.Chain(L, q, model, T=T, seed=21).sweep(12)
    assert np.array_equal(lat.spins().reshape(-1), ch.spins)
    assert np.array_equal(lat.labels().reshape(-1), ch.labels)
    ob = lat.measure()
    assert ob["t"] == 12 and ob["samples"] == 5
    assert abs(ob["mean_e"] - e.mean()) <= 1e-12 * max(1.0, abs(e.mean()))
    lat.close()


def test_labeler_rejects_unknown(swmc):
    lat = swmc.Lattice(16, 2, "potts", T=1.0)
    with pytest.raises(swmc.SwError):
        lat.set_labeler(3)
    lat.close()
