"""GPU parity over whole chains: per-sweep state hashes of the benchmark
workloads against the golden streams the CPU oracle wrote (tests/golden/,
make_golden.py).

The chain is a pure function of its parameters and seed, and the canonical
label of a cluster is its smallest site index (Sec. 2), so the spins and the
partition after every sweep are unique: H_s and H_l of every sweep must equal
the oracle's bit for bit.  The hashes are taken on the device from the label
forest after each sweep's border merge (SW_HASH), so every sweep of a fused
multi-sweep call is covered, in the launch configuration the benchmark times.
"""
import math
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")


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


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def chain_golden(name):
    """{t: (hash_spins, hash_labels)} of a chain's golden stream."""
    return {int(t): (int(hs, 16), int(hl, 16)) for t, hs, hl in _rows(f"{name}.txt")}


def _check_stream(got, gold, where):
    assert got.shape[0] > 0, f"{where}: no hashes recorded"
    for t, hs, hl in got.tolist():
        assert t in gold, f"{where}: sweep {t} has no golden value"
        ghs, ghl = gold[t]
        assert hs == ghs, f"{where}: spin hash differs at sweep {t}"
        assert hl == ghl, f"{where}: label hash differs at sweep {t}"


def _chunks(total, pattern):
    out, k = [], 0
    while sum(out) < total:
        out.append(min(pattern[k % len(pattern)], total - sum(out)))
        k += 1
    return out


# Ising L = 64 at T_c, all 1000 sweeps: single-sweep calls and fused calls of
# varying length, with both tile shapes.
@pytest.mark.parametrize("pattern", [(1,), (1, 2, 3, 5, 8, 13, 21, 34, 55, 89), (1000,), (7, 250, 1, 64)])
@pytest.mark.parametrize("waves", [4, 8])
def test_ising_L64_every_sweep(swmc, pattern, waves):
    from paper_1202_0635_amd.workloads import ISING_L64 as c

    gold = chain_golden(c.name)
    calls = _chunks(c.sweeps, pattern)
    _say(f"[golden C1] waves={waves} calls={len(calls)}")
    lat = swmc.Lattice(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed).set_tile_waves(waves)
    for n in calls:
        lat.sweep(n, hash=True)
    got = lat.hashes()
    assert got.shape == (c.sweeps, 3)
    assert np.array_equal(got[:, 0], np.arange(1, c.sweeps + 1))
    _check_stream(got, gold, "C1")
    assert lat.measure()["hash_spins"] == gold[c.sweeps][0]
    lat.close()


# The two L = 4096 workloads through their 200 thermalisation sweeps and 50
# more, in the benchmark's multi-sweep calls (fused flip-and-bond kernel) and
# with the autotuner's choice of waves per tile.
@pytest.mark.parametrize("name", ["potts2_L4096_Tc", "clock6_L4096_T0.9"])
@pytest.mark.parametrize("pattern", [(250,), (1, 1, 3, 45, 150, 50)])
def test_L4096_thermalisation(swmc, name, pattern):
    from paper_1202_0635_amd.workloads import CONFIGS

    c = CONFIGS[name]
    gold = chain_golden(name)
    n_gold = max(gold)
    calls = _chunks(n_gold, pattern)
    _say(f"[golden L4096] {name} calls={calls}")
    lat = swmc.Lattice(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
    if pattern == (250,):
        lat.sweep(5, hash=True)
        lat.tune(3)  # times each choice from this state and restores it
        calls = _chunks(n_gold - 5, pattern)
    for n in calls:
        lat.sweep(n, hash=True)
    got = lat.hashes()
    assert got.shape == (n_gold, 3)
    _check_stream(got, gold, name)
    ob = lat.measure()
    assert ob["t"] == n_gold and ob["hash_spins"] == gold[n_gold][0]
    lat.close()


def replica_golden():
    out = {}
    for r, t, hs, hl in _rows("potts3_replicas_256.txt"):
        out.setdefault(int(r), {})[int(t)] = (int(hs, 16), int(hl, 16))
    return out


# The 256 q = 3 replicas (L over 64 ... 512, T over [0.9, 1.1] T_c) at sweeps
# 1, 10, 100 and 500: uncaptured sweeps with hashes, and the 500 sweeps as one
# captured graph after the autotuner's choice, compared at the end by the state
# hash.
def test_replica_mix_256(swmc):
    from paper_1202_0635_amd.workloads import replica_mix_q3

    reps = replica_mix_q3(256)
    gold = replica_golden()
    specs = [(c.L, c.q, c.model, c.T, c.J, c.seed) for c in reps]
    _say("[golden C4] 256 replicas, 500 hashed sweeps")
    b = swmc.Batch(specs)
    b.sweep(500, hash=True)
    for r in range(len(reps)):
        got = b.hashes(r)
        assert got.shape == (500, 3)
        sub = {t: v for t, v in gold[r].items()}
        _check_stream(got[np.isin(got[:, 0], list(sub))], sub, f"replica {r}")
    b.close()
    _say("[golden C4] 256 replicas, tuned schedule, one graph of 500 sweeps")
    b = swmc.Batch(specs)
    b.tune(3)
    b.sweep(500)
    for r in range(len(reps)):
        ob = b.measure(r)
        assert ob["t"] == 500 and ob["hash_spins"] == gold[r][500][0], f"replica {r}"
    b.close()


def trace_golden():
    out = {}
    for row in _rows("request_trace_sample40.txt"):
        i, t, hs = int(row[0]), int(row[1]), int(row[2], 16)
        rest = list(map(int, row[3:]))
        q = len(rest) // 2
        out[i] = (t, hs, np.array(rest[:q]), np.array(rest[q:]))
    return out


# The 2000-request trace through the continuous-batching server (all arriving
# at once, a 2 GiB budget so admission binds): the 40 sampled requests must
# end in the oracle's state alone-vs-in-the-mix, and every request must run
# exactly its sweeps.
def test_request_trace_served(swmc):
    from paper_1202_0635_amd import serve
    from paper_1202_0635_amd.workloads import request_trace

    trace = request_trace(2000)
    gold = trace_golden()
    _say("[golden C5] 2000 requests through the server")
    out = serve.run_trace(trace, serve.poisson_arrivals(len(trace), 0.0), budget_bytes=2 << 30, max_slots=128,
                          sweeps_per_step=25)
    st = out["stats"]
    assert st["completed"] == len(trace) and st["rejected"] == 0 and st["used_bytes"] == 0
    for i, c in enumerate(trace):
        assert out["results"][i]["status"] == 0 and out["results"][i]["t"] == c.sweeps
    for i, (t, hs, hist, pair) in gold.items():
        r = out["results"][i]
        q = trace[i].q
        assert r["t"] == t and r["spin_hash"] == hs, f"request {i}"
        assert np.array_equal(r["hist"][:q], hist) and np.array_equal(r["pair_hist"][:q], pair), f"request {i}"


# The device hashes of sw_measure against host definitions of the same sums.
def test_measure_hashes_match_host(swmc, orc):
    from paper_1202_0635_amd import serve

    for L, q, model, T in [(64, 2, "potts", 1.1345927), (77, 6, "clock", 0.9), (130, 3, "potts", 0.9)]:
        lat = swmc.Lattice(L, q, model, T=T, seed=4)
        lat.sweep(3, verify=True)
        ob = lat.measure()
        assert ob["hash_spins"] == serve.spin_hash(lat.spins())
        assert ob["hash_labels"] == orc.hash_labels(lat.labels())
        assert abs(ob["absm"] - math.sqrt(ob["m2"])) <= 1e-15
        lat.close()


# The paper's labelers (Sec. 3) follow the same chain.
@pytest.mark.parametrize("labeler", ["hawick", "kalentev"])
def test_labelers_follow_golden_chain(swmc, labeler):
    from paper_1202_0635_amd.workloads import ISING_L64 as c

    gold = chain_golden(c.name)
    lat = swmc.Lattice(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed).set_labeler(labeler)
    lat.sweep(40, hash=True)
    _check_stream(lat.hashes(), gold, labeler)
    lat.close()
