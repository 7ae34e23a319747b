"""GPU: the continuous-batching server.  Every request's result (final
counts, observables, spin fingerprint) must equal the same lattice run alone,
and the oracle's for a sample; admission keeps within the memory budget."""
import math
import sys

import numpy as np
import pytest

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


def _trace(n, seed):
    from paper_1202_0635_amd.workloads import TC_POTTS, T_CLOCK6, LatticeConfig

    rng = np.random.default_rng(seed)
    kinds = [("potts", 2), ("potts", 3), ("potts", 4), ("clock", 6)]
    out = []
    for i in range(n):
        L = int(rng.integers(2, 200))
        model, q = kinds[int(rng.integers(0, 4))]
        tc = TC_POTTS[q] if model == "potts" else T_CLOCK6
        out.append(LatticeConfig(f"t{i}", L, q, model, tc * (0.8 + 0.4 * rng.random()), seed=0x50000 + i,
                                 sweeps=int(rng.integers(1, 60))))
    return out


def test_server_results_equal_alone_and_oracle(swmc, orc):
    from paper_1202_0635_amd import serve

    trace = _trace(30, 11)
    arrivals = serve.poisson_arrivals(len(trace), rate=400.0, seed=3)
    _say("[serve] 30 requests, 4 MiB budget, 6 slots, 7 sweeps per step")
    out = serve.run_trace(trace, arrivals, budget_bytes=4 << 20, max_slots=6, sweeps_per_step=7)
    st = out["stats"]
    assert st["completed"] == len(trace) and st["rejected"] == 0 and st["active"] == 0 and st["waiting"] == 0
    assert st["used_bytes"] == 0
    for i, c in enumerate(trace):
        r = out["results"][i]
        assert r["status"] == 0 and r["t"] == c.sweeps
        lat = swmc.Lattice(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
        lat.sweep(c.sweeps)
        ob = lat.measure()
        assert r["spin_hash"] == serve.spin_hash(lat.spins()), f"request {i}"
        assert np.array_equal(r["hist"][: c.q], ob["hist"]) and np.array_equal(r["pair_hist"][: c.q], ob["pair_hist"])
        assert r["e"] == ob["e"] and r["m2"] == ob["m2"]
        lat.close()
        if i < 6:
            ch = orc.Chain(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed).sweep(c.sweeps)
            assert r["spin_hash"] == orc.hash_spins(ch.spins)


def test_server_rejects_what_cannot_fit(swmc):
    from paper_1202_0635_amd import serve

    srv = serve.Server(budget_bytes=2 << 20, max_slots=2, sweeps_per_step=5)
    _say("[serve] rejection")
    srv.submit(2048, 2, "potts", 1.0, 1.0, 1, 10, tag=7)  # needs ~40 MB
    srv.submit(16, 2, "potts", 1.0, 1.0, 2, 12, tag=8)
    res = {}
    for _ in range(10):
        srv.step()
        for r in srv.poll():
            res[r["tag"]] = r
        if len(res) == 2:
            break
    assert res[7]["status"] == -5 and res[8]["status"] == 0 and res[8]["t"] == 12
    srv.close()
