"""The allocation-free entry point sw_sweep_static against sw_sweep.

sw_sweep_static keeps every intermediate array of the sweep in the library's
static device buffer; its spins and canonical labels must equal those of a
context (sw_init + sw_write_spins + sw_sweep) bit for bit.  Two calls in a
row, the second on a smaller lattice, show that the shared buffer keeps no
state between calls that matters."""
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


def _reference(swmc, L, q, model, T, seed, t0, n):
    """State after t0 sweeps from the random start, and the state and
    canonical labels after n more, through a context."""
    lat = swmc.Lattice(L, q, model, T=T, seed=seed)
    lat.sweep(t0)
    start = lat.spins().copy()
    lat.sweep(n, verify=True)
    out = (start, lat.spins().copy(), lat.labels().copy())
    lat.close()
    return out


def _static(swmc, L, q, model, T, seed, t0, n, start):
    import torch

    spins = torch.from_numpy(start.reshape(-1).copy()).to("cuda")
    table = torch.from_numpy(swmc.cutoff_table(L, q, model, T).view(np.int32)).to("cuda")
    labels = torch.full((L * L,), -1, dtype=torch.int32, device="cuda")
    fault = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    swmc.sweep_static(spins, L, q, model, T=T, seed=seed, t=t0, nsweeps=n, table=table, labels=labels, fault=fault)
    torch.cuda.synchronize()
    return (spins.cpu().numpy().reshape(L, L), labels.cpu().numpy().reshape(L, L), int(fault.cpu()[0]))


# The largest size the buffer holds, then a smaller ragged lattice of the
# other model: the second call finds the first call's forest in the buffer.
CASES = [
    (1024, 2, "potts", 1.134592657106511, 21, 3, 4),
    (300, 6, "clock", 0.9, 22, 5, 3),
    (70, 3, "potts", 0.994972861071817, 23, 0, 2),
]


def test_static_sweeps_equal_context_sweeps(swmc):
    for (L, q, model, T, seed, t0, n) in CASES:
        _say(f"[no-alloc] L={L} q={q} {model} t0={t0} n={n}")
        start, want_s, want_l = _reference(swmc, L, q, model, T, seed, t0, n)
        got_s, got_l, fault = _static(swmc, L, q, model, T, seed, t0, n, start)
        assert fault == 0, f"L={L}: fault bits {fault}"
        assert np.array_equal(got_s, want_s), f"L={L}: spins differ"
        assert np.array_equal(got_l, want_l), f"L={L}: canonical labels differ"


def test_static_sweep_without_labels_and_zero_sweeps(swmc):
    import torch

    # without labels the flatten leaves root copies; L = 131 (odd side) takes
    # the flip's column-per-lane layout
    for (L, q, model, T, seed) in ((200, 4, "potts", 0.9102392266268373, 24), (131, 6, "clock", 0.9, 25)):
        _say(f"[no-alloc] no labels L={L} q={q} {model}")
        start, want_s, _ = _reference(swmc, L, q, model, T, seed, 2, 5)
        spins = torch.from_numpy(start.reshape(-1).copy()).to("cuda")
        table = torch.from_numpy(swmc.cutoff_table(L, q, model, T).view(np.int32)).to("cuda")
        swmc.sweep_static(spins, L, q, model, T=T, seed=seed, t=2, nsweeps=0, table=table)
        torch.cuda.synchronize()
        assert np.array_equal(spins.cpu().numpy().reshape(L, L), start)
        swmc.sweep_static(spins, L, q, model, T=T, seed=seed, t=2, nsweeps=5, table=table)
        torch.cuda.synchronize()
        assert np.array_equal(spins.cpu().numpy().reshape(L, L), want_s), f"L={L}: spins differ"


def test_static_rejects_beyond_maximum(swmc):
    import torch

    L = swmc.STATIC_MAX_L + 1
    spins = torch.zeros(L * L, dtype=torch.int8, device="cuda")
    table = torch.from_numpy(swmc.cutoff_table(L, 2, "potts", 1.0).view(np.int32)).to("cuda")
    with pytest.raises(swmc.SwError) as err:
        swmc.sweep_static(spins, L, 2, "potts", T=1.0, nsweeps=1, table=table)
    assert err.value.status == swmc._lib.SW_EINVAL
