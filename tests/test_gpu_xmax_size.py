"""GPU: the largest single lattice, L = 65535 (N = 4 294 836 225 sites, just
below 2^32).  Site indices, canonical labels and node keys are 32-bit
unsigned words with no flag bit, so labels pass 2^31 here (the label read
back is uint32); the last tile column and tile row are 63 sites wide.  A whole
oracle sweep would take minutes, so each sweep is checked on outputs the
oracle computes one site at a time (bonds of sampled sites from the state
before the sweep, their new values from their canonical labels and old
values) and on properties that hold at any size: every active bond joins two
sites of equal label, a label is never larger than its site and labels
itself, and the counts equal those of the state read back.  A second lattice
runs the same sweeps in one call (the fused flip-and-bond kernel after the
first sweep) and must end in the same state.  (Sec. 5 names the lattice size
as the limit of the paper's labeling; both lattices together take about
130 GB of device memory.)
"""
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

L = 65535
N = L * L
TC2 = 1.0 / math.log(1.0 + math.sqrt(2.0))
ROWS = 1024  # rows per chunk of the whole-array checks


_progress = None


def _say(*a):
    """Progress lines that pytest does not capture: this test runs for minutes
    of host-side checks, and its output must show that it is alive."""
    if _progress is not None:
        with _progress.disabled():
            print(*a, flush=True)
    else:
        print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def swmc():
    import torch

    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    import paper_1202_0635_amd as swmc

    swmc._lib.lib()
    return swmc


def _samples(rng):
    """Random sites plus sites on tile edges, in the narrow last tiles and at
    the wrap."""
    edge = np.array([0, 1, 63, 64, 127, 128, L - 65, L - 64, L - 63, L - 62, L - 2, L - 1], dtype=np.int64)
    rand = rng.integers(0, N, 100_000, dtype=np.int64)
    ey = np.repeat(edge, 400) * L + rng.integers(0, L, edge.size * 400)
    ex = rng.integers(0, L, edge.size * 400) * L + np.repeat(edge, 400)
    corner = (edge[:, None] * L + edge[None, :]).reshape(-1)
    return np.unique(np.concatenate([rand, ey, ex, corner]))


def _check_labels(lab, br, bd):
    """Active bonds join equal labels; lab[i] <= i; roots label themselves."""
    for y0 in range(0, L, ROWS):
        if y0 % (16 * ROWS) == 0:
            _say(f"    label checks, rows {y0}..")
        y1 = min(L, y0 + ROWS)
        blk = lab[y0:y1]
        idx = np.arange(y0 * L, y1 * L, dtype=np.int64).reshape(y1 - y0, L)
        assert np.all(blk <= idx), f"a label above its site in rows {y0}..{y1}"
        right = np.roll(blk, -1, axis=1)
        assert not np.any(br[y0:y1].astype(bool) & (blk != right)), f"right bond across labels, rows {y0}..{y1}"
        below = lab[np.arange(y0 + 1, y1 + 1) % L]
        assert not np.any(bd[y0:y1].astype(bool) & (blk != below)), f"down bond across labels, rows {y0}..{y1}"


def _counts(s, q):
    """n[k] and the neighbour pairs by (s_j - s_i) mod q, by byte arithmetic."""
    hist = np.zeros(q, dtype=np.int64)
    pair = np.zeros(q, dtype=np.int64)
    uq = np.uint8(q)
    for y0 in range(0, L, ROWS):
        if y0 % (16 * ROWS) == 0:
            _say(f"    counts, rows {y0}..")
        y1 = min(L, y0 + ROWS)
        blk = s[y0:y1].view(np.uint8)
        hist += [np.count_nonzero(blk == k) for k in range(q)]
        for nb in (np.roll(blk, -1, axis=1), s[np.arange(y0 + 1, y1 + 1) % L].view(np.uint8)):
            d = nb + uq - blk
            d %= uq
            pair += [np.count_nonzero(d == k) for k in range(q)]
    return hist, pair


@pytest.mark.timeout(900)
@pytest.mark.parametrize("model,q,T,nsw", [("potts", 2, TC2, 2), ("clock", 6, 0.9, 2)])
def test_maximum_size(swmc, orc, model, q, T, nsw, capsys):
    global _progress
    _progress = capsys
    seed = 11
    rng = np.random.default_rng(3)
    S = _samples(rng)
    table = orc.cutoffs(model, q, T)
    _say(f"[max size] L={L} {model} q={q}: random start")
    a = swmc.Lattice(L, q, model, T=T, seed=seed)
    s = a.spins()
    flat = s.reshape(-1)
    few = S[:: max(1, S.size // 4000)]
    want = [orc.qmap(int(orc.draw(seed, int(i), 0, 4)[0]), q) for i in few]
    assert np.array_equal(flat[few], np.array(want, dtype=np.int8)), "random start differs"
    for t in range(nsw):
        _say(f"[max size] {model} sweep {t} (one sweep per call, verified)")
        a.sweep(1, verify=True)
        br, bd = a.bonds()
        _say(f"    bonds read")
        wr, wd = orc.bonds_at(L, q, model, table, seed, t, s, S)
        assert np.array_equal(br.reshape(-1)[S], wr), f"right bonds differ at sweep {t}"
        assert np.array_equal(bd.reshape(-1)[S], wd), f"down bonds differ at sweep {t}"
        lab = a.labels()
        _say(f"    labels read")
        _check_labels(lab, br, bd)
        del br, bd
        lf = lab.reshape(-1)
        assert np.array_equal(lf[lf[S]], lf[S]), f"a label that does not label itself at sweep {t}"
        s_new = a.spins()
        want = orc.flip_at(q, model, seed, t, lf[S].view(np.int32), s.reshape(-1)[S])  # (uint32 words)
        assert np.array_equal(s_new.reshape(-1)[S], want), f"flipped values differ at sweep {t}"
        del lab, lf
        s = s_new
    _say(f"[max size] {model}: the same sweeps in one call")
    b = swmc.Lattice(L, q, model, T=T, seed=seed)
    b.sweep(nsw)
    assert np.array_equal(b.spins(), s), "the one-call run ends in another state"
    _say(f"[max size] {model}: one measured sweep of each")
    b.sweep(1, measure=True)
    a.sweep(1, measure=True)
    sb = b.spins()
    assert np.array_equal(a.spins(), sb)
    ob = b.measure()
    hist, pair = _counts(sb, q)
    assert ob["t"] == nsw + 1 and ob["samples"] == 1
    assert np.array_equal(ob["hist"], hist) and np.array_equal(ob["pair_hist"], pair)
    assert int(hist.sum()) == N and int(pair.sum()) == 2 * N
    a.close()
    b.close()
