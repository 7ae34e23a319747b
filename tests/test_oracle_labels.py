"""Pins of the oracle's Hoshen-Kopelman labeling (Sec. 2).

The canonical label of a site is the smallest site index of its cluster (the
paper's proper label is the smallest label).  Labeling is reduced to a library
routine -- scipy's connected components on the periodic bond graph -- plus a
numpy minimum per component, and to brute-force breadth-first search on tiny
lattices.
"""
from collections import deque

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def scipy_canonical(L, br, bd):
    n = L * L
    idx = np.arange(n).reshape(L, L)
    right = np.roll(idx, -1, axis=1)
    down = np.roll(idx, -1, axis=0)
    src = np.concatenate([idx[br.astype(bool)], idx[bd.astype(bool)]])
    dst = np.concatenate([right[br.astype(bool)], down[bd.astype(bool)]])
    g = coo_matrix((np.ones(src.size), (src, dst)), shape=(n, n))
    ncomp, comp = connected_components(g, directed=False)
    mins = np.full(ncomp, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp].reshape(L, L).astype(np.int32), ncomp


def bfs_canonical(L, br, bd):
    n = L * L
    adj = [[] for _ in range(n)]
    for y in range(L):
        for x in range(L):
            i = y * L + x
            if br[y, x]:
                j = y * L + (x + 1) % L
                adj[i].append(j)
                adj[j].append(i)
            if bd[y, x]:
                j = ((y + 1) % L) * L + x
                adj[i].append(j)
                adj[j].append(i)
    lab = [-1] * n
    for s in range(n):  # increasing order: the first visit of a cluster is its minimum
        if lab[s] >= 0:
            continue
        lab[s] = s
        dq = deque([s])
        while dq:
            u = dq.popleft()
            for v in adj[u]:
                if lab[v] < 0:
                    lab[v] = s
                    dq.append(v)
    return np.array(lab, dtype=np.int32).reshape(L, L)


@pytest.mark.parametrize("L", [2, 3, 4, 5, 7, 16, 33, 64, 100])
@pytest.mark.parametrize("density", [0.0, 0.3, 0.5, 0.6, 0.9, 1.0])
def test_labels_match_scipy(orc, L, density):
    rng = np.random.default_rng(L * 1000 + int(density * 100))
    for _ in range(3):
        br = (rng.random((L, L)) < density).astype(np.uint8)
        bd = (rng.random((L, L)) < density).astype(np.uint8)
        lab = orc.label(L, br, bd)
        ref, _ = scipy_canonical(L, br, bd)
        assert np.array_equal(lab, ref)


@pytest.mark.parametrize("L", [2, 3, 4, 6])
def test_labels_match_bfs(orc, L):
    rng = np.random.default_rng(99 + L)
    for _ in range(50):
        d = rng.random()
        br = (rng.random((L, L)) < d).astype(np.uint8)
        bd = (rng.random((L, L)) < d).astype(np.uint8)
        assert np.array_equal(orc.label(L, br, bd), bfs_canonical(L, br, bd))


def test_labels_special_cases(orc):
    L = 9
    z = np.zeros((L, L), np.uint8)
    o = np.ones((L, L), np.uint8)
    assert np.array_equal(orc.label(L, z, z).reshape(-1), np.arange(L * L))
    assert np.all(orc.label(L, o, o) == 0)
    # A horizontal stripe closed only through the periodic wrap bond: row 4,
    # bonds everywhere except between x=2 and x=3; the wrap joins x=8 to x=0,
    # so the whole row is one cluster with minimum at x=0.
    br = z.copy()
    br[4, :] = 1
    br[4, 2] = 0
    lab = orc.label(L, br, z)
    assert np.all(lab[4] == 4 * L)
    # A vertical stripe through the bottom wrap bond joins row 8 to row 0.
    bd = z.copy()
    bd[:, 5] = 1
    bd[3, 5] = 0
    lab = orc.label(L, z, bd)
    assert np.all(lab[:, 5] == 5)
    # L = 2: the two right bonds of a row join the same pair (a multigraph).
    L2z = np.zeros((2, 2), np.uint8)
    br2 = L2z.copy()
    br2[0, 1] = 1  # only the wrap bond of row 0
    lab = orc.label(2, br2, L2z)
    assert lab.reshape(-1).tolist() == [0, 0, 2, 3]


def test_spiral_and_comb(orc):
    # Adversarial shapes for label chasing: a spiral and a comb.
    L = 31
    br = np.zeros((L, L), np.uint8)
    bd = np.zeros((L, L), np.uint8)
    # comb: a spine along row 30 (through the wrap), teeth going up every other column
    br[30, :] = 1
    for x in range(0, L, 2):
        bd[0:29, x] = 1
        bd[29, x] = 1
    ref, _ = scipy_canonical(L, br, bd)
    assert np.array_equal(orc.label(L, br, bd), ref)
    # spiral
    br[:] = 0
    bd[:] = 0
    x0, y0, x1, y1 = 0, 0, L - 1, L - 1
    while x0 < x1 and y0 < y1:
        br[y0, x0:x1] = 1
        bd[y0:y1, x1] = 1
        br[y1, x0 + 1:x1] = 1
        bd[y0 + 2:y1, x0] = 1
        x0 += 2
        y0 += 2
        x1 -= 2
        y1 -= 2
    ref, _ = scipy_canonical(L, br, bd)
    assert np.array_equal(orc.label(L, br, bd), ref)


def test_labels_of_real_bonds(orc):
    # Bonds drawn by the oracle itself at the Ising critical point.
    L = 128
    T = 1.0 / np.log(1.0 + np.sqrt(2.0))
    ch = orc.Chain(L, 2, "potts", T=T, seed=11)
    ch.sweep(5)
    ref, ncomp = scipy_canonical(L, ch.bond_r.reshape(L, L), ch.bond_d.reshape(L, L))
    assert np.array_equal(ch.labels.reshape(L, L), ref)
    assert ch.clusters == ncomp
