"""Exact results for tiny and finite periodic lattices, used to pin the oracle.

Everything here is computed from the model definitions (Sec. 2, Eq. 1 Potts;
Sec. 4 clock) and textbook closed forms, never from the oracle's code:
  * brute-force enumeration of the Boltzmann distribution,
  * the exact one-sweep Swendsen-Wang transition matrix on the 2x2 torus,
  * Kaufman's partition function of the finite L x L Ising torus
    (Kaufman, Phys. Rev. 76, 1232 (1949); in the form of Beale, PRL 76, 78 (1996)).
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def torus_edges(L):
    """The 2N owned bonds (site, right neighbour) and (site, down neighbour)."""
    e = []
    for y in range(L):
        for x in range(L):
            i = y * L + x
            e.append((i, y * L + (x + 1) % L))
            e.append((i, ((y + 1) % L) * L + x))
    return e


def energy_m2(states, L, q, model, J=1.0):
    """Energy per site and normalised M^2 for an array of states [n, N]."""
    N = L * L
    edges = torus_edges(L)
    a = np.array([i for i, _ in edges])
    b = np.array([j for _, j in edges])
    sa = states[:, a].astype(np.int64)
    sb = states[:, b].astype(np.int64)
    if model == "potts":
        H = J * (sa != sb).sum(axis=1)
        n = np.stack([(states == k).sum(axis=1) for k in range(q)], axis=1).astype(np.float64)
        m2 = (q * (n**2).sum(axis=1) - N * N) / ((q - 1) * N * N)
    else:
        H = -J * np.cos(2 * np.pi * (sa - sb) / q).sum(axis=1)
        th = 2 * np.pi * states / q
        m2 = (np.cos(th).sum(axis=1) ** 2 + np.sin(th).sum(axis=1) ** 2) / (N * N)
    return H / N, m2


def exact_averages(L, q, model, T, J=1.0, chunk=1 << 20):
    """<e>, <m2>, <m4> = <m2^2> by enumeration of all q^(L^2) states."""
    N = L * L
    total = q**N
    pw = q ** np.arange(N, dtype=np.int64)
    logw_max = None
    acc = np.zeros(4)
    parts = []
    for start in range(0, total, chunk):
        idx = np.arange(start, min(total, start + chunk), dtype=np.int64)
        states = ((idx[:, None] // pw[None, :]) % q).astype(np.int8)
        e, m2 = energy_m2(states, L, q, model, J)
        logw = -e * N / T
        parts.append((logw, e, m2))
    logw_max = max(p[0].max() for p in parts)
    for logw, e, m2 in parts:
        w = np.exp(logw - logw_max)
        acc += [w.sum(), (w * e).sum(), (w * m2).sum(), (w * m2 * m2).sum()]
    return acc[1] / acc[0], acc[2] / acc[0], acc[3] / acc[0]


def _components(n, edges, subset):
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            x = parent[x]
        return x

    for k in subset:
        i, j = edges[k]
        ri, rj = find(i), find(j)
        if ri != rj:
            parent[max(ri, rj)] = min(ri, rj)
    comp = {}
    for s in range(n):
        comp.setdefault(find(s), []).append(s)
    return list(comp.values())


def sw_transition_matrix(L, q, model, bond_prob):
    """Exact one-sweep SW kernel P[s, s'] on the L x L torus (L = 2 or tiny).

    bond_prob(a, b, m) -> probability that a bond between spins a, b is active
    (for Potts m is ignored).  Potts: every cluster takes a uniform value.
    Clock: the mirror m is uniform over q; each cluster is reflected a -> m - a
    with probability 1/2."""
    N = L * L
    edges = torus_edges(L)
    nE = len(edges)
    n_states = q**N
    subsets = []
    for mask in range(1 << nE):
        sub = [k for k in range(nE) if mask >> k & 1]
        subsets.append((mask, sub, _components(N, edges, sub)))
    P = np.zeros((n_states, n_states))
    pw = [q**i for i in range(N)]
    mirrors = range(q) if model == "clock" else [0]
    for idx in range(n_states):
        s = [(idx // pw[i]) % q for i in range(N)]
        for m in mirrors:
            pe = [bond_prob(s[i], s[j], m) for (i, j) in edges]
            pm = (1.0 / q) if model == "clock" else 1.0
            for mask, sub, comps in subsets:
                w = pm
                for k in range(nE):
                    w *= pe[k] if (mask >> k & 1) else (1.0 - pe[k])
                    if w == 0.0:
                        break
                if w == 0.0:
                    continue
                if model == "potts":
                    # every cluster takes each of the q values with probability 1/q
                    for vals in itertools.product(range(q), repeat=len(comps)):
                        t = [0] * N
                        for c, v in zip(comps, vals):
                            for site in c:
                                t[site] = v
                        P[idx, sum(t[i] * pw[i] for i in range(N))] += w / q ** len(comps)
                else:
                    for flips in itertools.product((0, 1), repeat=len(comps)):
                        t = list(s)
                        for c, f in zip(comps, flips):
                            if f:
                                for site in c:
                                    t[site] = (m - s[site]) % q
                        P[idx, sum(t[i] * pw[i] for i in range(N))] += w / 2 ** len(comps)
    return P


def boltzmann(L, q, model, T, J=1.0):
    N = L * L
    pw = q ** np.arange(N, dtype=np.int64)
    idx = np.arange(q**N, dtype=np.int64)
    states = ((idx[:, None] // pw[None, :]) % q).astype(np.int8)
    e, _ = energy_m2(states, L, q, model, J)
    logw = -e * N / T
    w = np.exp(logw - logw.max())
    return w / w.sum()


def kaufman_logz(L, K):
    """ln Z of the L x L periodic Ising model with Z = sum exp(K sum_<ij> s_i s_j)."""
    n = m = L
    c2, s2 = math.cosh(2 * K), math.sinh(2 * K)

    def gamma(l):
        if l == 0:
            return 2 * K + math.log(math.tanh(K))
        return math.acosh(c2 * c2 / s2 - math.cos(math.pi * l / n))

    def log_prod(kind, parity):
        # ln prod_r 2cosh(m g/2) or ln |prod_r 2sinh(m g/2)| with its sign, using
        # 2cosh(x) = e^|x| (1 + e^-2|x|) and 2|sinh(x)| = e^|x| (1 - e^-2|x|).
        tot, sign = 0.0, 1
        for r in range(n):
            x = m * gamma(2 * r + parity) / 2
            if kind == "cosh":
                tot += abs(x) + math.log1p(math.exp(-2 * abs(x)))
            else:
                if x == 0.0:
                    return -math.inf, 0
                sign *= 1 if x > 0 else -1
                tot += abs(x) + math.log1p(-math.exp(-2 * abs(x)))
        return tot, sign

    terms = [log_prod("cosh", 1), log_prod("sinh", 1), log_prod("cosh", 0), log_prod("sinh", 0)]
    mx = max(t for t, _ in terms if t != -math.inf)
    ssum = sum(sg * math.exp(t - mx) for t, sg in terms if t != -math.inf)
    return math.log(0.5) + 0.5 * n * m * math.log(2 * s2) + mx + math.log(ssum)


def kaufman_bond_sum(L, K, h=1e-6):
    """<sum_<ij> s_i s_j> = d ln Z / dK by a central difference."""
    return (kaufman_logz(L, K + h) - kaufman_logz(L, K - h)) / (2 * h)


def ising_potts_energy(L, T, J=1.0):
    """Exact Potts q=2 energy per site (H = -J sum (delta - 1)) on the L x L
    torus, from Kaufman's Z with Ising coupling K = J / (2T)."""
    K = J / (2.0 * T)
    N = L * L
    return J * (1.0 - kaufman_bond_sum(L, K) / (2.0 * N))


def binned_mean(x, nbins=50):
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // nbins
    b = x[: nb * nbins].reshape(nbins, nb).mean(axis=1)
    return b.mean(), b.std(ddof=1) / math.sqrt(nbins)
