"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE).

The oracle is the plain sequential Swendsen-Wang sweep of Komura & Okabe
(arXiv:1202.0635, Sec. 2 procedure with Hoshen-Kopelman labeling; Sec. 4 clock
model with embedded clusters).  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module; the product package never
does.  The arithmetic lives in ``sw_oracle.c``; this file only marshals arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sw_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sw.so")

POTTS = 0
CLOCK = 1
MODELS = {"potts": POTTS, "clock": CLOCK}


# Plain ISO C11 (no fast-math: floating point follows the source order, so
# -O3 changes no result), libm.
BUILD_FLAGS = "gcc -std=c11 -O3"


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (BUILD_FLAGS, libm)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            [*BUILD_FLAGS.split(), "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        i8p = ctypes.POINTER(ctypes.c_int8)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        i32p = ctypes.POINTER(ctypes.c_int32)
        i64p = ctypes.POINTER(ctypes.c_int64)
        f64p = ctypes.POINTER(ctypes.c_double)
        c_int, c_u64, c_i64, c_dbl, c_u32 = (
            ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32)
        sig = {
            "or_philox4x32_10": (None, [u32p, u32p, u32p]),
            "or_draw": (None, [c_u64, c_u32, c_u64, c_u32, u32p]),
            "or_qmap": (c_u32, [c_u32, c_u32]),
            "or_table_size": (c_int, [c_int, c_int]),
            "or_cutoffs": (c_int, [c_int, c_int, c_dbl, c_dbl, u32p]),
            "or_clock_projection": (c_dbl, [c_int, c_int, c_int, c_int]),
            "or_init": (None, [c_int, c_int, c_u64, i8p]),
            "or_mirror": (c_int, [c_int, c_u64, c_u64]),
            "or_bonds": (None, [c_int, c_int, c_int, u32p, c_u64, c_u64, i8p, u8p, u8p]),
            "or_bonds_at": (None, [c_int, c_int, c_int, u32p, c_u64, c_u64, i8p, c_i64, i64p, u8p, u8p]),
            "or_label": (None, [c_int, u8p, u8p, i32p]),
            "or_flip": (None, [c_int, c_int, c_int, c_u64, c_u64, i32p, i8p]),
            "or_flip_at": (None, [c_int, c_int, c_u64, c_u64, c_i64, i32p, i8p, i8p]),
            "or_sweep": (c_i64, [c_int, c_int, c_int, u32p, c_u64, c_u64, i8p, u8p, u8p, i32p]),
            "or_counts": (None, [c_int, c_int, i8p, i64p, i64p]),
            "or_corr_counts": (None, [c_int, c_int, i8p, c_int, i64p]),
            "or_corr_g": (c_dbl, [c_int, c_int, i64p]),
            "or_observables": (None, [c_int, c_int, c_int, c_dbl, i64p, i64p, f64p, f64p]),
            "or_run": (c_int, [c_int, c_int, c_int, c_dbl, c_dbl, c_u64, c_i64, c_i64, i8p, f64p, f64p]),
            "or_transition_counts": (c_int, [c_int, c_int, c_int, c_dbl, c_dbl, i8p, c_u64, c_u64, c_i64, i64p]),
            "or_mix64": (c_u64, [c_u64]),
            "or_hash_spins": (c_u64, [c_i64, i8p]),
            "or_hash_labels": (c_u64, [c_i64, i32p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def model_id(model) -> int:
    return MODELS[model] if isinstance(model, str) else int(model)


def philox(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def draw(seed: int, c0: int, t: int, purpose: int) -> np.ndarray:
    out = np.zeros(4, dtype=np.uint32)
    lib().or_draw(seed, c0, t, purpose, _p(out, ctypes.c_uint32))
    return out


def qmap(w: int, q: int) -> int:
    return int(lib().or_qmap(w, q))


def cutoffs(model, q: int, T: float, J: float = 1.0) -> np.ndarray:
    m = model_id(model)
    n = lib().or_table_size(m, q)
    if n < 0:
        raise ValueError("invalid model/q")
    tab = np.zeros(n, dtype=np.uint32)
    if lib().or_cutoffs(m, q, T, J, _p(tab, ctypes.c_uint32)) < 0:
        raise ValueError("invalid T/J")
    return tab


def clock_projection(q: int, a: int, b: int, m: int) -> float:
    return float(lib().or_clock_projection(q, a, b, m))


def init(L: int, q: int, seed: int) -> np.ndarray:
    s = np.zeros(L * L, dtype=np.int8)
    lib().or_init(L, q, seed, _p(s, ctypes.c_int8))
    return s.reshape(L, L)


def mirror(q: int, seed: int, t: int) -> int:
    return int(lib().or_mirror(q, seed, t))


def bonds(L, q, model, table, seed, t, spins):
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    br = np.zeros(L * L, dtype=np.uint8)
    bd = np.zeros(L * L, dtype=np.uint8)
    lib().or_bonds(L, q, model_id(model), _p(table, ctypes.c_uint32), seed, t,
                   _p(s, ctypes.c_int8), _p(br, ctypes.c_uint8), _p(bd, ctypes.c_uint8))
    return br.reshape(L, L), bd.reshape(L, L)


def bonds_at(L, q, model, table, seed, t, spins, sites):
    """Bonds owned by the given row-major sites (Sec. 2 steps (i)-(iii)), from the whole state."""
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    assert s.size == L * L
    idx = np.ascontiguousarray(sites, dtype=np.int64).reshape(-1)
    br = np.zeros(idx.size, dtype=np.uint8)
    bd = np.zeros(idx.size, dtype=np.uint8)
    lib().or_bonds_at(L, q, model_id(model), _p(table, ctypes.c_uint32), seed, t, _p(s, ctypes.c_int8),
                      idx.size, _p(idx, ctypes.c_int64), _p(br, ctypes.c_uint8), _p(bd, ctypes.c_uint8))
    return br, bd


def label(L, bond_r, bond_d) -> np.ndarray:
    br = np.ascontiguousarray(bond_r, dtype=np.uint8).reshape(-1)
    bd = np.ascontiguousarray(bond_d, dtype=np.uint8).reshape(-1)
    lab = np.zeros(L * L, dtype=np.int32)
    lib().or_label(L, _p(br, ctypes.c_uint8), _p(bd, ctypes.c_uint8), _p(lab, ctypes.c_int32))
    return lab.reshape(L, L)


def flip(L, q, model, seed, t, labels, spins) -> np.ndarray:
    s = np.array(spins, dtype=np.int8).reshape(-1)
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    lib().or_flip(L, q, model_id(model), seed, t, _p(lab, ctypes.c_int32), _p(s, ctypes.c_int8))
    return s.reshape(L, L)


def flip_at(q, model, seed, t, roots, old):
    """New values of single sites (Sec. 2 steps (v)-(vii)): site k belongs to
    the cluster whose canonical label is roots[k] and had value old[k]."""
    r = np.ascontiguousarray(roots, dtype=np.int32).reshape(-1)
    o = np.ascontiguousarray(old, dtype=np.int8).reshape(-1)
    out = np.zeros(r.size, dtype=np.int8)
    lib().or_flip_at(q, model_id(model), seed, t, r.size, _p(r, ctypes.c_int32), _p(o, ctypes.c_int8),
                     _p(out, ctypes.c_int8))
    return out


class Chain:
    """A lattice state advanced sweep by sweep by the oracle."""

    def __init__(self, L: int, q: int, model="potts", T: float = 1.0, J: float = 1.0,
                 seed: int = 0, spins=None, t: int = 0):
        self.L, self.q, self.model, self.T, self.J, self.seed = L, q, model_id(model), T, J, seed
        self.table = cutoffs(self.model, q, T, J)
        self.spins = (init(L, q, seed).reshape(-1).copy() if spins is None
                      else np.array(spins, dtype=np.int8).reshape(-1).copy())
        self.t = t
        n = L * L
        self.bond_r = np.zeros(n, dtype=np.uint8)
        self.bond_d = np.zeros(n, dtype=np.uint8)
        self.labels = np.zeros(n, dtype=np.int32)
        self.clusters = 0

    def sweep(self, n: int = 1):
        for _ in range(n):
            self.clusters = lib().or_sweep(
                self.L, self.q, self.model, _p(self.table, ctypes.c_uint32), self.seed, self.t,
                _p(self.spins, ctypes.c_int8), _p(self.bond_r, ctypes.c_uint8),
                _p(self.bond_d, ctypes.c_uint8), _p(self.labels, ctypes.c_int32))
            self.t += 1
        return self

    def corr_counts(self):
        """Correlation counts of the current state at r = L/4 and r = L/2 (Sec. 4)."""
        return corr_counts(self.L, self.q, self.spins, self.L // 4), corr_counts(self.L, self.q, self.spins, self.L // 2)

    def counts(self):
        h = np.zeros(32, dtype=np.int64)
        p = np.zeros(32, dtype=np.int64)
        lib().or_counts(self.L, self.q, _p(self.spins, ctypes.c_int8), _p(h, ctypes.c_int64),
                        _p(p, ctypes.c_int64))
        return h[: self.q].copy(), p[: self.q].copy()

    def observables(self):
        h, p = self.counts()
        h32 = np.zeros(32, dtype=np.int64)
        p32 = np.zeros(32, dtype=np.int64)
        h32[: self.q] = h
        p32[: self.q] = p
        e = ctypes.c_double()
        m2 = ctypes.c_double()
        lib().or_observables(self.L, self.q, self.model, self.J, _p(h32, ctypes.c_int64),
                             _p(p32, ctypes.c_int64), ctypes.byref(e), ctypes.byref(m2))
        return e.value, m2.value


def corr_counts(L, q, spins, r) -> np.ndarray:
    """Histogram of (s_{i+r} - s_i) mod q over both directions (2N pairs), Sec. 4."""
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    h = np.zeros(32, dtype=np.int64)
    lib().or_corr_counts(L, q, _p(s, ctypes.c_int8), int(r), _p(h, ctypes.c_int64))
    return h[:q].copy()


def corr_g(L, q, corr_hist) -> float:
    """G(r) = <S_i . S_{i+r}> from the correlation counts (Sec. 4)."""
    h = np.zeros(32, dtype=np.int64)
    h[: len(corr_hist)] = corr_hist
    return float(lib().or_corr_g(L, q, _p(h, ctypes.c_int64)))


def observables_from_counts(L, q, model, J, hist, pair_hist):
    h32 = np.zeros(32, dtype=np.int64)
    p32 = np.zeros(32, dtype=np.int64)
    h32[:q] = hist
    p32[:q] = pair_hist
    e = ctypes.c_double()
    m2 = ctypes.c_double()
    lib().or_observables(L, q, model_id(model), J, _p(h32, ctypes.c_int64), _p(p32, ctypes.c_int64),
                         ctypes.byref(e), ctypes.byref(m2))
    return e.value, m2.value


def run(L, q, model, T, J, seed, n_therm, n_meas):
    """Chain from the random start; returns (e[n_meas], m2[n_meas], final spins)."""
    s = np.zeros(L * L, dtype=np.int8)
    e = np.zeros(max(n_meas, 1), dtype=np.float64)
    m2 = np.zeros(max(n_meas, 1), dtype=np.float64)
    rc = lib().or_run(L, q, model_id(model), T, J, seed, n_therm, n_meas, _p(s, ctypes.c_int8),
                      _p(e, ctypes.c_double), _p(m2, ctypes.c_double))
    if rc != 0:
        raise ValueError("or_run rejected its parameters")
    return e[:n_meas], m2[:n_meas], s.reshape(L, L)


def transition_counts(L, q, model, T, J, s0, t, seed0, nseeds) -> np.ndarray:
    s = np.ascontiguousarray(s0, dtype=np.int8).reshape(-1)
    counts = np.zeros(q ** (L * L), dtype=np.int64)
    rc = lib().or_transition_counts(L, q, model_id(model), T, J, _p(s, ctypes.c_int8), t, seed0,
                                    nseeds, _p(counts, ctypes.c_int64))
    if rc != 0:
        raise ValueError("or_transition_counts rejected its parameters")
    return counts


def hash_spins(spins) -> int:
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
    return int(lib().or_hash_spins(s.size, _p(s, ctypes.c_int8)))


def hash_labels(labels) -> int:
    lab = np.ascontiguousarray(labels, dtype=np.int32).reshape(-1)
    return int(lib().or_hash_labels(lab.size, _p(lab, ctypes.c_int32)))
