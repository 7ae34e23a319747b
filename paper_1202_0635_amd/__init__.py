"""MI355X-native Swendsen-Wang multi-cluster sweep for 2D Potts and clock models.

Method: Komura & Okabe, arXiv:1202.0635 -- Sec. 2 (the three SW steps), Sec. 3
(cluster labeling on a GPU), Sec. 4 (clock model via embedded clusters,
observables M^2 and the moment ratio).  The sweep runs in hand-written HIP
kernels of libswmc.so (include/sw.h); this module only marshals arguments.
PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from . import _lib
from ._lib import (SW_CLOCK, SW_HASH, SW_MEASURE, SW_NO_GRAPH, SW_POTTS, SW_PROFILE, SW_VERIFY, SwError, SwLattice,
                   SwObs, check)

__all__ = ["Lattice", "Batch", "SwError", "critical_temperature", "cutoff_table", "state_bytes", "sweep_static",
           "SW_MEASURE", "SW_VERIFY", "SW_PROFILE", "SW_NO_GRAPH", "SW_HASH"]

MODELS = {"potts": SW_POTTS, "clock": SW_CLOCK}


def critical_temperature(model: str, q: int) -> float:
    """Potts: T_c/J = 1/ln(1+sqrt q) (Sec. 4, printed for q = 2, 3).  Clock q = 6:
    the upper KT temperature T_2/J ~ 0.9 quoted in Sec. 4."""
    if model == "potts":
        return 1.0 / math.log(1.0 + math.sqrt(q))
    if model == "clock" and q == 6:
        return 0.9
    raise ValueError("no critical temperature for this model/q")


def _lattice(L, q, model, T, J, seed) -> SwLattice:
    m = MODELS[model] if isinstance(model, str) else int(model)
    return SwLattice(int(L), int(q), m, 0, float(T), float(J), int(seed) & (2**64 - 1))


def state_bytes(L, q, model="potts", T=1.0, J=1.0, seed=0) -> int:
    return int(_lib.lib().sw_state_bytes(ctypes.byref(_lattice(L, q, model, T, J, seed))))


def cutoff_table(L, q, model="potts", T=1.0, J=1.0) -> np.ndarray:
    """The host FP64 -> uint32 cutoff table of the bond rule (no GPU needed)."""
    p = _lattice(L, q, model, T, J, 0)
    n = q * q if p.model == SW_POTTS else q * q * q
    out = np.zeros(n, dtype=np.uint32)
    check(_lib.lib().sw_cutoff_table(ctypes.byref(p), out.ctypes.data_as(ctypes.c_void_p), n), "sw_cutoff_table")
    return out


STATIC_MAX_L = 1024


def sweep_static(spins, L, q, model="potts", T=None, J=1.0, seed=0, t=0, nsweeps=1, table=None, labels=None,
                 fault=None, stream=None):
    """nsweeps sweeps of the state `spins` (a torch int8 CUDA tensor of L*L
    sites at sweep index t, replaced in place) through sw_sweep_static, which
    allocates no device memory.  table: torch CUDA tensor of the cutoff table
    (int32 or uint32 words); labels: optional torch int32 CUDA tensor [L*L]
    for the last sweep's canonical labels; fault: optional torch int32 CUDA
    tensor [1].  Enqueued on `stream` (default: torch's current stream)."""
    import torch

    if T is None:
        T = critical_temperature(model, q)
    p = _lattice(L, q, model, T, J, seed)
    s = stream if stream is not None else torch.cuda.current_stream(spins.device)

    def ptr(x):
        return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)

    check(_lib.lib().sw_sweep_static(ctypes.byref(p), ptr(spins), int(t), int(nsweeps), ptr(table), ptr(labels),
                                     ptr(fault), ctypes.c_void_p(s.cuda_stream)), "sw_sweep_static")


class Lattice:
    """One L x L periodic lattice resident in device memory.

    Device memory is a torch uint8 tensor on the current CUDA (HIP) device; the
    kernels run on the current torch stream at construction time."""

    def __init__(self, L: int, q: int, model: str = "potts", T: float | None = None, J: float = 1.0,
                 seed: int = 0, device=None, stream=None):
        import torch

        if T is None:
            T = critical_temperature(model, q)
        self.L, self.q, self.model, self.T, self.J, self.seed = int(L), int(q), model, float(T), float(J), int(seed)
        self._p = _lattice(L, q, model, T, J, seed)
        lib = _lib.lib()
        nbytes = int(lib.sw_state_bytes(ctypes.byref(self._p)))
        if nbytes == 0:
            check(_lib.SW_EINVAL, "sw_state_bytes")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        base = self._arena.data_ptr()
        aligned = (base + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(dev)
        ctx = ctypes.c_void_p()
        with torch.cuda.device(dev):
            check(lib.sw_init(ctypes.byref(self._p), ctypes.c_void_p(aligned), nbytes,
                              ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(ctx)), "sw_init")
        self._ctx = ctx
        self.N = self.L * self.L

    # -- sweeps ------------------------------------------------------------
    def sweep(self, n: int = 1, measure: bool = False, verify: bool = False, profile: bool = False,
              hash: bool = False):
        flags = ((SW_MEASURE if measure else 0) | (SW_VERIFY if verify else 0) | (SW_PROFILE if profile else 0)
                 | (SW_HASH if hash else 0))
        check(_lib.lib().sw_sweep(self._ctx, int(n), flags), "sw_sweep")
        return self

    def hashes(self) -> np.ndarray:
        """Per-sweep state hashes recorded by sweeps run with hash=True since
        the last read: rows (t, hash_spins, hash_labels), uint64."""
        return _read_hashes(lambda out, cap, n: _lib.lib().sw_read_hashes(self._ctx, out, cap, n), "sw_read_hashes")

    def measure(self) -> dict:
        o = SwObs()
        check(_lib.lib().sw_measure(self._ctx, ctypes.byref(o)), "sw_measure")
        return _obs_dict(o, self.q)

    # -- state ---------------------------------------------------------------
    def spins(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int8)
        check(_lib.lib().sw_read_spins(self._ctx, out.ctypes.data_as(ctypes.c_void_p), self.N), "sw_read_spins")
        return out.reshape(self.L, self.L)

    def labels(self) -> np.ndarray:
        out = np.zeros(self.N, dtype=np.int32)
        check(_lib.lib().sw_read_labels(self._ctx, out.ctypes.data_as(ctypes.c_void_p), self.N), "sw_read_labels")
        # site indices reach 2^31 above L = 46340: the words are unsigned
        return out.reshape(self.L, self.L).view(np.uint32) if self.L > 46340 else out.reshape(self.L, self.L)

    def bonds(self):
        r = np.zeros(self.N, dtype=np.uint8)
        d = np.zeros(self.N, dtype=np.uint8)
        check(_lib.lib().sw_read_bonds(self._ctx, r.ctypes.data_as(ctypes.c_void_p),
                                       d.ctypes.data_as(ctypes.c_void_p), self.N), "sw_read_bonds")
        return r.reshape(self.L, self.L), d.reshape(self.L, self.L)

    def set_spins(self, spins, t: int = 0):
        s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1)
        check(_lib.lib().sw_write_spins(self._ctx, s.ctypes.data_as(ctypes.c_void_p), s.size, int(t)),
              "sw_write_spins")
        return self

    def spins_device(self):
        """torch int8 view [L, L] of the device spin array (no copy)."""
        import torch

        ptr = ctypes.c_void_p()
        check(_lib.lib().sw_device_spins(self._ctx, ctypes.byref(ptr)), "sw_device_spins")
        off = ptr.value - self._arena.data_ptr()
        return self._arena[off: off + self.N].view(torch.int8).view(self.L, self.L)

    def profile(self) -> dict:
        names = (ctypes.c_char_p * 32)()
        launches = (ctypes.c_int64 * 32)()
        ms = (ctypes.c_double * 32)()
        nk = ctypes.c_int32()
        check(_lib.lib().sw_profile_read(self._ctx, names, launches, ms, 32, ctypes.byref(nk)), "sw_profile_read")
        return {names[k].decode(): (int(launches[k]), float(ms[k])) for k in range(nk.value)}

    LABELERS = {"union_find": 0, "hawick": 1, "kalentev": 2}

    def set_labeler(self, labeler):
        """Cluster labeler (Sec. 3): "union_find" (default), or the paper's
        label-equivalence labelers "hawick" and "kalentev" (an ablation)."""
        code = self.LABELERS[labeler] if isinstance(labeler, str) else int(labeler)
        check(_lib.lib().sw_set_labeler(self._ctx, code), "sw_set_labeler")
        return self

    def labeler_stats(self) -> dict:
        it, sw = ctypes.c_uint64(), ctypes.c_uint64()
        check(_lib.lib().sw_labeler_stats(self._ctx, ctypes.byref(it), ctypes.byref(sw)), "sw_labeler_stats")
        return {"iterations": int(it.value), "sweeps": int(sw.value)}

    def set_tile_waves(self, waves: int):
        """Waves per 64 x 64 tile of the bond kernel (4 or 8); results do not depend on it."""
        check(_lib.lib().sw_set_tile_waves(self._ctx, int(waves)), "sw_set_tile_waves")
        return self

    def tune(self, sweeps: int = 5) -> int:
        out = ctypes.c_int32()
        check(_lib.lib().sw_tune(self._ctx, int(sweeps), ctypes.byref(out)), "sw_tune")
        return int(out.value)

    def synchronize(self):
        self._stream.synchronize()

    def close(self):
        if getattr(self, "_ctx", None):
            _lib.lib().sw_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _read_hashes(call, where) -> np.ndarray:
    rows = []
    cap = 4096
    while True:
        out = np.zeros(3 * cap, dtype=np.uint64)
        n = ctypes.c_size_t()
        check(call(out.ctypes.data_as(ctypes.c_void_p), cap, ctypes.byref(n)), where)
        rows.append(out[: 3 * n.value].reshape(-1, 3))
        if n.value < cap:
            return np.concatenate(rows) if rows else np.zeros((0, 3), dtype=np.uint64)


def _obs_dict(o: SwObs, q: int) -> dict:
    return {
        "t": int(o.sweeps_done), "samples": int(o.samples),
        "hist": np.array(o.hist[:q], dtype=np.int64), "pair_hist": np.array(o.pair_hist[:q], dtype=np.int64),
        "e": o.e_per_site, "m2": o.m2, "mean_e": o.mean_e, "mean_m2": o.mean_m2,
        "mean_m4": o.mean_m4, "binder_u": o.binder_u,
        # clock model (Sec. 4): correlation counts and G at r = L/4 and L/2, R = <G(L/2)>/<G(L/4)>
        "corr_hist": np.array([o.corr_hist[0][:q], o.corr_hist[1][:q]], dtype=np.int64),
        "g_quarter": o.g_quarter, "g_half": o.g_half, "mean_g_quarter": o.mean_g_quarter,
        "mean_g_half": o.mean_g_half, "corr_ratio": o.corr_ratio,
        "absm": o.absm, "hash_spins": int(o.hash_spins), "hash_labels": int(o.hash_labels),
    }


class Batch:
    """Many independent lattices swept together (one launch per phase for all
    of them, a captured hipGraph per sweep).  `specs` is a list of dicts or
    tuples (L, q, model, T, J, seed)."""

    def __init__(self, specs, device=None, stream=None):
        import torch

        ps = []
        self.specs = []
        for sp in specs:
            if isinstance(sp, dict):
                L, q, model = sp["L"], sp["q"], sp.get("model", "potts")
                T = sp.get("T") or critical_temperature(model, q)
                J, seed = sp.get("J", 1.0), sp.get("seed", 0)
            else:
                L, q, model, T, J, seed = sp
            self.specs.append((int(L), int(q), model, float(T), float(J), int(seed)))
            ps.append(_lattice(L, q, model, T, J, seed))
        n = len(ps)
        self._ps = (SwLattice * n)(*ps)
        lib = _lib.lib()
        nbytes = int(lib.sw_batch_bytes(self._ps, n))
        if nbytes == 0:
            check(_lib.SW_EINVAL, "sw_batch_bytes")
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self._arena = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        aligned = (self._arena.data_ptr() + 255) // 256 * 256
        self._stream = stream if stream is not None else torch.cuda.current_stream(dev)
        b = ctypes.c_void_p()
        with torch.cuda.device(dev):
            check(lib.sw_batch_init(self._ps, n, ctypes.c_void_p(aligned), nbytes,
                                    ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(b)), "sw_batch_init")
        self._b = b
        self.n = n

    def __len__(self):
        return self.n

    def sweep(self, n: int = 1, measure: bool = False, verify: bool = False, profile: bool = False,
              graph: bool = True, hash: bool = False):
        flags = ((SW_MEASURE if measure else 0) | (SW_VERIFY if verify else 0) | (SW_PROFILE if profile else 0)
                 | (0 if graph else SW_NO_GRAPH) | (SW_HASH if hash else 0))
        check(_lib.lib().sw_batch_sweep(self._b, int(n), flags), "sw_batch_sweep")
        return self

    def hashes(self, r: int) -> np.ndarray:
        """Replica r's per-sweep hashes (rows t, hash_spins, hash_labels) since the last read."""
        return _read_hashes(lambda out, cap, n: _lib.lib().sw_batch_read_hashes(self._b, int(r), out, cap, n),
                            "sw_batch_read_hashes")

    def measure(self, r: int) -> dict:
        o = SwObs()
        check(_lib.lib().sw_batch_measure(self._b, int(r), ctypes.byref(o)), "sw_batch_measure")
        return _obs_dict(o, self.specs[r][1])

    def spins(self, r: int) -> np.ndarray:
        L = self.specs[r][0]
        out = np.zeros(L * L, dtype=np.int8)
        check(_lib.lib().sw_batch_read_spins(self._b, int(r), out.ctypes.data_as(ctypes.c_void_p), L * L),
              "sw_batch_read_spins")
        return out.reshape(L, L)

    def labels(self, r: int) -> np.ndarray:
        L = self.specs[r][0]
        out = np.zeros(L * L, dtype=np.int32)
        check(_lib.lib().sw_batch_read_labels(self._b, int(r), out.ctypes.data_as(ctypes.c_void_p), L * L),
              "sw_batch_read_labels")
        return out.reshape(L, L)

    def set_schedule(self, merge_tiles: int):
        check(_lib.lib().sw_batch_set_schedule(self._b, int(merge_tiles)), "sw_batch_set_schedule")
        return self

    def set_tile_waves(self, waves: int):
        check(_lib.lib().sw_batch_set_tile_waves(self._b, int(waves)), "sw_batch_set_tile_waves")
        return self

    def tune(self, sweeps: int = 5) -> tuple:
        """(merge schedule, waves per tile) the autotuner keeps."""
        mt, w = ctypes.c_int32(), ctypes.c_int32()
        check(_lib.lib().sw_batch_tune(self._b, int(sweeps), ctypes.byref(mt), ctypes.byref(w)), "sw_batch_tune")
        return int(mt.value), int(w.value)

    def profile(self) -> dict:
        names = (ctypes.c_char_p * 8)()
        launches = (ctypes.c_int64 * 8)()
        ms = (ctypes.c_double * 8)()
        nk = ctypes.c_int32()
        check(_lib.lib().sw_batch_profile_read(self._b, names, launches, ms, 8, ctypes.byref(nk)),
              "sw_batch_profile_read")
        return {names[k].decode(): (int(launches[k]), float(ms[k])) for k in range(nk.value)}

    def synchronize(self):
        self._stream.synchronize()

    def close(self):
        if getattr(self, "_b", None):
            _lib.lib().sw_batch_free(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
