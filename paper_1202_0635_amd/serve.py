"""Serving: continuous batching of Swendsen-Wang simulation requests.

`Server` wraps the C-ABI server of libswmc (admission by device-memory
budget, lattice states resident on the device, batched sweeps over all active
lattices, retirement of finished ones).  `run_trace` replays a request trace
with Poisson arrivals against it; `run_plain` replays the same trace through
the one-lattice-per-launch path (first come, first served) for comparison.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import MODELS, Lattice, _lib
from ._lib import SwRequest, SwResult, SwServerStats, check

__all__ = ["Server", "run_trace", "run_plain", "spin_hash", "poisson_arrivals"]

_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def spin_hash(spins) -> int:
    """sum_i mix64((i << 8) | s_i) mod 2^64 with the SplitMix64 output function
    (Steele, Lea & Flood 2014): an order-independent fingerprint of a state,
    on the host (the server and `Lattice.measure` compute it on the device)."""
    s = np.ascontiguousarray(spins, dtype=np.int8).reshape(-1).view(np.uint8).astype(np.uint64)
    z = (np.arange(s.size, dtype=np.uint64) << np.uint64(8)) | s
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return int(z.sum(dtype=np.uint64))


def _result_dict(r: SwResult) -> dict:
    q = 32
    return {
        "tag": int(r.tag), "status": int(r.status), "t": int(r.obs.sweeps_done),
        "hist": np.array(r.obs.hist[:q], dtype=np.int64), "pair_hist": np.array(r.obs.pair_hist[:q], dtype=np.int64),
        "e": r.obs.e_per_site, "m2": r.obs.m2, "spin_hash": int(r.spin_hash),
        "t_arrival": r.t_arrival, "t_admit": r.t_admit, "t_done": r.t_done,
    }


class Server:
    def __init__(self, budget_bytes: int = 2 << 30, max_slots: int = 64, sweeps_per_step: int = 20, stream=None):
        import torch

        self._stream = stream if stream is not None else torch.cuda.current_stream()
        s = ctypes.c_void_p()
        check(_lib.lib().sw_server_create(int(budget_bytes), int(max_slots), int(sweeps_per_step),
                                          ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(s)),
              "sw_server_create")
        self._s = s

    def now(self) -> float:
        return float(_lib.lib().sw_server_now(self._s))

    def submit(self, L, q, model, T, J, seed, sweeps, tag, t_arrival=None):
        from . import _lattice

        req = SwRequest(_lattice(L, q, model, T, J, seed), int(sweeps), int(tag),
                        float(self.now() if t_arrival is None else t_arrival))
        check(_lib.lib().sw_server_submit(self._s, ctypes.byref(req)), "sw_server_submit")

    def step(self) -> int:
        n = ctypes.c_int32()
        check(_lib.lib().sw_server_step(self._s, ctypes.byref(n)), "sw_server_step")
        return int(n.value)

    def poll(self) -> list:
        out = (SwResult * 256)()
        res = []
        while True:
            n = ctypes.c_int32()
            check(_lib.lib().sw_server_poll(self._s, out, 256, ctypes.byref(n)), "sw_server_poll")
            res += [_result_dict(out[i]) for i in range(n.value)]
            if n.value < 256:
                return res

    def stats(self) -> dict:
        st = SwServerStats()
        check(_lib.lib().sw_server_stats_read(self._s, ctypes.byref(st)), "sw_server_stats_read")
        return {f: int(getattr(st, f)) for f, _ in SwServerStats._fields_}

    def close(self):
        if getattr(self, "_s", None):
            _lib.lib().sw_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def poisson_arrivals(n: int, rate: float, seed: int = 7) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate; rate <= 0 or
    inf: everything arrives at t = 0 (saturation)."""
    if not rate or rate <= 0 or not np.isfinite(rate):
        return np.zeros(n)
    return np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))


def _summary(lat: np.ndarray, updates: float, makespan: float) -> dict:
    return {"requests": int(lat.size), "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "makespan_s": makespan, "spin_updates": updates,
            "spin_updates_per_s": updates / makespan if makespan > 0 else float("nan")}


def run_trace(trace, arrivals, budget_bytes=2 << 30, max_slots=64, sweeps_per_step=20, progress=None) -> dict:
    """Continuous batching of `trace` (LatticeConfig list) arriving at `arrivals`."""
    srv = Server(budget_bytes, max_slots, sweeps_per_step)
    order = np.argsort(arrivals, kind="stable")
    t_start = srv.now()
    nxt = 0
    results = {}
    n = len(trace)
    while len(results) < n:
        now = srv.now() - t_start
        while nxt < n and arrivals[order[nxt]] <= now:
            i = int(order[nxt])
            c = trace[i]
            srv.submit(c.L, c.q, c.model, c.T, c.J, c.seed, c.sweeps, tag=i, t_arrival=t_start + arrivals[i])
            nxt += 1
        active = srv.step()
        for r in srv.poll():
            results[r["tag"]] = r
        if active == 0 and nxt < n:
            wait = arrivals[order[nxt]] - (srv.now() - t_start)
            if wait > 0:
                time.sleep(min(wait, 0.05))
        if progress and len(results) and len(results) % 200 == 0:
            progress(len(results))
    makespan = max(r["t_done"] for r in results.values()) - t_start
    lat = np.array([results[i]["t_done"] - results[i]["t_arrival"] for i in range(n)])
    updates = float(sum(c.L * c.L * c.sweeps for c in trace))
    out = _summary(lat, updates, makespan)
    out["stats"] = srv.stats()
    out["results"] = results
    srv.close()
    return out


def run_plain(trace, arrivals) -> dict:
    """The same trace, one lattice per launch, first come first served."""
    import torch

    order = np.argsort(arrivals, kind="stable")
    t0 = time.perf_counter()
    done = {}
    results = {}
    for i in order:
        i = int(i)
        c = trace[i]
        wait = arrivals[i] - (time.perf_counter() - t0)
        if wait > 0:
            time.sleep(wait)
        lat = Lattice(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
        lat.sweep(c.sweeps)
        ob = lat.measure()  # synchronises; counts and the spin hash come from the device, as in the server
        done[i] = time.perf_counter() - t0
        results[i] = {"spin_hash": ob["hash_spins"], "hist": ob["hist"], "pair_hist": ob["pair_hist"],
                      "e": ob["e"], "m2": ob["m2"], "t": ob["t"]}
        lat.close()
    torch.cuda.synchronize()
    makespan = max(done.values())
    lat = np.array([done[i] - arrivals[i] for i in range(len(trace))])
    updates = float(sum(c.L * c.L * c.sweeps for c in trace))
    out = _summary(lat, updates, makespan)
    out["results"] = results
    return out
