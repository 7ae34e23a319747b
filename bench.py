"""Benchmark: ns per spin update of the Swendsen-Wang sweep on one MI355X.

Default workload: q = 2 Potts (Ising) at T_c = 1/ln(1+sqrt 2), L = 4096,
random start, 200 warm-up (thermalisation) sweeps, then the timed sweeps --
the L = 4096 column of Table 1 (update only).  A "step" is one sweep of the
whole hot path (bonds + labeling + flip) over the lattice resident in HBM.

Prints one JSON line with the metric, a roofline object for the dominant
kernel (algorithmic bytes per launch / HIP-event launch time) and the CPU
oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0          # MI355X HBM3E, 8 TB/s
PAPER_NS_PER_UPDATE = {"potts2_L4096_Tc": 2.51, "clock6_L4096_T0.9": 2.42}  # GTX580, Tables 1 and 3


def alg_bytes_per_launch(kernel: str, L: int, model: str, tile_w: int = 64, tile_h: int = 64,
                         merge_tiles: int = 1) -> float:
    """Algorithmic HBM bytes of one launch (the method's own traffic, perf mode).

    k_bond_local: spins read once (1 B/site) plus the halo column and row of
      every tile (L*L*(1/tile_w + 1/tile_h) B), bonds written (2 bits/site =
      0.25 B/site), labels written (4 B/site).
    k_border_merge, k_flatten: per tile-border site, one bond bit read
      (counted as 1/8 B) and the two label words of its endpoints (8 B).
    k_flip: labels read (4 B/site), spins written (1 B/site); the clock model
      also reads the old spin (1 B/site).
    Single lattices run the same three steps with two-level labels; their
    kernels are booked with the same per-site figures, so the fraction of
    peak measures the method's work, not this layout's (smaller) traffic:
    k_code_bond as k_bond_local, k_code_flip_bond (the previous sweep's flip
    fused with this sweep's bonds and tile labeling) as k_flip + k_bond_local,
    k_node_merge as k_border_merge with one-tile blocks, k_code_flip as k_flip.
    """
    N = float(L) * L
    if kernel == "k_code_bond":
        return alg_bytes_per_launch("k_bond_local", L, model, tile_w, tile_h)
    if kernel == "k_code_flip_bond":
        return (alg_bytes_per_launch("k_flip", L, model, tile_w, tile_h)
                + alg_bytes_per_launch("k_bond_local", L, model, tile_w, tile_h))
    if kernel == "k_node_merge":
        return alg_bytes_per_launch("k_border_merge", L, model, tile_w, tile_h, merge_tiles=1)
    if kernel == "k_code_flip":
        return alg_bytes_per_launch("k_flip", L, model, tile_w, tile_h)
    if kernel == "k_bond_local":
        return N * (1.0 + 1.0 / tile_w + 1.0 / tile_h + 0.25 + 4.0)
    if kernel in ("k_block_merge", "k_border_merge", "k_flatten"):
        mt = merge_tiles
        tiles = (-(-L // tile_w)) + (-(-L // tile_h))
        if kernel == "k_border_merge":   # block borders only (every mt-th tile border, and the wrap)
            tiles = (-(-L // (mt * tile_w))) + (-(-L // (mt * tile_h)))
        elif kernel == "k_block_merge":  # the borders inside the blocks (none for mt = 1)
            tiles -= (-(-L // (mt * tile_w))) + (-(-L // (mt * tile_h)))
        return L * tiles * (0.125 + 8.0)
    if kernel == "k_flip":
        return N * (4.0 + 1.0 + (1.0 if model == "clock" else 0.0))
    if kernel == "k_counts":
        return N * (1.0 + 1.0 / tile_w + 1.0 / tile_h)
    raise KeyError(kernel)


# the kernels of one sweep inside a multi-sweep call
SWEEP_KERNELS = ("k_code_flip_bond", "k_node_merge")
COPY_BYTES = 256 << 20
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1202_0635_amd", "csrc", f)
                  for f in ("sw_kernels.hip", "sw_device.hpp", "sw_internal.hpp")]


def kernel_source_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (profiles/traffic_<kernel>_<workload>.md), or None when there is none or
    the kernel sources changed since the counters were taken."""
    path = os.path.join(PROFILES, f"traffic_{kernel}_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    if fields.get("kernel_source_digest") != kernel_source_digest():
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _profile_fields(path: str) -> dict:
    fields = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                fields[k.strip()] = v.strip().strip("`")
    return fields


def traced_avg_us(kernel: str, workload: str):
    """Average duration (us) of `kernel` in the committed rocprofv3 kernel
    trace (profiles/kernel_trace_<workload>.md), or None when there is none or
    the kernel sources changed since the trace was taken."""
    path = os.path.join(PROFILES, f"kernel_trace_{workload}.md")
    if not os.path.exists(path):
        return None
    fields = _profile_fields(path)
    if fields.get("kernel_source_digest") != kernel_source_digest():
        return None
    try:
        return float(fields[f"avg_us {kernel}"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, budget_s: float) -> dict:
    """The oracle (single thread) on the first sweeps of the same workload."""
    import oracle

    ch = oracle.Chain(cfg.L, cfg.q, cfg.model, T=cfg.T, J=cfg.J, seed=cfg.seed)
    t0 = time.perf_counter()
    n = 0
    while True:
        ch.sweep(1)
        n += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": dt * 1e9 / (n * cfg.L * cfg.L), "unit": "ns/spin-update", "cores": 1, "kind": "oracle",
            "sample": f"first {n} sweeps of {cfg.name} from the random start (single-threaded C oracle)",
            "cpu_model": cpu_model(), "oracle_build": oracle.BUILD_FLAGS}


def bench_batch(args) -> dict:
    """256 q = 3 Potts replicas (L cycling over 64..512, T over [0.9, 1.1] T_c), 500
    sweeps: batched launches, the 500 sweeps captured as one graph launch,
    merge schedule and waves per tile picked by the autotuner, against the
    same replicas swept one lattice per launch."""
    import torch

    import paper_1202_0635_amd as swmc
    from paper_1202_0635_amd.workloads import replica_mix_q3

    reps = replica_mix_q3(args.replicas)
    sweeps = args.steps
    specs = [(c.L, c.q, c.model, c.T, c.J, c.seed) for c in reps]
    sites = sum(c.L * c.L for c in reps)
    b = swmc.Batch(specs)
    mt, waves = b.tune(5)
    b.sweep(args.warmup)
    b.sweep(sweeps)  # captures the run of `sweeps` sweeps (one graph), outside the timed region
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.sweep(sweeps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    b.close()
    # the plain path: one lattice per launch, replicas one after another
    lats = [swmc.Lattice(*sp[:3], T=sp[3], J=sp[4], seed=sp[5]) for sp in specs]
    for lat in lats:
        lat.sweep(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for lat in lats:
        lat.sweep(sweeps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    for lat in lats:
        lat.close()
    return {"metric": "batched vs plain speedup (SW sweep, replica mix)", "value": t_plain / t_batch, "unit": "x",
            "higher_is_better": True, "n_gpus": 1, "steps": sweeps, "warmup": args.warmup, "dtype": "int8",
            "data": "synthetic",
            "config": {"workload": "potts3_replicas_256_L64-512", "replicas": len(reps), "sites": sites,
                       "merge_tiles": mt, "tile_waves": waves, "graph_sweeps": min(sweeps, 512)},
            "batched_spin_updates_per_s": sites * sweeps / t_batch,
            "plain_spin_updates_per_s": sites * sweeps / t_plain,
            "batched_ns_per_update": t_batch * 1e9 / (sites * sweeps), "batched_s": t_batch, "plain_s": t_plain}


def bench_labelers(args) -> dict:
    """The paper's labelers (Sec. 3, label equivalence after Hawick et al. and
    after Kalentev et al.) against the union-find path: ns per spin update and
    iterations per sweep for the Ising model at T_c, L = 256 ... 4096 (the
    sizes of Table 1).  Each lattice is warmed up with the union-find path,
    then every labeler runs the same number of sweeps from there."""
    import paper_1202_0635_amd as swmc

    tc = 1.0 / math.log(1.0 + math.sqrt(2.0))
    rows = []
    for L in (256, 512, 1024, 2048, 4096):
        lat = swmc.Lattice(L, 2, "potts", T=tc, seed=2)
        lat.sweep(args.warmup)
        lat.measure()  # synchronises
        row = {"L": L}
        for name in ("union_find", "kalentev", "hawick"):
            lat.set_labeler(name)
            sweeps = args.steps if name == "union_find" else max(5, args.steps // 20)
            before = lat.labeler_stats()
            t0 = time.perf_counter()
            lat.sweep(sweeps)
            lat.measure()
            dt = time.perf_counter() - t0
            after = lat.labeler_stats()
            row[name] = {"ns_per_update": dt * 1e9 / (L * L * sweeps), "sweeps": sweeps}
            if name != "union_find":
                row[name]["iterations_per_sweep"] = (after["iterations"] - before["iterations"]) / sweeps
            print(f"[labelers] L={L} {name}: {row[name]}", file=sys.stderr, flush=True)
        lat.close()
        rows.append(row)
    big = rows[-1]
    return {"metric": "labeler ablation: ns per spin update, Ising at T_c (union-find vs the paper's labelers)",
            "value": big["kalentev"]["ns_per_update"] / big["union_find"]["ns_per_update"], "unit": "x",
            "higher_is_better": True, "n_gpus": 1, "dtype": "int8", "data": "synthetic",
            "config": {"workload": "potts2_Tc_L256-4096", "warmup": args.warmup, "steps": args.steps},
            "rows": rows}


def bench_tscan(args) -> dict:
    """Temperature dependence of the time per spin update (Figs. 3 and 5: q = 2
    and q = 3 Potts and the q = 6 clock model at L = 1024; also q = 4 Potts and
    the q = 32 clock model, close to the XY model), for the union-find path and
    the label-equivalence labeler of Kalentev et al. (with its iterations per
    sweep), and for the union-find path at L = 4096.  Temperatures are given
    relative to T_c (Potts) or to 0.9 (clock models, near the upper KT
    temperature of q = 6 and the XY model's)."""
    import paper_1202_0635_amd as swmc

    def run(L, q, model, T, labeler, sweeps):
        lat = swmc.Lattice(L, q, model, T=T, seed=3)
        lat.sweep(args.warmup)
        lat.set_labeler(labeler)
        lat.measure()
        before = lat.labeler_stats()
        t0 = time.perf_counter()
        lat.sweep(sweeps)
        lat.measure()
        dt = time.perf_counter() - t0
        it = (lat.labeler_stats()["iterations"] - before["iterations"]) / sweeps
        lat.close()
        return dt * 1e9 / (L * L * sweeps), it

    rows = []
    for q, model, tc in ((2, "potts", 1.0 / math.log(1.0 + math.sqrt(2.0))),
                         (3, "potts", 1.0 / math.log(1.0 + math.sqrt(3.0))),
                         (4, "potts", 1.0 / math.log(3.0)), (6, "clock", 0.9), (32, "clock", 0.9)):
        for f in (0.5, 0.7, 0.85, 0.95, 1.0, 1.05, 1.2, 1.5, 2.0):
            T = tc * f
            row = {"model": model, "q": q, "T": T, "T_over_ref": f}
            row["uf_L1024_ns"], _ = run(1024, q, model, T, "union_find", args.steps)
            row["kalentev_L1024_ns"], row["kalentev_iterations"] = run(1024, q, model, T, "kalentev",
                                                                        max(5, args.steps // 20))
            row["uf_L4096_ns"], _ = run(4096, q, model, T, "union_find", args.steps)
            print(f"[tscan] {row}", file=sys.stderr, flush=True)
            rows.append(row)
    return {"metric": "temperature dependence of ns per spin update (L = 1024 and 4096)", "value": None,
            "unit": "ns/spin-update", "higher_is_better": False, "n_gpus": 1, "dtype": "int8", "data": "synthetic",
            "config": {"workload": "tscan_potts2_potts3_potts4_clock6_clock32", "warmup": args.warmup, "steps": args.steps},
            "rows": rows}


def crossings(temps, curves):
    """Temperatures where the curves of consecutive sizes cross: for each pair,
    the sign changes of their difference on the grid, located by linear
    interpolation (the difference is taken larger size minus smaller)."""
    sizes = sorted(curves)
    out = []
    for a, b in zip(sizes, sizes[1:]):
        d = [curves[b][k] - curves[a][k] for k in range(len(temps))]
        for k in range(len(temps) - 1):
            if d[k] == 0.0 or d[k] * d[k + 1] < 0.0:
                f = 0.0 if d[k] == 0.0 else d[k] / (d[k] - d[k + 1])
                out.append({"L_pair": [a, b], "T": temps[k] + f * (temps[k + 1] - temps[k])})
    return out


def bench_uscan(args) -> dict:
    """Moment ratio U(T) = <M^4>/<M^2>^2 of the q = 2 and q = 3 Potts models
    (Sec. 4, Fig. 4) and the correlation ratio R(T) = G(L/2)/G(L/4) of the q = 6
    clock model (Sec. 4, Fig. 6) on a temperature grid for several sizes.  All
    replicas of a model run in one batch: thermalisation sweeps, then measured
    sweeps.  For U the crossing temperature of each pair of consecutive sizes
    is reported beside the exact T_c; the R curves of different sizes coincide
    between the two KT temperatures and spread outside."""
    import paper_1202_0635_amd as swmc

    sizes = [int(v) for v in args.uscan_sizes.split(",")]
    therm, w = args.uscan_therm, args.uscan_width
    potts_grid = [1.0 - w + 0.25 * w * k for k in range(9)]  # T / T_c
    wanted = set(args.uscan_models.split(","))
    models = []
    for name, q, model, grid in (("potts2", 2, "potts", potts_grid), ("potts3", 3, "potts", potts_grid),
                                 ("clock6", 6, "clock", [0.6 + 0.0625 * k for k in range(9)])):
        if name not in wanted:
            continue
        meas = args.uscan_sweeps if (model == "potts" or args.uscan_clock_sweeps is None) else args.uscan_clock_sweeps
        tc = swmc.critical_temperature(model, q)
        temps = [tc * f for f in grid] if model == "potts" else list(grid)
        specs = [(L, q, model, T, 1.0, 0x600000 + 1000 * L + k) for L in sizes for k, T in enumerate(temps)]
        b = swmc.Batch(specs)
        t0 = time.perf_counter()
        b.sweep(therm)
        chunk = 10000
        for done in range(0, meas, chunk):
            b.sweep(min(chunk, meas - done), measure=True)
            b.measure(0)  # waits for the chunk
            print(f"[uscan] {model} q={q}: {min(done + chunk, meas)} of {meas} measured sweeps", file=sys.stderr,
                  flush=True)
        obs = [b.measure(r) for r in range(len(specs))]
        dt = time.perf_counter() - t0
        b.close()
        key = "binder_u" if model == "potts" else "corr_ratio"
        curves = {L: [obs[i * len(temps) + k][key] for k in range(len(temps))] for i, L in enumerate(sizes)}
        row = {"model": model, "q": q, "observable": "U" if model == "potts" else "R", "T": temps,
               "curves": {str(L): c for L, c in curves.items()}, "seconds": dt,
               "measured_sweeps": meas, "spin_updates": sum(L * L for L in sizes) * len(temps) * (therm + meas)}
        if model == "potts":
            row["T_c_exact"] = tc
            row["crossings"] = crossings(temps, curves)
        print(f"[uscan] {model} q={q} done in {dt:.1f} s", file=sys.stderr, flush=True)
        models.append(row)
    return {"metric": "moment ratio U(T) and correlation ratio R(T) scans", "value": None, "unit": None,
            "higher_is_better": None, "n_gpus": 1, "dtype": "int8", "data": "synthetic",
            "config": {"workload": "uscan_" + "_".join(m for m in ("potts2", "potts3", "clock6") if m in wanted),
                       "sizes": sizes, "therm_sweeps": therm, "potts_grid_half_width": w},
            "models": models}


def bench_serve(args) -> dict:
    """Request trace (L log-uniform in [128, 2048], Potts q = 2, 3, 4 or clock q = 6,
    T in [0.8, 1.2] T_c, 100-1000 sweeps): capacity from a saturation run, then
    Poisson arrivals at 0.8 x capacity through the continuous-batching server
    and through the one-lattice-per-launch path."""
    import paper_1202_0635_amd  # noqa: F401
    from paper_1202_0635_amd import serve
    from paper_1202_0635_amd.workloads import request_trace

    trace = request_trace(args.requests)
    budget = int(args.budget_gib * (1 << 30))
    note = lambda msg: print(f"[serve] {msg}", file=sys.stderr, flush=True)
    sat = serve.run_trace(trace, serve.poisson_arrivals(len(trace), 0.0), budget, args.slots, args.sweeps_per_step)
    capacity = len(trace) / sat["makespan_s"]
    note(f"saturation run done: {sat['makespan_s']:.2f} s, capacity {capacity:.1f} requests/s")
    arrivals = serve.poisson_arrivals(len(trace), 0.8 * capacity, seed=20120203)
    served = serve.run_trace(trace, arrivals, budget, args.slots, args.sweeps_per_step)
    note(f"served run done: {served['makespan_s']:.2f} s")
    plain = serve.run_plain(trace, arrivals)
    note(f"plain run done: {plain['makespan_s']:.2f} s")
    same = all(served["results"][i]["spin_hash"] == plain["results"][i]["spin_hash"] for i in range(len(trace)))
    strip = lambda d: {k: v for k, v in d.items() if k not in ("results", "stats")}
    return {"metric": "served vs plain throughput (SW requests, continuous batching)",
            "value": served["spin_updates_per_s"] / plain["spin_updates_per_s"], "unit": "x",
            "higher_is_better": True, "n_gpus": 1, "dtype": "int8", "data": "synthetic",
            "config": {"workload": f"request_trace_{len(trace)}", "budget_bytes": budget, "slots": args.slots,
                       "sweeps_per_step": args.sweeps_per_step, "arrival_rate_per_s": 0.8 * capacity},
            "saturation": strip(sat), "served": strip(served), "plain": strip(plain),
            "results_identical": same}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mode", choices=["sweep", "batch", "serve", "labelers", "tscan", "uscan"], default="sweep",
                    help="sweep: one L=4096 lattice (default); batch: replica mix; serve: request trace")
    ap.add_argument("--replicas", type=int, default=256)
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--slots", type=int, default=128)
    ap.add_argument("--sweeps-per-step", type=int, default=25)
    ap.add_argument("--uscan-sizes", default="32,64,128")
    ap.add_argument("--uscan-therm", type=int, default=2000)
    ap.add_argument("--uscan-sweeps", type=int, default=20000)
    ap.add_argument("--uscan-width", type=float, default=0.03, help="Potts grid: T/T_c from 1 - w to 1 + w")
    ap.add_argument("--uscan-models", default="potts2,potts3,clock6", help="comma list of potts2, potts3, clock6")
    ap.add_argument("--uscan-clock-sweeps", type=int, default=None,
                    help="measured sweeps of the clock model (default: --uscan-sweeps)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="potts2_L4096_Tc")
    ap.add_argument("--tile-waves", type=int, choices=[4, 8], default=None,
                    help="waves per tile of the sweep mode's bond kernel (default: the autotuner's pick)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched- and served-vs-plain measurements")
    ap.add_argument("--no-serve", action="store_true", help="skip the served-vs-plain measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the single-lattice sweep "
              "is not sharded across GPUs here.", file=sys.stderr)
        return 2

    import torch

    if args.mode == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.mode == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return 0
    if args.mode == "labelers":
        print(json.dumps(bench_labelers(args)), flush=True)
        return 0
    if args.mode == "tscan":
        print(json.dumps(bench_tscan(args)), flush=True)
        return 0
    if args.mode == "uscan":
        print(json.dumps(bench_uscan(args)), flush=True)
        return 0

    import paper_1202_0635_amd as swmc
    from paper_1202_0635_amd.workloads import CONFIGS

    cfg = CONFIGS[args.config]
    torch.cuda.set_device(0)
    N = cfg.L * cfg.L
    lat = swmc.Lattice(cfg.L, cfg.q, cfg.model, T=cfg.T, J=cfg.J, seed=cfg.seed)
    # the workload's thermalisation (200 sweeps for the L = 4096 workloads), or
    # more if --warmup asks for it, before anything is timed
    therm = max(args.warmup, cfg.therm)
    lat.sweep(therm)
    # the autotuner picks the waves per tile on the thermalised state and restores it
    if args.tile_waves is None:
        waves = lat.tune(10)
    else:
        waves = args.tile_waves
        lat.set_tile_waves(waves)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.sweep(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    ns_per_update = ms * 1e6 / (args.steps * N)

    # The same number of sweeps with the per-sweep counts (update + measurement).
    e0.record(stream)
    lat.sweep(args.steps, measure=True)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_measure = e0.elapsed_time(e1)

    # Per-kernel launch times over further passes of the same number of sweeps
    # (the second with the per-sweep counts, for the count kernel's time).
    lat.sweep(args.steps, profile=True)
    prof = lat.profile()
    kernels = {k: {"launches": n, "avg_us": 1e3 * t / n} for k, (n, t) in prof.items() if n}
    lat.sweep(args.steps, measure=True, profile=True)
    n_c, t_c = lat.profile().get("k_counts", (0, 0.0))
    count_us = 1e3 * t_c / n_c if n_c else None
    dom = max(kernels, key=lambda k: kernels[k]["avg_us"] * kernels[k]["launches"])
    bytes_of = lambda k: alg_bytes_per_launch(k, cfg.L, cfg.model)
    dom_bytes = bytes_of(dom)
    achieved = dom_bytes / (kernels[dom]["avg_us"] * 1e-6) / 1e9
    # a sweep inside a multi-sweep call: the fused kernel and the merges that ran
    sweep_kernels = [k for k in SWEEP_KERNELS if k in kernels]
    sweep_bytes = sum(bytes_of(k) for k in sweep_kernels)
    sweep_gbps = sweep_bytes / (ms * 1e-3 / args.steps) / 1e9

    paper = PAPER_NS_PER_UPDATE.get(cfg.name)
    out = {
        "metric": "ns per spin update (SW sweep)",
        "value": ns_per_update,
        "unit": "ns/spin-update",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": (ns_per_update / paper) if paper else None,
        "dtype": "int8",
        "data": "synthetic",
        "config": {"workload": cfg.name, "L": cfg.L, "q": cfg.q, "model": cfg.model, "T": cfg.T, "J": cfg.J,
                   "seed": cfg.seed, "thermalisation_sweeps": therm, "workload_thermalisation": cfg.therm,
                   "timed_sweeps": args.steps, "tile_waves": waves},
        "spin_updates_per_s": N * args.steps / (ms * 1e-3),
        "ns_per_update_with_measurement": ms_measure * 1e6 / (args.steps * N),
        "k_counts_avg_us": count_us,
        "sweep_alg_bytes": sweep_bytes,
        "sweep_alg_GBps": sweep_gbps,
        "sweep_hbm_frac": sweep_gbps / HBM_PEAK_GBPS,
        "kernels": kernels,
        # the dominant kernel: algorithmic bytes per launch over its HIP-event
        # average (events bracket every launch, so this average includes the
        # gap between launches); frac_rocprof uses the committed rocprofv3
        # trace average of the same kernel when its sources are unchanged
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": None, "alg_bytes_per_launch": dom_bytes,
                     "hip_event_avg_us": kernels[dom]["avg_us"]},
    }
    traffic = measured_traffic(dom, cfg.name)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
    trace_us = traced_avg_us(dom, cfg.name)
    if trace_us is not None:
        out["roofline"]["rocprof_avg_us"] = trace_us
        out["roofline"]["frac_rocprof"] = dom_bytes / (trace_us * 1e-6) / 1e9 / HBM_PEAK_GBPS
    lat.close()
    if args.copy_calibration:
        src = torch.empty(COPY_BYTES, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
    if not args.no_batch:
        # the replica mix, batched against one lattice per launch (500 sweeps)
        bargs = argparse.Namespace(replicas=256, steps=500, warmup=20)
        bb = bench_batch(bargs)
        out["batched_vs_plain"] = {k: bb[k] for k in ("value", "config", "batched_spin_updates_per_s",
                                                      "plain_spin_updates_per_s", "batched_s", "plain_s")}
        out["batched_vs_plain"]["sweeps"] = bargs.steps
        if not args.no_serve:
            # the whole request trace (2000 requests), served against one lattice per launch
            sargs = argparse.Namespace(requests=args.requests, budget_gib=args.budget_gib, slots=args.slots,
                                       sweeps_per_step=args.sweeps_per_step)
            ss = bench_serve(sargs)
            sat = ss["saturation"]
            out["served_vs_plain"] = {"value": ss["value"], "config": ss["config"],
                                      "results_identical": ss["results_identical"],
                                      "served": ss["served"], "plain": ss["plain"],
                                      "saturation": {"makespan_s": sat["makespan_s"],
                                                     "spin_updates_per_s": sat["spin_updates_per_s"],
                                                     "vs_plain": sat["spin_updates_per_s"]
                                                     / ss["plain"]["spin_updates_per_s"]}}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
