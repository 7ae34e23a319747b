"""Write the golden hash streams of the benchmark workloads from the CPU oracle.

Every stored value comes from `oracle/` (the plain sequential sweep of Sec. 2,
Hoshen-Kopelman labeling with the smallest label as the proper label; Sec. 4
for the clock model): per-sweep state hashes

    H_s = sum_i mix64((i << 8) | s_i),  H_l = sum_i mix64((i << 32) | l_i)  (mod 2^64)

with mix64 the SplitMix64 output function and l_i the canonical label (the
smallest site index of i's cluster).  Workload parameters come from
`paper_1202_0635_amd.workloads`, which names sizes, temperatures and seeds and
holds none of the method's arithmetic.  Nothing here calls the GPU library.

    python tests/golden/make_golden.py [--only NAME] [--jobs 8]

Files (one record per line, integers in decimal, hashes in hex):
  potts2_L64_Tc.txt        t hs hl          every sweep t = 1..1000 (Ising L = 64 at T_c, seed 1)
  potts2_L4096_Tc.txt      t hs hl          t = 1..250 (200 thermalisation sweeps + 50; seed 2)
  clock6_L4096_T0.9.txt    t hs hl          t = 1..250 (q = 6 clock, T = 0.9; seed 3)
  potts3_replicas_256.txt  r t hs hl        the 256 q = 3 replicas at t = 1, 10, 100, 500
  request_trace_sample40.txt  i t hs hist... pair_hist...   40 requests of the 2000-request
                           trace (10 per model kind, spread over L), final state
"""
from __future__ import annotations

import argparse
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

REPLICA_CHECKPOINTS = (1, 10, 100, 500)


def _chain_stream(name: str, sweeps: int):
    import oracle
    from paper_1202_0635_amd.workloads import CONFIGS

    c = CONFIGS[name]
    ch = oracle.Chain(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
    rows = []
    t0 = time.time()
    for _ in range(sweeps):
        ch.sweep(1)
        rows.append((ch.t, oracle.hash_spins(ch.spins), oracle.hash_labels(ch.labels)))
        if ch.t % 25 == 0:
            print(f"[golden] {name}: sweep {ch.t} of {sweeps} ({time.time() - t0:.0f} s)", flush=True)
    return rows


def _replica(r: int):
    import oracle
    from paper_1202_0635_amd.workloads import replica_mix_q3

    c = replica_mix_q3(256)[r]
    ch = oracle.Chain(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
    out = []
    for t in REPLICA_CHECKPOINTS:
        ch.sweep(t - ch.t)
        out.append((r, ch.t, oracle.hash_spins(ch.spins), oracle.hash_labels(ch.labels)))
    return out


def trace_sample():
    """Ten requests of each model kind, at evenly spaced ranks of L within the
    kind (smallest and largest included), in trace order."""
    from paper_1202_0635_amd.workloads import request_trace

    trace = request_trace(2000)
    picked = []
    for kind in (("potts", 2), ("potts", 3), ("potts", 4), ("clock", 6)):
        idx = sorted((i for i, c in enumerate(trace) if (c.model, c.q) == kind), key=lambda i: (trace[i].L, i))
        for k in range(10):
            picked.append(idx[round(k * (len(idx) - 1) / 9)])
    return sorted(picked)


def _request(i: int):
    import oracle
    from paper_1202_0635_amd.workloads import request_trace

    c = request_trace(2000)[i]
    ch = oracle.Chain(c.L, c.q, c.model, T=c.T, J=c.J, seed=c.seed)
    ch.sweep(c.sweeps)
    h, p = ch.counts()
    return (i, ch.t, oracle.hash_spins(ch.spins), list(map(int, h)), list(map(int, p)))


HEADER = ("# Golden values written by tests/golden/make_golden.py from the CPU oracle only\n"
          "# (Sec. 2 procedure with Hoshen-Kopelman labeling, smallest label = proper label;\n"
          "# Sec. 4 embedded clusters for the clock model).\n")


def write_chain(name, sweeps, rows):
    path = os.path.join(HERE, f"{name}.txt")
    with open(path, "w") as fh:
        fh.write(HEADER)
        fh.write(f"# workload {name}: per-sweep state hashes, sweeps 1..{sweeps} from the random start\n")
        fh.write("# columns: t hash_spins hash_labels\n")
        for t, hs, hl in rows:
            fh.write(f"{t} {hs:016x} {hl:016x}\n")
    print(f"[golden] wrote {path}", flush=True)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default=None)
    ap.add_argument("--jobs", type=int, default=8)
    args = ap.parse_args()
    want = lambda n: args.only in (None, n)
    chains = [("potts2_L64_Tc", 1000), ("potts2_L4096_Tc", 250), ("clock6_L4096_T0.9", 250)]
    with ProcessPoolExecutor(args.jobs) as pool:
        futs = {name: pool.submit(_chain_stream, name, n) for name, n in chains if want(name)}
        rep = [pool.submit(_replica, r) for r in range(256)] if want("potts3_replicas_256") else []
        sample = trace_sample() if want("request_trace_sample40") else []
        req = [pool.submit(_request, i) for i in sample]
        if rep:
            path = os.path.join(HERE, "potts3_replicas_256.txt")
            with open(path, "w") as fh:
                fh.write(HEADER)
                fh.write("# workload potts3_replicas_256: q = 3 Potts replicas r = 0..255, L = {64,128,256,512}[r % 4],\n"
                         "# T = T_c(3) (0.9 + 0.2 r / 255), seed 0x4000 + r; state hashes at sweeps 1, 10, 100, 500\n")
                fh.write("# columns: r t hash_spins hash_labels\n")
                for f in rep:
                    for r, t, hs, hl in f.result():
                        fh.write(f"{r} {t} {hs:016x} {hl:016x}\n")
            print(f"[golden] wrote {path}", flush=True)
        if req:
            path = os.path.join(HERE, "request_trace_sample40.txt")
            with open(path, "w") as fh:
                fh.write(HEADER)
                fh.write("# workload request_trace_2000 (numpy seed 20120203): 40 requests, ten per model kind at\n"
                         "# evenly spaced ranks of L; final state after the request's sweeps\n")
                fh.write("# columns: i t hash_spins hist[0..q) pair_hist[0..q)\n")
                for f in req:
                    i, t, hs, h, p = f.result()
                    fh.write(f"{i} {t} {hs:016x} {' '.join(map(str, h))} {' '.join(map(str, p))}\n")
            print(f"[golden] wrote {path}", flush=True)
        for name, n in chains:
            if name in futs:
                write_chain(name, n, futs[name].result())
    return 0


if __name__ == "__main__":
    sys.exit(main())
