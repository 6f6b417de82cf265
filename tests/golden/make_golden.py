"""Write expected degrees for the synthetic workloads, computed by the oracle
only (exact SNF + kernel points + brute-force volume).  Nothing here touches
the product library.

    python tests/golden/make_golden.py cfg1 cfg2 cfg3 cfg4 cfg5 [--threads T]

cfg5 stores a stated subset of the 4000-request serving trace (its 20 largest
requests and 400 more drawn by a seeded stream, see ``cfg5_subset``); each
record's ``index`` is the request's position in the trace.

Each output file records the generator version it was made with; tests refuse
a file whose version differs from ``gen.GEN_VERSION``.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import gen  # noqa: E402
import oracle  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def record(sysobj, threads):
    t = time.time()
    r = oracle.oracle_degree(sysobj.A, seed=0x60D + sysobj.index, bits=sysobj.lift_bits, threads=threads)
    N = sysobj.n + 1
    return dict(index=sysobj.index, m=sysobj.m, n=sysobj.n, k=r["k"], rank=r["rank"], comps=r["comps"],
                nvol=r["nvol"], candidates=oracle.binom(N, r["k"] + 1) if r["k"] else 0,
                oracle_s=round(time.time() - t, 3))


CFG5_SUBSET = 400  # seeded requests of the serving trace, plus its 20 largest
CFG5_LARGEST = 20


def cfg5_subset(trace):
    """The serving trace's requests with stored oracle degrees: its CFG5_LARGEST
    largest by candidate count (ties broken by index) and CFG5_SUBSET others
    drawn without replacement by a seeded stream."""
    import math

    cand = [math.comb(q.system.n + 1, q.system.n - q.system.m + 1) for q in trace]
    largest = sorted(range(len(trace)), key=lambda i: (-cand[i], i))[:CFG5_LARGEST]
    rng = gen.stream(gen.SEED_CFG[5], 0, gen.PURPOSE_SIZES ^ 0x601D)
    rest = [i for i in range(len(trace)) if i not in set(largest)]
    pick = []
    for _ in range(CFG5_SUBSET):
        j = rng.bounded(len(rest))
        pick.append(rest.pop(j))
    return sorted(largest + pick)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+")
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--count", type=int, default=4096, help="systems of the batch workload")
    ap.add_argument("--trace", type=int, default=4000, help="requests of the serving trace")
    a = ap.parse_args()
    oracle.build(force=False)
    makers = {
        "cfg1": lambda: [gen.cfg1_system()],
        "cfg2": lambda: [gen.cfg2_system()],
        "cfg3": lambda: gen.cfg3_systems(a.count),
        "cfg4": lambda: [gen.cfg4_system()],
        "cfg5": lambda: (lambda tr: [tr[i].system for i in cfg5_subset(tr)])(gen.cfg5_trace(a.trace)),
    }
    for w in a.which:
        systems = makers[w]()
        out = dict(workload=w, gen_version=gen.GEN_VERSION, systems=[])
        for s in systems:
            out["systems"].append(record(s, a.threads))
            print(w, out["systems"][-1], flush=True)
        with open(os.path.join(HERE, f"{w}_expected.json"), "w") as f:
            json.dump(out, f, indent=0)


if __name__ == "__main__":
    main()
