"""Write expected degrees for the synthetic workloads, computed by the oracle
only (exact SNF + kernel points + brute-force volume).  Nothing here touches
the product library.

    python tests/golden/make_golden.py cfg1 cfg2 cfg3 cfg4 [--threads T]

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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", nargs="+")
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("--count", type=int, default=4096, help="systems of the batch workload")
    a = ap.parse_args()
    oracle.build(force=False)
    makers = {
        "cfg1": lambda: [gen.cfg1_system()],
        "cfg2": lambda: [gen.cfg2_system()],
        "cfg3": lambda: gen.cfg3_systems(a.count),
        "cfg4": lambda: [gen.cfg4_system()],
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
