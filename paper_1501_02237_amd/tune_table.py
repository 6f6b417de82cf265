"""Write the autotuner's schedule table for this device (needs the GPU).

    python -m paper_1501_02237_amd.tune_table [--out PATH] [--reps R]

Runs bdeg_batch_tune on the benchmark workloads -- the 4096-system
quiver-like batch (k = 3..7, every lane-group width it holds) and the
single n = 28 and n = 36 systems -- and writes the fastest schedule of each
(k, lane-group width) bucket to tuning/gfx950.json beside the library, where
bdeg_batch_create picks it up.  Every schedule the tuner times must reproduce
the default schedule's sums exactly, or nothing is written.
"""
from __future__ import annotations

import argparse
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "tuning", "gfx950.json"))
    ap.add_argument("--reps", type=int, default=3)
    a = ap.parse_args()
    import gen
    import paper_1501_02237_amd as bd

    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    work = [("batch of 4096", [s.A for s in gen.cfg3_systems(4096)], 3, 20)]
    for s in (gen.cfg2_system(), gen.cfg4_system()):
        work.append((f"n = {s.n}", [s.A], 1, s.lift_bits))
    for name, mats, seed, bits in work:
        print(f"tuning: {name}", flush=True)
        b = bd.Batch(mats, seed=seed, lift_bits=bits)
        try:
            b.tune(a.out, reps=a.reps)
        finally:
            b.close()
    print(open(a.out).read(), flush=True)


if __name__ == "__main__":
    main()
