"""Benchmark: exact candidate simplices decided per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu]

Headline workload (one "step" = one full device pass over one system, inputs
resident in HBM): the plain quiver-like system n = 28 (20 rows p - q of weight
2-3, k = 8, N = 29 points, C(29, 9) = 10,015,005 candidates, heights < 2^20).
A step clears the accumulators, draws the lifting, enumerates and tests every
candidate and reads the 128-bit volume back (tie redraws included).

Also reported (keys under "extra"): end-to-end plain solves (host prologue +
copies), the 4096-system batch in one launch vs plain one-by-one solves, the
n = 36 (k = 10) system, and the serving trace when available.

Prints ONE JSON line.  Only one GPU is used: --gpus above 1 exits.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_ALU = 256 * 4 * 16 * 2.4e9  # 32-bit integer VALU lane-ops/s: CUs x SIMDs x lanes x clock

# HBM traffic of one headline enumeration launch, from the rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes summarised in profiles/enum_kernel_quiver28_pmc.md (KiB
# per dispatch, mean of the timed dispatches), each scaled by what the counter
# reads for a device copy of known size in the same run (FETCH_SIZE reads half
# of the 256 MiB copied, WRITE_SIZE all of it).  Valid only for the kernel
# source and the work-unit sizing (runtime.cpp) the counters were taken on; any
# change to them makes `traffic` null.
TRAFFIC = {
    "sources": ("enum_device.hpp", "exact_div.hpp", "kernels_k8.hip", "runtime.cpp"),
    "sha256": "24dbb4a52de4e5af1b2451c2e41be4fd107d4567f7e2a1706dd6ec0e4a50467d",
    "fetch_kib": 1786.59, "fetch_scale": 262144.0 / 131093.0,
    "write_kib": 1007.72, "write_scale": 262144.0 / 262144.0,
}


def traffic_bytes():
    h = hashlib.sha256()
    for f in TRAFFIC["sources"]:
        with open(os.path.join(ROOT, "paper_1501_02237_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


def ops_per_launch(stats: dict, N: int, k: int) -> float:
    """Algorithmic 32-bit integer operations of one enumeration launch.

    Op model (32-bit lane operations of the minimal instruction sequence; a
    32 x 32 -> 64 multiply counts 2, a 64-bit add/shift 2):
      spatial residual entry  8   (two products, a 64-bit difference, a shift, the inverse multiply)
      height residual entry  24   (two 64-bit halves of two products each, shift-add, 64-bit inverse multiply, split)
      leaf test per point    20   (two halves, carry fold, sign and zero tests)
    Every node update runs on all N points; a leaf tests the N - k - 1 other points."""
    sp = stats["spatial_updates"] + stats["ridges"]
    ht = stats["inner_nodes"] + stats["ridges"]
    return N * (8.0 * sp + 24.0 * ht) + 20.0 * (N - k - 1) * stats["leaves"]


def walk_leg(bd, gen, m: int, k: int) -> dict:
    """The cell walk on the Table 4 system W_{m,k}, end to end (prologue,
    allocation, every level) after a warm-up walk, checked against the
    paper's degree."""
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as fh:
        deg = json.load(fh)["table4_degrees"][f"{m},{k}"]
    A = gen.master_space_matrix(m, k)
    bd.degree_pivot(gen.master_space_matrix(3, 4), seed=5, lift_bits=20)
    t = time.perf_counter()
    r = bd.degree_pivot(A, seed=5, lift_bits=20)
    wt = time.perf_counter() - t
    assert r["status"] == 0 and r["comps"] * r["nvol"] == deg, (r, deg)
    N = len(A[0]) + 1
    log(f"[bench] walk W_{m},{k}: k={r['k']} N={N} {r['cells']} cells in {wt:.3f} s")
    return {"s": round(wt, 4), "cells": r["cells"], "cells_per_s": r["cells"] / wt}


def prune_leg(bd, gen, name: str, reps: int = 5) -> dict:
    """The prefix-pruned enumeration on a bench system (its points and the
    lifting of its plain solve), device time of both phases, checked against
    the plain path's volume."""
    s = {"headline": gen.cfg2_system, "large36": gen.cfg4_system}[name]()
    sub = bd.subdivision(s.A, seed=1, lift_bits=s.lift_bits, cap=0)
    P, H = sub["points"], sub["heights"]
    bd.nvol_points_pruned(P, H)
    dev, wall = [], []
    for _ in range(reps):
        t = time.perf_counter()
        g = bd.nvol_points_pruned(P, H)
        wall.append(time.perf_counter() - t)
        assert g["nvol"] == sub["nvol"] and not g["tie"], (g, sub["nvol"])
        dev.append(g["stats"]["filter_ms"] + g["stats"]["enum_ms"])
    st = g["stats"]
    N, k = P.shape
    cand = math.comb(N, k + 1)
    ms = sum(dev) / len(dev)
    log(f"[bench] pruned {name}: {ms:.3f} ms device (filter {st['filter_ms']:.3f}, enumeration {st['enum_ms']:.3f}), "
        f"{st['pruned']} of {st['prefixes']} prefixes pruned")
    return {"device_ms": round(ms, 4), "filter_ms": round(st["filter_ms"], 4), "enum_ms": round(st["enum_ms"], 4),
            "wall_ms": round(1e3 * sum(wall) / len(wall), 4), "cand_per_s": cand / (ms * 1e-3),
            "width": st["width"], "prefixes": st["prefixes"], "pruned": st["pruned"], "units": st["units"]}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    xs = sorted(xs)
    return xs[min(len(xs) - 1, int(q * len(xs)))]


def serve_trace(bd, gen, count):
    """Poisson arrivals (mean 200 req/s) of quiver-like systems, n ~ U[12,32],
    k ~ U[4,9]: served by the continuous-batching engine vs plain sequential
    solves (one bdeg_degree at a time, in arrival order)."""
    log(f"[bench] serving: generating {count} requests")
    trace = gen.cfg5_trace(count)
    mats = [q.system.A for q in trace]
    out = {}
    # plain sequential solves: measured service times, FIFO queue simulated on the arrival times
    plain, service = [], []
    for A in mats:
        t = time.perf_counter()
        plain.append(bd.degree(A, seed=5, lift_bits=20))
        service.append(time.perf_counter() - t)
    free, lat_plain = 0.0, []
    for q, sv in zip(trace, service):
        free = max(free, q.arrival_s) + sv
        lat_plain.append((free - q.arrival_s) * 1e3)
    out["serve_plain_p50_ms"] = round(pct(lat_plain, 0.5), 3)
    out["serve_plain_p99_ms"] = round(pct(lat_plain, 0.99), 3)
    out["serve_plain_systems_per_s"] = count / sum(service)
    # served, real time: submit at the arrival times
    srv = bd.Server(256 << 20)
    t0 = time.perf_counter()
    tickets = []
    for q, A in zip(trace, mats):
        while time.perf_counter() - t0 < q.arrival_s:
            pass
        tickets.append(srv.submit(A, seed=5, lift_bits=20))
    got = [srv.wait(t) for t in tickets]
    t_end = time.perf_counter() - t0
    lat = [srv.latency_ms(t) for t in tickets]
    srv.close()
    assert all(g["nvol"] == p["nvol"] and g["status"] == 0 for g, p in zip(got, plain))
    out["serve_p50_ms"] = round(pct(lat, 0.5), 3)
    out["serve_p99_ms"] = round(pct(lat, 0.99), 3)
    out["serve_trace_systems_per_s"] = count / t_end
    # saturated: everything submitted at once, served vs plain
    srv = bd.Server(256 << 20)
    t = time.perf_counter()
    tickets = [srv.submit(A, seed=5, lift_bits=20) for A in mats]
    got = [srv.wait(x) for x in tickets]
    sat = time.perf_counter() - t
    srv.close()
    assert all(g["nvol"] == p["nvol"] for g, p in zip(got, plain))
    out["serve_saturated_systems_per_s"] = count / sat
    log(f"[bench] serving: p50 {out['serve_p50_ms']} ms p99 {out['serve_p99_ms']} ms "
        f"(plain sequential p50 {out['serve_plain_p50_ms']} p99 {out['serve_plain_p99_ms']}); "
        f"saturated {count / sat:.0f} sys/s vs plain {out['serve_plain_systems_per_s']:.0f} sys/s")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a dispatch of known "
                         "traffic, for scaling hardware byte counters)")
    ap.add_argument("--pruned", default="", choices=["", "headline", "large36"],
                    help="run only the prefix-pruned enumeration of this system and print its figures")
    ap.add_argument("--walk", default="",
                    help="M,K: run only the cell walk on the Table 4 system W_{M,K} and print its figures")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {a.gpus}); "
              "the multi-GPU design is described in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch

    import gen
    import paper_1501_02237_amd as bd

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if a.calibrate_copy_mib > 0:
        src = torch.ones(a.calibrate_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {a.calibrate_copy_mib} MiB read + {a.calibrate_copy_mib} MiB written")
        del src, dst

    if a.pruned:
        print(json.dumps({"pruned": a.pruned, **prune_leg(bd, gen, a.pruned)}), flush=True)
        return

    if a.walk:
        m, k = (int(x) for x in a.walk.split(","))
        print(json.dumps({"walk": f"W_{{{m},{k}}}", **walk_leg(bd, gen, m, k)}), flush=True)
        return

    s2 = gen.cfg2_system()
    N2, k2 = s2.n + 1, s2.n - s2.m
    cand2 = math.comb(N2, k2 + 1)
    log(f"[bench] headline: quiver n={s2.n} m={s2.m} k={k2} N={N2} candidates={cand2}")
    b = bd.Batch([s2.A], seed=1, lift_bits=s2.lift_bits)
    for _ in range(a.warmup):
        b.run()
        b.results()
    kms, ref = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        b.run()
        r = b.results()[0]
        st = b.stats()
        kms.append(st["kernel_ms"])
        if ref is None:
            ref = r
        assert r["status"] == 0 and r["nvol"] == ref["nvol"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = b.profile()  # work counters of the same pass (counting kernel variant, untimed)
    b.close()
    ms_step = dt * 1e3 / a.steps
    value = cand2 * a.steps / dt
    k_ms = sum(kms) / len(kms)
    ops = ops_per_launch(st, N2, k2)
    achieved = ops / (k_ms * 1e-3)
    log(f"[bench] headline: {ms_step:.3f} ms/step, kernel {k_ms:.3f} ms, nvol={ref['nvol']}, "
        f"{value:.3e} cand/s, ops/launch {ops:.3e}")

    extra = {"nvol": ref["nvol"], "kernel_ms": round(k_ms, 4), "leaves": st["leaves"], "ridges": st["ridges"],
             "inner_nodes": st["inner_nodes"], "pruned": st["pruned"], "units": st["tiles"]}
    if not a.no_extras:
        # end-to-end plain solve (host prologue, tiling, copies, device pass)
        reps = 10
        t = time.perf_counter()
        for _ in range(reps):
            bd.degree(s2.A, seed=1, lift_bits=s2.lift_bits)
        e2e = (time.perf_counter() - t) / reps
        extra["plain_e2e_ms"] = round(e2e * 1e3, 3)
        extra["plain_e2e_cand_per_s"] = cand2 / e2e
        extra["plain_resident_systems_per_s"] = 1e3 / ms_step

        # batch of 4096 systems in one launch vs the same systems one by one
        log("[bench] generating the 4096-system batch")
        sy3 = gen.cfg3_systems(4096)
        mats = [x.A for x in sy3]
        cand3 = sum(math.comb(x.n + 1, x.n - x.m + 1) for x in sy3)
        t = time.perf_counter()
        b3 = bd.Batch(mats, seed=3, lift_bits=20)
        prep = time.perf_counter() - t
        b3.run()
        b3.results()
        reps = 5
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(reps):
            b3.run()
            res3 = b3.results()
        torch.cuda.synchronize()
        bt = (time.perf_counter() - t) / reps
        st3 = b3.stats()
        b3.close()
        assert all(r["status"] == 0 for r in res3)
        extra["batch4096_systems_per_s"] = 4096 / bt
        extra["batch4096_cand_per_s"] = cand3 / bt
        extra["batch4096_ms"] = round(bt * 1e3, 3)
        extra["batch4096_kernel_ms"] = round(st3["kernel_ms"], 3)
        extra["batch4096_e2e_systems_per_s"] = 4096 / (bt + prep)
        sample = mats[:512]
        t = time.perf_counter()
        for A in sample:
            bd.degree(A, seed=3, lift_bits=20)
        pt = (time.perf_counter() - t) / len(sample)
        extra["plain_one_by_one_systems_per_s"] = 1.0 / pt
        log(f"[bench] batch 4096: {bt*1e3:.2f} ms ({4096/bt:.0f} sys/s), plain one-by-one {1/pt:.0f} sys/s")

        # the n = 36, k = 10 system
        s4 = gen.cfg4_system()
        b4 = bd.Batch([s4.A], seed=1, lift_bits=s4.lift_bits)
        b4.run()
        b4.results()
        b4.run()
        r4 = b4.results()[0]
        st4 = b4.stats()
        b4.close()
        cand4 = math.comb(s4.n + 1, s4.n - s4.m + 1)
        extra["large36_nvol"] = r4["nvol"]
        extra["large36_kernel_ms"] = round(st4["kernel_ms"], 3)
        extra["large36_cand_per_s"] = cand4 / (st4["total_ms"] * 1e-3)
        log(f"[bench] n=36 k=10: nvol={r4['nvol']} kernel {st4['kernel_ms']:.2f} ms")

        # the prefix-pruned enumeration of the headline and n = 36 systems
        for name in ("headline", "large36"):
            extra.update({f"pruned_{name}_{key}": v for key, v in prune_leg(bd, gen, name).items()})

        # the cell walk on the largest Table 4 system, W_{4,5} (k = 22, N = 61)
        extra.update({f"walk_w45_{key}": v for key, v in walk_leg(bd, gen, 4, 5).items()})

        if a.serve_requests > 0:
            extra.update(serve_trace(bd, gen, a.serve_requests))

    cpu = None
    if not a.no_cpu:
        import oracle

        oracle.build(force=False)
        from oracle import algebra

        threads = oracle.default_threads()
        t = time.perf_counter()
        kk, comps, pts = algebra.kernel_points(s2.A.tolist())
        part = oracle.nvol_range(pts, oracle.oracle_heights(1, 0, len(pts), s2.lift_bits), 0, cand2, threads=threads)
        ct = time.perf_counter() - t
        assert part.nvol == ref["nvol"], (part.nvol, ref["nvol"])
        cpu = {"value": cand2 / ct, "unit": "candidates/s", "cores": threads, "kind": "oracle",
               "sample": f"the whole headline system (all {cand2} candidates, exact SNF + brute force), {ct:.1f} s"}
        log(f"[bench] oracle: {ct:.2f} s on {threads} threads")

    out = {
        "metric": "exact candidate simplices decided per second (plain single system, 1 GPU)",
        "value": value,
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32/i64 (exact integer, 128-bit products)",
        "data": "synthetic (seeded quiver-like exponent matrix)",
        "config": {"workload": "plain quiver-like system n=28 m=20 k=8 N=29, heights < 2^20, device-resident",
                   "candidates": cand2, "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU, "unit": "int32 lane-ops/s",
                     "frac": achieved / PEAK_ALU, "traffic": traffic_bytes()},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
