"""Benchmark: exact candidate simplices decided per second on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-extras] [--no-cpu] [--only LEG]

Headline workload (one "step" = one full device pass over one system, inputs
resident in HBM): the large quiver-like system n = 36 (26 rows p - q of
weight 2-4, k = 10, N = 37 points, C(37, 11) = 854,992,152 candidates,
heights < 2^24), the largest single-system workload.  A step resets the
accumulators, draws the lifting, enumerates and tests every candidate, runs
the (empty) tie-redraw rounds and reads the 128-bit volume back.

Also reported (keys under "extra"): the n = 28 system (k = 8) the same way,
end-to-end plain solves (host prologue + copies), the 4096-system batch in
one captured pass vs plain one-by-one solves, the prefix-pruned enumeration,
the cell walk, and the serving trace.  The oracle leg times the oracle on a
bounded colex rank slice of the headline system, on all host threads and on
one.

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

# 32-bit integer VALU lane-ops/s: 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz (the fp32 vector
# rate, 157.3 TFLOP/s, is this many FMA lanes x 2 flops).  Plain 32-bit adds sustain 6.1e13 lane-ops/s
# on the part (77 % of this, the clock under load); 32 x 32 -> 64 multiply-adds issue at half this rate,
# which is why the op model counts each as 2 operations.
PEAK_ALU = 256 * 4 * 32 * 2.4e9

# HBM traffic of one headline enumeration launch (n = 36 system), from the
# rocprofv3 FETCH_SIZE and WRITE_SIZE passes summarised in
# profiles/enum_kernel_large36.md (KiB per dispatch, mean of the timed
# dispatches), each scaled by what the counter reads for a device copy of
# known size in the same run.  Valid only for the kernel sources and the
# work-unit sizing (the tuned schedule table) the counters were taken on: any
# change to the listed files makes `traffic` null.
TRAFFIC = {
    "sources": ("enum_device.hpp", "enum_dense.hpp", "exact_div.hpp", "kernels_k10.hip", "runtime.cpp",
                "bdeg_internal.hpp", "lifting.hpp"),
    "table": os.path.join("tuning", "gfx950.json"),
    "sha256": "9c6a796339797578bd87de35f2939b340537a297a96147d19112d4b095818b4a",
    "fetch_kib": 31881.77, "fetch_scale": 262144.0 / 131088.44,
    "write_kib": 839970.56, "write_scale": 262144.0 / 262144.0,
}


def traffic_bytes():
    h = hashlib.sha256()
    pkg = os.path.join(ROOT, "paper_1501_02237_amd")
    for f in TRAFFIC["sources"]:
        with open(os.path.join(pkg, "csrc", f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(pkg, TRAFFIC["table"]), "rb") as fh:
            h.update(fh.read())
    except OSError:
        return None
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return 1024.0 * (TRAFFIC["fetch_kib"] * TRAFFIC["fetch_scale"] + TRAFFIC["write_kib"] * TRAFFIC["write_scale"])


def ops_per_launch(stats: dict) -> float:
    """Algorithmic 32-bit integer operations of one enumeration launch.

    Op model (32-bit lane operations of the minimal instruction sequence; a
    32 x 32 -> 64 multiply counts 2, a 64-bit add/shift 2):
      spatial residual entry  8   (two products, a 64-bit difference, a shift, the inverse multiply)
      height residual entry  24   (two 64-bit halves of two products each, shift-add, 64-bit inverse multiply, split)
      lanes-as-points schedule:
        leaf test per point  20   (two halves, carry fold, sign and zero tests)
      lane-dense schedule (no ridges):
        candidate set-up    198   (three spatial and three height 2 x 2 minors, 24 + 72; the 3 x 3 spatial
                                   minor, 12; three 3 x 3 height minors in split limbs, 90)
        test per point       19   (eight products, the low limbs' carry shift, the sign accumulation)
    Every node update runs on all N points of its system; a leaf (a
    candidate with D != 0) tests the N - k - 1 other points with lanes as
    points, and in the lane-dense schedule the points up to its first point
    proved below (a full test batch stops once every candidate has one), as
    counted by the counting variant; the lane-dense schedule sets up every
    candidate of its nodes, D = 0 or not (tail quadruples at the rate of a
    triple).  The counting
    kernel variant reports the counts already weighted by each system's N
    (exact for batches of mixed sizes): a ridge adds one spatial and one
    height entry per point, an inner node one height entry and W - 1 spatial
    entries per point.  (When a launch mixes both schedules the leaf test is
    counted at the smaller rate.)"""
    sp = stats["point_spatial"] + stats["point_ridges"]
    ht = stats["point_inner"] + stats["point_ridges"]
    leaf = 19.0 if stats.get("dense_units", 0) > 0 else 20.0
    return 8.0 * sp + 24.0 * ht + leaf * stats["leaf_points"] + 198.0 * stats.get("triples", 0)


def batch_leg(bd, torch, gen, reps: int) -> dict:
    """The 4096-system batch in one prepared, captured device pass (the tuned
    schedule table when one is installed), against the same systems solved
    one by one with bdeg_degree."""
    log("[bench] generating the 4096-system batch")
    sy3 = gen.cfg3_systems(4096)
    mats = [x.A for x in sy3]
    cand3 = sum(math.comb(x.n + 1, x.n - x.m + 1) for x in sy3)
    t = time.perf_counter()
    b3 = bd.Batch(mats, seed=3, lift_bits=20)
    prep = time.perf_counter() - t
    b3.run()
    b3.results()
    torch.cuda.synchronize()
    t = time.perf_counter()
    kms = []
    for _ in range(reps):
        b3.run()
        res3 = b3.results()
        kms.append(b3.stats()["kernel_ms"])
    torch.cuda.synchronize()
    bt = (time.perf_counter() - t) / reps
    st3 = b3.stats()
    prof = b3.profile()
    b3.close()
    assert all(r["status"] == 0 for r in res3)
    k_ms = sum(kms) / len(kms)
    out = {"batch4096_systems_per_s": 4096 / bt, "batch4096_cand_per_s": cand3 / bt,
           "batch4096_ms": round(bt * 1e3, 3), "batch4096_kernel_ms": round(k_ms, 3),
           "batch4096_e2e_systems_per_s": 4096 / (bt + prep), "batch4096_captured": st3["captured"],
           "batch4096_redraws": st3["redraws"],
           "batch4096_alu_frac": ops_per_launch(prof) / (k_ms * 1e-3) / PEAK_ALU,
           "batch4096_tuned_table": os.path.exists(os.path.join(ROOT, "paper_1501_02237_amd", "tuning",
                                                                "gfx950.json"))}
    sample = mats[:512]
    t = time.perf_counter()
    for A in sample:
        bd.degree(A, seed=3, lift_bits=20)
    pt = (time.perf_counter() - t) / len(sample)
    out["plain_one_by_one_systems_per_s"] = 1.0 / pt
    log(f"[bench] batch 4096: {bt*1e3:.2f} ms ({4096/bt:.0f} sys/s, kernel {k_ms:.2f} ms, ALU fraction "
        f"{out['batch4096_alu_frac']:.3f}, captured {st3['captured']}), plain one-by-one {1/pt:.0f} sys/s")
    return out


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


def plain_leg(bd, torch, s, steps: int, warmup: int, seed: int = 1) -> dict:
    """One system as a prepared batch: `steps` timed device passes (clear,
    lifting, enumeration of every candidate, tie redraws, readback), after
    `warmup` untimed ones; then one counting pass for the op model."""
    N, k = s.n + 1, s.n - s.m
    cand = math.comb(N, k + 1)
    b = bd.Batch([s.A], seed=seed, lift_bits=s.lift_bits)
    for _ in range(warmup):
        b.run()
        b.results()
    kms, ref = [], None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        b.run()
        r = b.results()[0]
        st = b.stats()
        kms.append(st["kernel_ms"])
        if ref is None:
            ref = r
        assert r["status"] == 0 and r["nvol"] == ref["nvol"]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    captured = b.stats()["captured"]
    st = b.profile()  # work counters of the same pass (counting kernel variant, untimed)
    b.close()
    k_ms = sum(kms) / len(kms)
    ops = ops_per_launch(st)
    return {"N": N, "k": k, "candidates": cand, "ms_step": dt * 1e3 / steps, "value": cand * steps / dt,
            "kernel_ms": k_ms, "ops": ops, "achieved": ops / (k_ms * 1e-3), "nvol": ref["nvol"], "stats": st,
            "captured": captured}


def oracle_leg(s, all_ranks: int, one_ranks: int) -> dict:
    """The oracle as it stands on a bounded sample of the headline system:
    its own prologue (Smith form, kernel points, LLL) once, then the colex
    rank slice [0, all_ranks) on every host thread it uses, and [0, one_ranks)
    on one thread."""
    import oracle

    oracle.build(force=False)
    from oracle import algebra

    threads = oracle.default_threads()
    t = time.perf_counter()
    _, _, pts = algebra.kernel_points(s.A.tolist())
    prologue = time.perf_counter() - t
    H = oracle.oracle_heights(1, 0, len(pts), s.lift_bits)
    t = time.perf_counter()
    oracle.nvol_range(pts, H, 0, all_ranks, threads=threads)
    t_all = time.perf_counter() - t
    t = time.perf_counter()
    oracle.nvol_range(pts, H, 0, one_ranks, threads=1)
    t_one = time.perf_counter() - t
    log(f"[bench] oracle: prologue {prologue:.2f} s; ranks [0, {all_ranks}) in {t_all:.2f} s on {threads} threads; "
        f"[0, {one_ranks}) in {t_one:.2f} s on 1 thread")
    return {"value": all_ranks / t_all, "unit": "candidates/s", "cores": threads, "kind": "oracle",
            "sample": f"the n=36 k=10 system's candidates of colex rank [0, {all_ranks}) on {threads} threads "
                      f"({t_all:.1f} s; the oracle's own Smith form, kernel basis and lifting, prologue "
                      f"{prologue:.1f} s not included)",
            "single_core_value": one_ranks / t_one,
            "single_core_sample": f"ranks [0, {one_ranks}) on 1 thread ({t_one:.1f} s)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=4000)
    ap.add_argument("--oracle-ranks", type=int, default=20_000_000,
                    help="colex ranks of the headline system the oracle decides on all host threads")
    ap.add_argument("--oracle-ranks-1core", type=int, default=1_000_000,
                    help="colex ranks of the headline system the oracle decides on one thread")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="first run one plain device-to-device copy of this many MiB (a dispatch of known "
                         "traffic, for scaling hardware byte counters)")
    ap.add_argument("--only", default="", choices=["", "headline", "headline28", "batch"],
                    help="run only this leg's timed steps and print its figures (for profiling)")
    ap.add_argument("--pruned", default="", choices=["", "headline", "large36"],
                    help="run only the prefix-pruned enumeration of this system and print its figures")
    ap.add_argument("--schedule", default="auto", choices=["auto", "points"],
                    help="enumeration schedule of every leg (the headline is also run under the other one as an "
                         "extra unless --no-extras)")
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
    sched = {"auto": bd.SCHED_AUTO, "points": bd.SCHED_POINTS}[a.schedule]
    bd.set_schedule(sched)
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

    if a.only == "batch":
        print(json.dumps(batch_leg(bd, torch, gen, a.steps)), flush=True)
        return
    if a.only == "headline28":
        h = plain_leg(bd, torch, gen.cfg2_system(), a.steps, a.warmup)
        st = h.pop("stats")
        h["work"] = {key: st[key] for key in ("tiles", "inner_nodes", "ridges", "leaves", "triples", "ridge_steps",
                                              "leaf_steps", "empty_steps", "dense_units", "quads", "pruned")}
        print(json.dumps(h), flush=True)
        return

    s4 = gen.cfg4_system()
    log(f"[bench] headline: quiver n={s4.n} m={s4.m} k={s4.n - s4.m} N={s4.n + 1} "
        f"candidates={math.comb(s4.n + 1, s4.n - s4.m + 1)}")
    h = plain_leg(bd, torch, s4, a.steps, a.warmup)
    log(f"[bench] headline: {h['ms_step']:.3f} ms/step, kernel {h['kernel_ms']:.3f} ms, nvol={h['nvol']}, "
        f"{h['value']:.3e} cand/s, ops/launch {h['ops']:.3e}, ALU fraction {h['achieved'] / PEAK_ALU:.3f}")
    if a.only == "headline":
        st = h.pop("stats")
        h["work"] = {key: st[key] for key in ("tiles", "inner_nodes", "ridges", "leaves", "triples", "ridge_steps",
                                              "leaf_steps", "empty_steps", "dense_units", "quads", "pruned")}
        print(json.dumps(h), flush=True)
        return
    st = h["stats"]
    extra = {"schedule": a.schedule, "nvol": h["nvol"], "kernel_ms": round(h["kernel_ms"], 4),
             "captured": h["captured"], "leaves": st["leaves"], "ridges": st["ridges"],
             "inner_nodes": st["inner_nodes"], "triples": st["triples"], "pruned": st["pruned"],
             "units": st["tiles"], "dense_units": st["dense_units"], "ops_per_launch": h["ops"]}
    if not a.no_extras:
        # the same headline under the other schedule (same candidates, same result)
        other = "points" if a.schedule == "auto" else "auto"
        bd.set_schedule({"auto": bd.SCHED_AUTO, "points": bd.SCHED_POINTS}[other])
        ho = plain_leg(bd, torch, s4, max(3, a.steps // 4), 1)
        bd.set_schedule(sched)
        assert ho["nvol"] == h["nvol"]
        extra.update({f"{other}_schedule_kernel_ms": round(ho["kernel_ms"], 4),
                      f"{other}_schedule_cand_per_s": ho["value"],
                      f"{other}_schedule_alu_frac": ho["achieved"] / PEAK_ALU,
                      f"{other}_schedule_ops_per_launch": ho["ops"]})
        log(f"[bench] headline under the {other} schedule: kernel {ho['kernel_ms']:.3f} ms, "
            f"{ho['value']:.3e} cand/s, ALU fraction {ho['achieved'] / PEAK_ALU:.3f}")
        # the n = 28 system, same measurement
        h2 = plain_leg(bd, torch, gen.cfg2_system(), a.steps, a.warmup)
        extra.update({"headline28_cand_per_s": h2["value"], "headline28_ms_step": round(h2["ms_step"], 4),
                      "headline28_kernel_ms": round(h2["kernel_ms"], 4), "headline28_nvol": h2["nvol"],
                      "headline28_alu_frac": h2["achieved"] / PEAK_ALU})
        log(f"[bench] n=28: {h2['ms_step']:.3f} ms/step, kernel {h2['kernel_ms']:.3f} ms, "
            f"{h2['value']:.3e} cand/s, ALU fraction {h2['achieved'] / PEAK_ALU:.3f}")
        # end-to-end plain solve of the n = 28 system (host prologue, tiling, copies, device pass)
        s2 = gen.cfg2_system()
        reps = 10
        t = time.perf_counter()
        for _ in range(reps):
            bd.degree(s2.A, seed=1, lift_bits=s2.lift_bits)
        e2e = (time.perf_counter() - t) / reps
        extra["plain_e2e_ms"] = round(e2e * 1e3, 3)
        extra["plain_e2e_cand_per_s"] = h2["candidates"] / e2e
        extra["plain_resident_systems_per_s"] = 1e3 / h2["ms_step"]

        extra.update(batch_leg(bd, torch, gen, 5))

        # the prefix-pruned enumeration of the n = 28 and n = 36 systems
        for name in ("headline", "large36"):
            extra.update({f"pruned_{name}_{key}": v for key, v in prune_leg(bd, gen, name).items()})

        # the cell walk on the largest Table 4 system, W_{4,5} (k = 22, N = 61)
        extra.update({f"walk_w45_{key}": v for key, v in walk_leg(bd, gen, 4, 5).items()})

        if a.serve_requests > 0:
            extra.update(serve_trace(bd, gen, a.serve_requests))

    cpu = None if a.no_cpu else oracle_leg(s4, a.oracle_ranks, a.oracle_ranks_1core)

    out = {
        "metric": "exact candidate simplices decided per second (plain single system, 1 GPU)",
        "value": h["value"],
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(h["ms_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32/i64 (exact integer, 128-bit products)",
        "data": "synthetic (seeded quiver-like exponent matrix)",
        "config": {"workload": "large quiver-like system n=36 m=26 k=10 N=37, row weights 2-4, heights < 2^24, "
                               "device-resident", "candidates": h["candidates"], "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": h["achieved"], "peak": PEAK_ALU, "unit": "int32 lane-ops/s",
                     "frac": h["achieved"] / PEAK_ALU, "traffic": traffic_bytes()},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
