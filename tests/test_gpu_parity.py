"""Parity of the HIP path with the oracle (exact: integers, tolerance 0).

* ``bdeg_nvol_points`` against ``oracle.nvol_range`` on the same point sets,
  the same explicit heights and the same colex rank ranges: the volume sum,
  the number of lower facets and the tie flag must all be equal.
* ``bdeg_degree`` / ``bdeg_degree_batch`` / prepared batches against
  ``oracle.oracle_degree`` (independent Smith form, kernel basis, lifting).
* The paper's master-space degrees, and stored oracle values for the full
  workloads (``tests/golden``).
"""
import json
import math
import os

import numpy as np
import pytest
from sympy import Matrix

import gen
import oracle
import paper_1501_02237_amd as bd

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
PAPER = json.load(open(os.path.join(GOLD, "paper_values.json")))


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    say("gpu fixture: importing torch")
    import torch

    assert torch.cuda.is_available(), "gpu tests need a GPU"
    say("gpu fixture: torch ready")
    oracle.build(force=False)
    bd.lib()


def _points(seed, N, k, lo=-2, hi=2):
    if k >= 7:  # keep the bordered Hadamard bound within the device's certified range
        lo, hi = max(lo, -1), min(hi, 1)
    rng = gen.stream(seed, N * 100 + k, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k] + [[rng.uniform_int(lo, hi) for _ in range(k)] for _ in range(N - 1)]
        if Matrix(P).rank() == k:
            return np.array(P, dtype=np.int64)


def _sparse_points(seed, N, k, density=0.2):
    """Points with few nonzero coordinates (in {-1, 1}), as in the master-space
    systems: deep k stays inside the device's certified minor bound."""
    rng = gen.stream(seed, N * 100 + k, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k]
        for _ in range(N - 1):
            P.append([(1 if rng.uniform_int(0, 1) else -1) if rng.uniform_int(0, 999) < density * 1000 else 0
                      for _ in range(k)])
        if Matrix(P).rank() == k:
            return np.array(P, dtype=np.int64)


def _same(P, H, lo=0, hi=None):
    g = bd.nvol_points(P, H, lo, hi)
    o = oracle.nvol_range(P, H, lo, hi)
    assert (g.nvol, g.cells, g.tie) == (o.nvol, o.cells, o.tie), (g, o)
    return g


# ------------------------------------------------------------------ explicit heights
def test_unit_square_gpu():
    say("unit square")
    g = _same([[0, 0], [0, 1], [1, 1], [1, 0]], [3, 1, 4, 1])
    assert g.nvol == 2 and g.cells == 2


CASES = [  # (N, k, bits): spans lane-group packings 8/16/32/64 and ragged N
    (4, 1, 12), (6, 2, 12), (8, 3, 16), (9, 3, 16), (12, 4, 16), (16, 4, 20), (17, 5, 20), (20, 3, 20),
    (24, 6, 20), (31, 4, 24), (32, 3, 24), (33, 3, 24), (40, 2, 24), (48, 3, 20), (63, 2, 20), (64, 2, 24),
    (64, 3, 24), (13, 6, 16), (14, 7, 16), (16, 9, 16), (15, 10, 16), (14, 12, 16), (13, 12, 20),
]


@pytest.mark.parametrize("N,k,bits", CASES)
def test_nvol_points_full_range(N, k, bits):
    say("nvol_points full", N, k, bits)
    P = _points(0xA11 + N, N, k)
    H = gen.random_heights(0xB22 + N * 7 + k, N, bits)
    _same(P, H)


@pytest.mark.parametrize("N,k", [(40, 5), (48, 4), (64, 4), (37, 10), (29, 8), (64, 6)])
def test_nvol_points_rank_slices(N, k):
    """Full-size point counts, sampled colex rank ranges (ragged edges)."""
    P = _points(0xC33 + N, N, k, -3, 3)
    H = gen.random_heights(0xD44 + N, N, 24)
    total = oracle.binom(N, k + 1)
    rng = gen.stream(0xE55, N * 31 + k, gen.PURPOSE_MATRIX)
    for _ in range(3):
        lo = rng.next() % total
        hi = min(total, lo + 1 + rng.next() % 60000)
        say("nvol_points slice", N, k, lo, hi)
        _same(P, H, lo, hi)
    _same(P, H, total - 777, total)
    _same(P, H, 0, 1)


@pytest.mark.parametrize("seed", range(6))
def test_ties_match_oracle(seed):
    """3-bit heights on small grids: ties are frequent; the flag, the partial
    sum and the cell count must match the oracle on every draw."""
    say("ties", seed)
    pts = np.array([[x, y] for x in range(3) for y in range(3)], dtype=np.int64)
    for a in range(6):
        H = gen.random_heights(0x7E + seed * 16 + a, 9, 3)
        _same(pts, H)
    P3 = np.array([[x, y, z] for x in range(2) for y in range(2) for z in range(3)], dtype=np.int64)
    _same(P3, gen.random_heights(0x7F + seed, len(P3), 3))


@pytest.mark.parametrize("N,k,bits", [(16, 13, 16), (18, 13, 20), (17, 14, 16), (20, 14, 16), (18, 15, 12),
                                       (19, 16, 12), (21, 16, 12), (24, 13, 16), (20, 17, 12), (21, 17, 16),
                                       (22, 18, 14), (23, 18, 16)])
def test_nvol_points_deep_k(N, k, bits):
    """k = 13..18 (single-k kernels beyond the mixed-k range, up to the
    device's deepest k), against the oracle on identical heights."""
    P = _sparse_points(0xDEE + N, N, k, 0.25)
    H = gen.random_heights(0xDEF + N + k, N, bits)
    say("deep k", N, k, bits)
    _same(P, H)


def test_single_candidate_and_empty_range():
    say("single candidate")
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.int64)
    g = _same(P, [5, 1, 2, 3])
    assert g.nvol == 1
    assert bd.nvol_points(P, [5, 1, 2, 3], 1, 1).nvol == 0


# ------------------------------------------------------------------ duplicate points
def _cube(k):
    import itertools

    return [list(v) for v in itertools.product([0, 1], repeat=k)]


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("which", ["origin", "vertex"])
def test_duplicate_points_equal_heights_tie(k, which):
    """A point repeated with the same height (v_i = v_j, or v_i = 0) lies on
    every lower facet through its twin: a non-generic lower face, so the tie
    flag is set, as the oracle says.  Cube vertices are vertices of the hull,
    so every copy is on the lower hull."""
    P = _cube(k)
    j = 0 if which == "origin" else len(P) - 1
    P = P + [list(P[j])]
    H = gen.random_heights(0xD0B + k, len(P), 16)
    H[-1] = H[j]
    say("duplicate equal heights", k, which)
    g = _same(np.array(P, dtype=np.int64), H)
    assert g.tie


@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("which", ["origin", "vertex", "inner"])
def test_duplicate_points_unequal_heights(k, which):
    """A repeated point with a different height: the higher copy is never on a
    lower facet, so the result is that of the set without it (no tie)."""
    P = _cube(k) + [[1] * (k - 1) + [0]]
    j = {"origin": 0, "vertex": len(P) - 2, "inner": len(P) - 1}[which]
    if which == "inner":  # a point strictly inside, repeated
        P = [[2 * x for x in v] for v in _cube(k)] + [[1] * k]
        j = len(P) - 1
    base = np.array(P, dtype=np.int64)
    Hb = gen.random_heights(0xD0C + k, len(P), 16)
    P2 = np.vstack([base, base[j:j + 1]])
    for up in (True, False):  # the copy above or below its twin
        H2 = np.append(Hb, Hb[j] + (12345 if up else -12345))
        say("duplicate unequal heights", k, which, up)
        g = _same(P2, H2)
        assert not g.tie
        want = oracle.nvol_range(base, Hb if up else np.where(np.arange(len(P)) == j, H2[-1], Hb))
        assert g.nvol == want.nvol


# ------------------------------------------------------------------ near the certified widths
def _cert_margin(P, span):
    """log2 of the slack of the device's width certificate for points P and
    height span (positive: inside).  Spatial Hadamard bound Hs (the smaller of
    its row- and column-wise forms) below 2^31, and (k+1) span Hs below 2^60."""
    import math

    P = np.asarray(P, dtype=np.int64)
    N, k = P.shape
    rows = sorted((1 + int((r * r).sum()) for r in P), reverse=True)[: k + 1]
    h2_rows = math.prod(rows)
    h2_cols = (k + 1) ** (k + 1) * math.prod(max(1, int(abs(P[:, i]).max())) ** 2 for i in range(k))
    h2 = min(h2_rows, h2_cols)
    return min(62 - math.log2(h2), 120 - math.log2(((k + 1) * max(span, 1)) ** 2 * h2)) / 2


@pytest.mark.parametrize("k,c,bits", [(2, 1, 39), (3, 12, 39), (4, 12, 36), (5, 9, 33), (5, 6, 36), (6, 2, 39),
                                      (7, 2, 36), (8, 1, 39)])
def test_heights_near_the_certified_width(k, c, bits):
    """Heights up to 2^39 in magnitude (the entry point takes |h| < 2^40) and
    point sets whose Hadamard bound leaves little room: the split 64-bit
    height arithmetic on the device agrees with the oracle's int128."""
    N = 3 * k + 4
    rng = gen.stream(0xCE27, k * 100 + c, gen.PURPOSE_MATRIX)
    from sympy import Matrix as M

    while True:
        P = [[0] * k] + [[rng.uniform_int(-c, c) for _ in range(k)] for _ in range(N - 1)]
        if M(P).rank() == k:
            break
    P = np.array(P, dtype=np.int64)
    H = gen.random_heights(0xCE28 + k, N, bits) - (1 << (bits - 1))
    H[0] = -(1 << bits) + 1 if bits < 40 else H[0]
    span = int(H.max() - H.min())
    margin = _cert_margin(P, span)
    say("near width", k, c, bits, "margin bits", round(margin, 2))
    assert 0 < margin < 17
    _same(P, H)


def test_nvol_points_bound_rejected():
    P = np.array([[0, 0], [1 << 20, 0], [0, 1 << 20]], dtype=np.int64)
    with pytest.raises(bd.BdegError) as e:
        bd.nvol_points(P, [0, 1, 2])
    assert e.value.code == bd.BDEG_E_OVERFLOW


# ------------------------------------------------------------------ whole degree
def _ores(A, bits=20):
    r = oracle.oracle_degree(A, bits=bits)
    return (r["k"], r["comps"], r["nvol"])


def _gres(r):
    return (r["k"], r["comps"], r["nvol"])


@pytest.mark.parametrize("idx", range(16))
def test_degree_random_quiver(idx):
    rng = gen.stream(0x5EED0201, idx, gen.PURPOSE_SIZES)
    n = rng.uniform_int(6, 18)
    k = rng.uniform_int(1, 7)
    A = gen.quiver_matrix(0x5EED0201, idx, n, n - k, 2, 3)
    say("degree quiver", idx, n, k)
    g = bd.degree(A, seed=idx, lift_bits=20)
    assert g["status"] == 0 and g["attempts"] >= 1
    assert _gres(g) == _ores(A)


@pytest.mark.parametrize("idx", range(6))
def test_degree_dense(idx):
    n = 7 + idx
    A = gen.dense_matrix(0x5EED0202, idx, n - 4, n, -2, 2)
    say("degree dense", idx)
    assert _gres(bd.degree(A, seed=3, lift_bits=24)) == _ores(A)


def test_degree_k1_closed_form():
    A = gen.dense_matrix(0x5EED0203, 0, 7, 8, -2, 2)
    g = bd.degree(A)
    k, _, _, P = bd.kernel_points(A)
    v = P[:, 0]
    assert g["k"] == 1 and g["nvol"] == max(0, v.max()) - min(0, v.min())


@pytest.mark.parametrize("n", [1, 4, 9, 12])
def test_degree_zero_matrix(n):
    g = bd.degree(np.zeros((1, n), dtype=np.int64))
    assert (g["k"], g["rank"], g["comps"], g["nvol"]) == (n, 0, 1, 1)


def test_degree_components_and_consistency_flag():
    A = np.array([[2, 0, 0, 1], [0, 3, 0, 1], [2, 3, 0, 2]], dtype=np.int64)  # row 3 = row 1 + row 2
    g = bd.degree(A)
    assert g["rank"] == 2 and g["flags"] & bd.BDEG_F_NEEDS_CONSISTENCY
    assert _gres(g) == _ores(A)


def test_degree_independent_of_seed_and_width():
    A = gen.quiver_matrix(0x5EED0204, 0, 16, 10, 2, 3)
    vals = {bd.degree(A, seed=s, lift_bits=b)["nvol"] for s, b in [(1, 20), (2, 24), (3, 12), (4, 30), (5, 8)]}
    assert len(vals) == 1
    assert vals.pop() == _ores(A)[2]


def test_degree_errors():
    with pytest.raises(bd.BdegError) as e:  # k = 19 > BDEG_MAX_K = 18
        bd.degree(np.zeros((1, 19), dtype=np.int64))
    assert e.value.code == bd.BDEG_E_TOO_LARGE
    assert bd.degree(np.zeros((1, 18), dtype=np.int64))["nvol"] == 1  # k = 18: the standard simplex
    with pytest.raises(bd.BdegError) as e:
        bd.degree(np.zeros((1, 5), dtype=np.int64), lift_bits=1)
    assert e.value.code == bd.BDEG_E_ARG


@pytest.mark.parametrize("mk", ["1,2", "1,3", "1,4", "1,5", "1,6", "1,7", "1,8", "2,2", "2,3", "3,2", "2,4", "4,2",
                                "3,3", "2,5"])
def test_master_space_degrees_gpu(mk):
    """Table 4 of the paper (Section 6): degree of V(dW_{m,k})."""
    m, k = map(int, mk.split(","))
    say("master space", mk)
    g = bd.degree(gen.master_space_matrix(m, k), seed=7, lift_bits=24)
    assert g["comps"] == 1
    assert g["k"] == PAPER["table2_dims"][str(m)][k - 1]
    assert g["nvol"] == PAPER["table4_degrees"][mk]


@pytest.mark.parametrize("mk", ["2,6", "3,4", "4,3", "6,2", "2,7", "7,2", "3,5"])
def test_master_space_degrees_beyond_k12(mk):
    """Table 4 entries with k = 14 (9.4e9 candidates), k = 16 (4.2e11) and
    k = 17 (2.8e12, about 75 s), decided exhaustively on the device; the
    expected degrees are the paper's printed values (beyond the oracle's
    reach)."""
    m, k = map(int, mk.split(","))
    say("master space beyond k = 12", mk)
    g = bd.degree(gen.master_space_matrix(m, k), seed=3, lift_bits=20)
    assert g["status"] == 0 and g["comps"] == 1
    assert g["k"] == PAPER["table2_dims"][str(m)][k - 1] > 12
    assert g["comps"] * g["nvol"] == PAPER["table4_degrees"][mk]


def test_batch_mixing_deep_and_shallow_systems():
    """One batch with k = 3..8 systems (the mixed-k kernel) and k = 13, 14
    systems (single-k kernels, their own launch ranges) gives the single
    results."""
    mats = [gen.master_space_matrix(2, 6), gen.master_space_matrix(2, 1), gen.master_space_matrix(1, 5)]
    for i in range(6):
        mats.append(gen.quiver_matrix(0xB7, i, 14 + i, 10, 2, 3))
    mats.append(gen.quiver_matrix(0xB8, 0, 20, 7, 1, 2))  # k = 13
    singles = [bd.degree(A, seed=4, lift_bits=20) for A in mats]
    assert {r["k"] for r in singles} >= {14, 13} and min(r["k"] for r in singles) <= 8
    batch = bd.degree_batch(mats, seed=4, lift_bits=20)
    for i, (b, s) in enumerate(zip(batch, singles)):
        assert b["status"] == s["status"] == 0, i
        assert (b["k"], b["comps"], b["nvol"]) == (s["k"], s["comps"], s["nvol"]), i
    assert batch[0]["nvol"] == PAPER["table4_degrees"]["2,6"]


# ------------------------------------------------------------------ batch
def _mixed(count, seed):
    mats = []
    for i in range(count):
        rng = gen.stream(seed, i, gen.PURPOSE_SIZES)
        n = rng.uniform_int(6, 16)
        k = rng.uniform_int(0, 6)
        mats.append(gen.quiver_matrix(seed, i, n, n - k, 2, 3) if k < n else np.zeros((1, n), dtype=np.int64))
    return mats


def test_batch_matches_singles_and_oracle():
    mats = _mixed(48, 0x5EED0301)
    say("batch 48")
    br = bd.degree_batch(mats, seed=11, lift_bits=20)
    for A, r in zip(mats, br):
        assert r["status"] == 0
        assert _gres(r) == _gres(bd.degree(A, seed=99, lift_bits=16))
        assert _gres(r) == _ores(A)


def test_prepared_batch_graph_replays():
    mats = _mixed(40, 0x5EED0302)
    expect = [_ores(A) for A in mats]
    b = bd.Batch(mats, seed=5, lift_bits=20)
    try:
        for rep in range(4):
            say("batch replay", rep)
            b.run()
            res = b.results()
            assert [_gres(r) for r in res] == expect
            st = b.stats()
            assert st["kernel_ms"] > 0
            assert st["captured"] == 1  # the pass replays its captured graphs
        st = b.profile()
        assert st["tiles"] > 0 and st["leaves"] > 0
        b.run()  # the profiling pass leaves the captured pass intact
        assert [_gres(r) for r in b.results()] == expect
    finally:
        b.close()


# ------------------------------------------------------------------ stored workload values
def _golden(name):
    p = os.path.join(GOLD, f"{name}_expected.json")
    if not os.path.exists(p):
        pytest.skip(f"{p} not generated")
    d = json.load(open(p))
    assert d["gen_version"] == gen.GEN_VERSION
    return d["systems"]


def test_cfg1_plain_6x12():
    e = _golden("cfg1")[0]
    say("cfg1")
    g = bd.degree(gen.cfg1_system().A, seed=1, lift_bits=16)
    assert (g["k"], g["comps"], g["nvol"]) == (e["k"], e["comps"], e["nvol"])


def test_cfg2_quiver_28():
    e = _golden("cfg2")[0]
    say("cfg2")
    g = bd.degree(gen.cfg2_system().A, seed=1, lift_bits=20)
    assert (g["k"], g["comps"], g["nvol"]) == (e["k"], e["comps"], e["nvol"])
    assert g["candidates"] == e["candidates"] == 10015005


def test_cfg4_large_36():
    e = _golden("cfg4")[0]
    say("cfg4")
    g = bd.degree(gen.cfg4_system().A, seed=1, lift_bits=24)
    assert (g["k"], g["comps"], g["nvol"]) == (e["k"], e["comps"], e["nvol"])


def test_degree_cost_model_prunes_large_systems():
    """A one-shot system of at least BDEG_PRUNE_MIN_CANDIDATES candidates goes
    through the prefix-pruned enumeration (BDEG_F_PRUNED) with the plain
    path's result, attempts and cells included; the plain path here is the
    lanes-as-points schedule, which never prunes.  12-bit heights make ties
    and redraws likely."""
    A = gen.cfg4_system().A
    assert math.comb(37, 11) >= bd.PRUNE_MIN_CANDIDATES
    for bits in (24, 12):
        say("cost model", bits)
        g = bd.degree(A, seed=3, lift_bits=bits, check=False)
        bd.set_schedule(bd.SCHED_POINTS)
        try:
            p = bd.degree(A, seed=3, lift_bits=bits, check=False)
        finally:
            bd.set_schedule(bd.SCHED_AUTO)
        assert g["flags"] & bd.BDEG_F_PRUNED and not p["flags"] & bd.BDEG_F_PRUNED
        assert (g["status"], g["k"], g["comps"], g["nvol"], g["attempts"], g["cells"]) == \
            (p["status"], p["k"], p["comps"], p["nvol"], p["attempts"], p["cells"])
        if g["status"] == 0:
            assert g["nvol"] == _golden("cfg4")[0]["nvol"]
    small = bd.degree(gen.cfg2_system().A, seed=3, lift_bits=20)
    assert not small["flags"] & bd.BDEG_F_PRUNED


def test_cfg3_batch_4096():
    exp = _golden("cfg3")
    say("cfg3 batch")
    systems = gen.cfg3_systems(len(exp))
    b = bd.Batch([s.A for s in systems], seed=3, lift_bits=20)
    try:
        b.run()
        res = b.results()
    finally:
        b.close()
    for e, r in zip(exp, res):
        assert r["status"] == 0
        assert (r["k"], r["comps"], r["nvol"]) == (e["k"], e["comps"], e["nvol"]), e["index"]


def test_prepared_batch_redraws_ties_inside_the_graph():
    """4-bit heights make ties frequent: the captured pass redraws the tied
    systems' liftings itself (up to three rounds), so each replay gives
    exactly the one-shot results, attempts and cell counts included, and
    reports the systems it redrew."""
    mats = [gen.quiver_matrix(0x5EED0303, i, 12 + i % 9, 4 + i % 4, 2, 3) for i in range(40)]
    alone = [bd.degree(A, seed=13, lift_bits=4, check=False) for A in mats]
    assert sum(a["attempts"] > 1 for a in alone) >= 5
    b = bd.Batch(mats, seed=13, lift_bits=4)
    try:
        for rep in range(3):
            say("batch ties replay", rep)
            b.run()
            res = b.results()
            st = b.stats()
            assert st["captured"] == 1
            assert st["redraws"] == sum(a["attempts"] > 1 for a in alone)
            for a, r in zip(alone, res):
                assert (r["status"], r["nvol"], r["attempts"], r["cells"]) == \
                    (a["status"], a["nvol"], a["attempts"], a["cells"])
    finally:
        b.close()
    for A, r in zip(mats[:8], res[:8]):
        if r["status"] == 0:
            assert _gres(r) == _ores(A)


def test_batch_tuner_writes_a_table_and_keeps_results(tmp_path):
    """The autotuner times every schedule of its grid on each (k, lane-group
    width) bucket of the batch (each must reproduce the default's sums),
    writes the fastest per bucket to a JSON table and applies it; the tuned
    batch still equals the oracle."""
    mats = _mixed(60, 0x5EED0304)
    expect = [_ores(A) for A in mats]
    path = str(tmp_path / "table.json")
    b = bd.Batch(mats, seed=7, lift_bits=20)
    try:
        say("tuner: tuning")
        b.tune(path, reps=2)
        b.run()
        assert [_gres(r) for r in b.results()] == expect
        assert b.stats()["captured"] == 1
    finally:
        b.close()
    table = json.load(open(path))
    ks = {r["k"] for r in (bd.degree(A) for A in mats) if r["k"] >= 1}
    assert {e["k"] for e in table["entries"]} == ks
    for e in table["entries"]:
        assert e["npad_min"] <= e["npad"] <= 6 and e["ms"] > 0 and e["systems"] > 0
        assert e["dense"] in (-1, 0, 1)


# ------------------------------------------------------------------ serving
def test_serving_mix_equals_alone():
    """Requests submitted together (they share device steps) give exactly the
    results of solving each one alone; the small ones also match the oracle."""
    rng = gen.stream(0x5EED0401, 0, gen.PURPOSE_SIZES)
    mats = []
    for i in range(40):
        n = rng.uniform_int(8, 24)
        k = rng.uniform_int(1, 7)
        mats.append(gen.quiver_matrix(0x5EED0401, i, n, n - k, 2, 3))
    mats.append(np.zeros((1, 6), dtype=np.int64))          # k = n
    mats.append(np.array([[1, 1], [0, 1]], dtype=np.int64))  # k = 0
    alone = [bd.degree(A, seed=17, lift_bits=20) for A in mats]
    srv = bd.Server(64 << 20)
    try:
        tickets = [srv.submit(A, seed=17, lift_bits=20) for A in mats]
        say("serving: submitted", len(tickets))
        got = [srv.wait(t) for t in tickets]
        lat = [srv.latency_ms(t) for t in tickets]
    finally:
        srv.close()
    for A, a, g in zip(mats, alone, got):
        assert g["status"] == 0
        assert (g["k"], g["comps"], g["nvol"], g["attempts"], g["cells"]) == \
            (a["k"], a["comps"], a["nvol"], a["attempts"], a["cells"])
    for A, g in zip(mats[:12], got[:12]):
        assert _gres(g) == _ores(A)
    assert all(x is not None and x >= 0 for x in lat)


def test_two_servers_at_once():
    """Two engines open together (each with its own stream, slots and step
    counters) serve interleaved requests; each result equals the one-shot
    path."""
    mats = [gen.quiver_matrix(0x5EED0403, i, 10 + i % 12, 5 + i % 4, 2, 3) for i in range(24)]
    alone = [bd.degree(A, seed=9, lift_bits=20) for A in mats]
    s1, s2 = bd.Server(32 << 20), bd.Server(32 << 20)
    try:
        t = [(s1 if i % 2 else s2).submit(A, seed=9, lift_bits=20) for i, A in enumerate(mats)]
        say("two servers: submitted", len(t))
        got = [(s1 if i % 2 else s2).wait(x) for i, x in enumerate(t)]
    finally:
        s1.close()
        s2.close()
    for a, g in zip(alone, got):
        assert g["status"] == 0
        assert (g["k"], g["comps"], g["nvol"], g["attempts"]) == (a["k"], a["comps"], a["nvol"], a["attempts"])


def test_cfg5_serving_trace_against_oracle():
    """The serving workload (n in [12, 32], k in [4, 9]): a stated subset of
    its 4000 requests (the 20 largest and 400 seeded others, oracle values
    in tests/golden/cfg5_expected.json) is submitted to one engine in trace
    order with the arrival gaps compressed to zero, so that the requests
    share device steps; every (k, components, nvol) equals the oracle's."""
    exp = _golden("cfg5")
    trace = gen.cfg5_trace(4000)
    srv = bd.Server(256 << 20)
    try:
        tickets = [srv.submit(trace[e["index"]].system.A, seed=5, lift_bits=20) for e in exp]
        say("cfg5: submitted", len(tickets))
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    assert max(e["k"] for e in exp) == 9 and max(e["n"] for e in exp) == 32
    for e, g in zip(exp, got):
        assert g["status"] == 0, e["index"]
        assert (g["k"], g["comps"], g["nvol"]) == (e["k"], e["comps"], e["nvol"]), e["index"]


def test_serving_small_budget_and_ties():
    """A budget of a few slots forces admission to wait; 4-bit heights force
    tie redraws inside the engine; results still equal the one-shot path."""
    mats = [gen.quiver_matrix(0x5EED0402, i, 14, 9, 2, 3) for i in range(12)]
    alone = [bd.degree(A, seed=5, lift_bits=4, check=False) for A in mats]
    srv = bd.Server(3 * 4096 + 2048)
    try:
        tickets = [srv.submit(A, seed=5, lift_bits=4) for A in mats]
        got = [srv.wait(t) for t in tickets]
    finally:
        srv.close()
    for a, g in zip(alone, got):
        assert (g["status"], g["nvol"], g["attempts"]) == (a["status"], a["nvol"], a["attempts"])
    assert any(g["attempts"] > 1 for g in got)
