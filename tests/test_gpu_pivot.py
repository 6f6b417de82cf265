"""Parity of the cell walk (simplicial pivoting, Section 4.2-4.4) with the oracle.

The walk visits the cells of the regular subdivision across their facets
from one start cell.  For a given lifting the cells are unique, so the walk's
cell set must equal the oracle's lower facets bit for bit, and the volumes
must agree.  Some tests build their own start cell and heights (height 0 on
an affinely independent set, so that set is a lower facet; positive seeded
heights elsewhere); the others give raw seeded heights and let Extend find
the start cell.  At sizes beyond the oracle the expected values are the
exhaustive device path's and the paper's Table 4.
"""
import json
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
    oracle.build(force=False)
    bd.lib()


def _independent_set(P):
    """Point 0 and, scanning backwards from the last point, each point that
    raises the affine rank (sympy ranks)."""
    k = len(P[0])
    chosen = [0]
    for j in range(len(P) - 1, 0, -1):
        M = Matrix([[P[c][q] - P[0][q] for q in range(k)] for c in chosen[1:] + [j]])
        if M.rank() == len(chosen):
            chosen.append(j)
        if len(chosen) == k + 1:
            break
    return chosen


def _lifting(P, seed, bits):
    start = _independent_set(P)
    r = gen.random_heights(seed, len(P), bits)
    H = np.array([0 if j in start else 1 + int(r[j]) for j in range(len(P))], dtype=np.int64)
    return sum(1 << j for j in start), H


def _points(seed, N, k, lo=-2, hi=2):
    if k >= 7:
        lo, hi = max(lo, -1), min(hi, 1)
    rng = gen.stream(seed, N * 100 + k, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k] + [[rng.uniform_int(lo, hi) for _ in range(k)] for _ in range(N - 1)]
        if Matrix(P).rank() == k:
            return P


@pytest.mark.parametrize("N,k,bits", [(5, 1, 12), (8, 2, 16), (12, 3, 16), (16, 4, 20), (20, 5, 20), (24, 6, 20),
                                       (33, 4, 20), (40, 3, 20), (18, 8, 16), (16, 10, 16), (64, 2, 24),
                                       # heights of 1-2 bits: non-generic liftings, the tie must be reported
                                       (12, 2, 1), (10, 3, 1), (16, 3, 2), (9, 2, 2)])
def test_walk_matches_oracle_cells(N, k, bits):
    P = _points(0x9A1 + N, N, k)
    start, H = _lifting(P, 0x9A2 + N * 7 + k, bits)
    say("walk", N, k, bits)
    g = bd.pivot_points(P, H, start, cap=1 << 20)
    o = oracle.cells_range(P, H)
    assert g["tie"] == o.tie
    if not o.tie:
        assert {int(m) for m in g["masks"]} == {int(m) for m in o.masks}
        assert g["cells"] == len(o.masks)
        assert g["nvol"] == sum(int(d) for d in o.den)


def test_walk_rejects_a_start_that_is_not_a_lower_facet():
    P = _points(0x9A3, 12, 3)
    start, H = _lifting(P, 0x9A4, 16)
    H = H.copy()
    H[[j for j in range(12) if (start >> j) & 1][0]] += 1 << 24  # lift one start vertex far up
    with pytest.raises(bd.BdegError) as e:
        bd.pivot_points(P, H, start)
    assert e.value.code == bd.BDEG_E_ARG


@pytest.mark.parametrize("idx", range(6))
def test_degree_pivot_equals_exhaustive(idx):
    rng = gen.stream(0x9A5, idx, gen.PURPOSE_SIZES)
    n = rng.uniform_int(10, 26)
    k = rng.uniform_int(2, 8)
    A = gen.quiver_matrix(0x9A6, idx, n, n - k, 2, 3)
    say("pivot vs exhaustive", n, k)
    p = bd.degree_pivot(A, seed=2)
    e = bd.degree(A, seed=2)
    assert (p["k"], p["comps"], p["nvol"]) == (e["k"], e["comps"], e["nvol"])


def test_degree_pivot_golden_systems():
    for name, s in (("cfg1", gen.cfg1_system()), ("cfg2", gen.cfg2_system()), ("cfg4", gen.cfg4_system())):
        gold = json.load(open(os.path.join(GOLD, f"{name}_expected.json")))["systems"][0]
        r = bd.degree_pivot(s.A, seed=1, lift_bits=s.lift_bits)
        say(name, r["nvol"], r["cells"])
        assert (r["k"], r["comps"], r["nvol"]) == (gold["k"], gold["comps"], gold["nvol"])


@pytest.mark.parametrize("mk", sorted(PAPER["table4_degrees"], key=lambda s: tuple(map(int, s.split(",")))))
def test_degree_pivot_table4(mk):
    """Every degree of the paper's Table 4 by the cell walk, up to W_{4,5} and
    W_{5,4} (k = 22, about 5e7 cells), beyond the exhaustive path's k <= 18."""
    m, k = map(int, mk.split(","))
    say("table 4 by pivoting", mk)
    r = bd.degree_pivot(gen.master_space_matrix(m, k), seed=5, lift_bits=20)
    assert r["status"] == 0 and r["comps"] * r["nvol"] == PAPER["table4_degrees"][mk]


# ------------------------------------------------------------------ Extend: the walk from a caller's lifting
EXT_CASES = [(5, 1, 16), (8, 2, 16), (12, 3, 16), (16, 4, 20), (20, 5, 20), (24, 6, 20), (33, 4, 20),
             (40, 3, 20), (18, 8, 16), (16, 10, 16), (64, 2, 24), (14, 12, 16), (29, 8, 20)]


@pytest.mark.parametrize("N,k,bits", EXT_CASES)
def test_extend_finds_one_of_the_oracles_cells(N, k, bits):
    """Extend on raw seeded heights (no constructed zeros): the facet it
    returns is one of the oracle's lower facets for the same lifting."""
    P = _points(0x9B1 + N, N, k)
    H = gen.random_heights(0x9B2 + N * 7 + k, N, bits)
    say("extend", N, k, bits)
    e = bd.extend_points(P, H)
    o = oracle.cells_range(P, H)
    assert not o.tie and not e["tie"]
    assert e["mask"] in {int(m) for m in o.masks}


@pytest.mark.parametrize("N,k,bits", EXT_CASES + [(12, 2, 1), (10, 3, 1), (16, 3, 2), (9, 2, 2), (20, 4, 3)])
def test_walk_from_extend_matches_oracle_cells_and_normals(N, k, bits):
    """The walk from Extend's facet, on a random lifting of the caller: its
    cells with their inner normals (mask, numerators, denominator) equal the
    oracle's lower facets bit for bit; with 1-3-bit heights the lifting is
    not generic and both report the tie."""
    P = _points(0x9B3 + N, N, k)
    H = gen.random_heights(0x9B4 + N * 7 + k, N, bits)
    say("walk from extend", N, k, bits)
    g = bd.pivot_cells(P, H)
    o = oracle.cells_range(P, H)
    assert g["tie"] == o.tie
    if not o.tie:
        assert g["cell_list"].as_set() == o.as_set()
        assert g["nvol"] == sum(int(d) for d in o.den) and g["cells"] == len(o.masks)


def test_walk_normals_deep_k_against_the_enumeration():
    """k = 14 and 16 master-space systems (beyond the oracle's reach): the
    walk's cells and normals from Extend equal the enumeration's cell list
    for the same points and heights."""
    for m, kk in ((2, 6), (3, 4)):
        sub = bd.subdivision(gen.master_space_matrix(m, kk), seed=3, lift_bits=20, cap=1 << 16)
        say("walk normals vs enumeration", m, kk, sub["k"])
        g = bd.pivot_cells(sub["points"], sub["heights"])
        assert not g["tie"]
        assert g["cell_list"].as_set() == sub["cell_list"].as_set()
        assert g["nvol"] == sub["nvol"]


@pytest.mark.parametrize("idx", range(8))
def test_degree_pivot_is_the_same_subdivision_as_degree(idx):
    """bdeg_degree_pivot draws bdeg_degree's lifting and starts from Extend:
    the same regular subdivision, so nvol, the cell count and the number of
    draws agree (8-bit heights make redraws likely)."""
    rng = gen.stream(0x9B5, idx, gen.PURPOSE_SIZES)
    n = rng.uniform_int(10, 24)
    k = rng.uniform_int(2, 7)
    A = gen.quiver_matrix(0x9B6, idx, n, n - k, 2, 3)
    bits = 8 if idx % 2 else 20
    say("degree_pivot vs degree", idx, n, k, bits)
    p = bd.degree_pivot(A, seed=idx, lift_bits=bits, check=False)
    e = bd.degree(A, seed=idx, lift_bits=bits, check=False)
    assert (p["status"], p["k"], p["comps"], p["nvol"], p["cells"], p["attempts"]) == \
        (e["status"], e["k"], e["comps"], e["nvol"], e["cells"], e["attempts"])


@pytest.mark.parametrize("mk", ["2,8", "3,5", "4,4", "3,6"])
def test_walk_from_extend_on_random_heights_table4(mk):
    """The walk of a Table 4 system's points from Extend's facet on fully
    random 30-bit heights (the origin is not lifted lowest, so the cells do
    not share a point): wide levels, pivots and base changes between claimed
    cells at scale.  The cells' normalized volumes sum to the volume of the
    points' convex hull whatever the lifting, so comps * nvol is the paper's
    degree (Section 2, the degree as a normalized volume)."""
    m, k = map(int, mk.split(","))
    kk, _, comps, P = bd.kernel_points(gen.master_space_matrix(m, k))
    for attempt in range(3):
        H = gen.random_heights(0x9D1 + 17 * m + k + 1000 * attempt, len(P), 30)
        say("walk on random heights", mk, kk, len(P), attempt)
        g = bd.pivot_points(P, H, 0)
        if not g["tie"]:
            break
    assert not g["tie"]
    assert comps * g["nvol"] == PAPER["table4_degrees"][mk]
    assert 0 < g["cells"] <= g["nvol"]


def test_walk_two_random_liftings_agree_off_the_pyramid():
    """Table 4 configurations are pyramids (every point but the origin lies on
    one hyperplane, so every cell holds the origin).  With the mirror image
    -p of one point added the cells share no point, so the walk changes its
    base between claimed cells.  The origin then lies inside, between p and
    -p, so the hull is the pyramid over the same base with apex -p at twice
    the origin's distance: its normalized volume is twice the configuration's,
    2 * degree / comps, for any lifting."""
    _, _, comps, P = bd.kernel_points(gen.master_space_matrix(3, 5))
    deg = PAPER["table4_degrees"]["3,5"]
    assert deg % comps == 0
    P2 = np.vstack([P, -P[1:2]]).astype(np.int32)
    vols = []
    for seed in (0x9E1, 0x9E2):
        for attempt in range(3):
            H = gen.random_heights(seed + 1000 * attempt, len(P2), 30)
            say("walk off the pyramid", seed, attempt, len(P2))
            g = bd.pivot_points(P2, H, 0)
            if not g["tie"]:
                break
        assert not g["tie"]
        assert 0 < g["cells"] <= g["nvol"]
        vols.append(g["nvol"])
    assert vols[0] == vols[1] == 2 * deg // comps
