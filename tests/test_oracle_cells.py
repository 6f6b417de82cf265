"""Pins of the oracle's cell list (lower facets with inner normals).

The cells of the regular subdivision are the lower facets of the lifted point
set; each has a unique inner normal (alpha, 1) (Section 5, eq.
``lower-d-face-again``), listed as alpha = num / den with den the cell's
normalized volume.  Pinned against hand-worked lower hulls of the paper's
unit-square example, against qhull's convex hull of the lifted points, and
against the defining equalities and strict inequalities in exact rationals.
"""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import ConvexHull
from sympy import Matrix

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def _verts(mask):
    return [i for i in range(64) if (int(mask) >> i) & 1]


def _random_case(seed, N, k, span, hbits):
    rng = gen.stream(0xCE11 + seed, N * 131 + k, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k] + [[rng.uniform_int(-span, span) for _ in range(k)] for _ in range(N - 1)]
        if Matrix(P[1:]).rank() == k and len({tuple(p) for p in P}) == N:
            break
    H = [int(x) for x in gen.random_heights(0xCE22 + seed, N, hbits)]
    return P, H


def test_hand_worked_cells(oracle_mod):
    cases = json.load(open(os.path.join(HERE, "golden", "cells_examples.json")))["cases"]
    for c in cases:
        got = oracle.cells_range(c["points"], c["heights"])
        assert not got.tie, c["name"]
        want = {(sum(1 << v for v in x["vertices"]), tuple(x["num"]), x["den"]) for x in c["cells"]}
        assert got.as_set() == want, c["name"]


@pytest.mark.parametrize("seed,N,k", [(0, 7, 2), (1, 9, 2), (2, 8, 3), (3, 10, 3), (4, 9, 4), (5, 11, 4)])
def test_cells_satisfy_the_definition(oracle_mod, seed, N, k):
    """Each cell: <a_v, alpha> + w_v equal on the vertices and strictly larger
    at every other point (exact rationals), and den = |det| of the simplex."""
    P, H = _random_case(seed, N, k, 3, 12)
    cells = oracle.cells_range(P, H)
    assert not cells.tie and len(cells.masks) > 0
    for m, num, den in zip(cells.masks, cells.num, cells.den):
        vs = _verts(m)
        assert len(vs) == k + 1
        alpha = [Fraction(int(x), int(den)) for x in num]
        val = [sum(a * p for a, p in zip(alpha, P[j])) + H[j] for j in range(N)]
        beta = val[vs[0]]
        for j in range(N):
            if j in vs:
                assert val[j] == beta
            else:
                assert val[j] > beta
        M = Matrix([[P[v][q] - P[vs[0]][q] for q in range(k)] for v in vs[1:]])
        assert abs(M.det()) == int(den)


@pytest.mark.parametrize("seed,N,k", [(10, 8, 2), (11, 12, 2), (12, 9, 3), (13, 12, 3)])
def test_cells_match_qhull_lower_hull(oracle_mod, seed, N, k):
    """Vertex sets of the lower facets of qhull's hull of the lifted points."""
    P, H = _random_case(seed, N, k, 4, 16)
    lifted = np.array([p + [h] for p, h in zip(P, H)], dtype=np.float64)
    hull = ConvexHull(lifted)
    lower = set()
    for simplex, eq in zip(hull.simplices, hull.equations):
        if eq[k] < -1e-9:  # outward normal points down: a lower facet
            lower.add(sum(1 << int(v) for v in simplex))
    cells = oracle.cells_range(P, H)
    assert not cells.tie
    assert {int(m) for m in cells.masks} == lower


@pytest.mark.parametrize("seed,N,k", [(20, 10, 3), (21, 13, 4), (22, 11, 5)])
def test_cells_sum_to_the_volume_and_partition_by_rank(oracle_mod, seed, N, k):
    P, H = _random_case(seed, N, k, 2, 20)
    whole = oracle.cells_range(P, H)
    part = oracle.nvol_range(P, H)
    assert int(sum(int(d) for d in whole.den)) == part.nvol
    assert len(whole.masks) == part.cells
    total = oracle.binom(N, k + 1)
    cuts = [0, total // 3, total // 2, total]
    pieces = set()
    for lo, hi in zip(cuts, cuts[1:]):
        pieces |= oracle.cells_range(P, H, lo, hi).as_set()
    assert pieces == whole.as_set()


def test_cells_flag_a_tie(oracle_mod):
    got = oracle.cells_range([[0, 0], [0, 1], [1, 1], [1, 0]], [0, 0, 0, 0])
    assert got.tie


def test_cells_grow_past_the_first_buffer(oracle_mod):
    pts, H = _random_case(30, 12, 3, 3, 20)
    cells = oracle.cells_range(pts, H, cap=2)
    part = oracle.nvol_range(pts, H)
    assert len(cells.masks) == part.cells > 2
    assert cells.as_set() == oracle.cells_range(pts, H).as_set()
    assert sum(int(d) for d in cells.den) == part.nvol
