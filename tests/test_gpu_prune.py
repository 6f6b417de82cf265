"""Parity of the prefix-pruned enumeration (Section 4.1) with the oracle.

The pruned path decides whole subtrees at once: a prefix certified (in exact
integer arithmetic) to lie in no lower face heads no lower facet and no tie.
Its volume, cell count and tie flag must therefore equal the oracle's and the
unpruned device path's on the same points and heights, for every prefix width,
and no prefix that is a lower face (a subset of one of the oracle's cells) may
be pruned.
"""
import itertools
import json
import os

import numpy as np
import pytest

import gen
import oracle
import paper_1501_02237_amd as bd
from test_gpu_pivot import _lifting, _points

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    say("gpu fixture: importing torch")
    import torch

    assert torch.cuda.is_available(), "gpu tests need a GPU"
    oracle.build(force=False)
    bd.lib()


def _face_prefixes(masks, N, d, W):
    """Prefixes of size d (lowest point >= W) that lie in some cell."""
    faces = set()
    for m in masks:
        idx = [i for i in range(N) if (int(m) >> i) & 1]
        for c in itertools.combinations(idx, d):
            if c[0] >= W:
                faces.add(c)
    return len(faces)


@pytest.mark.parametrize("N,k,bits", [(8, 2, 16), (12, 3, 16), (16, 4, 20), (20, 5, 20), (24, 6, 20), (30, 6, 20),
                                       (18, 8, 16), (40, 3, 20), (36, 5, 20), (16, 10, 16), (64, 2, 24),
                                       (12, 2, 1), (10, 3, 1), (16, 3, 2)])
def test_pruned_matches_oracle(N, k, bits):
    P = _points(0xA11 + N, N, k)
    H = gen.random_heights(0xA12 + N * 7 + k, N, bits).astype(np.int64)
    say("pruned", N, k, bits)
    g = bd.nvol_points_pruned(P, H)
    o = oracle.cells_range(P, H)
    u = bd.nvol_points(P, H)
    assert g["tie"] == o.tie == u.tie
    assert (g["nvol"], g["cells"]) == (u.nvol, u.cells)
    if not o.tie:
        assert g["nvol"] == sum(int(d) for d in o.den) and g["cells"] == len(o.masks)
        st = g["stats"]
        W, d = st["width"], st["prefix_size"]
        kept = st["prefixes"] - st["degenerate"] - st["pruned"]
        assert kept >= _face_prefixes(o.masks, N, d, W), st  # no lower-face prefix was pruned


@pytest.mark.parametrize("width", range(1, 9))
def test_pruned_every_width(width):
    P = _points(0xA13, 24, 8)
    H = gen.random_heights(0xA14, 24, 20).astype(np.int64)
    u = bd.nvol_points(P, H)
    g = bd.nvol_points_pruned(P, H, width=width)
    say("width", width, g["stats"])
    assert g["stats"]["width"] == width
    assert (g["nvol"], g["cells"], g["tie"]) == (u.nvol, u.cells, u.tie)


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg4"])
def test_pruned_golden_systems(name):
    s = {"cfg1": gen.cfg1_system, "cfg2": gen.cfg2_system, "cfg4": gen.cfg4_system}[name]()
    gold = json.load(open(os.path.join(GOLD, f"{name}_expected.json")))["systems"][0]
    sub = bd.subdivision(s.A, seed=1, lift_bits=s.lift_bits, cap=0)
    g = bd.nvol_points_pruned(sub["points"], sub["heights"])
    say(name, g["nvol"], g["stats"])
    assert not g["tie"] and g["nvol"] == gold["nvol"] and g["cells"] == sub["cells"]
    assert g["stats"]["pruned"] > 0


def test_pruned_table4_entries():
    paper = json.load(open(os.path.join(GOLD, "paper_values.json")))["table4_degrees"]
    for mk in ["2,2", "2,3", "3,3", "2,4", "2,5"]:
        m, k = map(int, mk.split(","))
        sub = bd.subdivision(gen.master_space_matrix(m, k), seed=3, lift_bits=20, cap=0)
        g = bd.nvol_points_pruned(sub["points"], sub["heights"])
        say(mk, g["nvol"], g["stats"])
        assert not g["tie"] and sub["comps"] * g["nvol"] == paper[mk]
