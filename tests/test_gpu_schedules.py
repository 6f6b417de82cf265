"""Both enumeration schedules against the oracle (exact integers).

The default schedule runs certified systems with k >= 3 in the lane-dense
kernel (the other parity tests exercise it); here the same kinds of cases
run under the lanes-as-points schedule, and a few under both, so that each
kernel is checked on its own: the volume sum, the cell count and the tie flag
of ``bdeg_nvol_points`` must equal ``oracle.nvol_range`` on identical heights,
and whole degrees must equal the oracle's."""
import numpy as np
import pytest
from sympy import Matrix

import gen
import oracle
import paper_1501_02237_amd as bd

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available(), "gpu tests need a GPU"
    oracle.build(force=False)
    bd.lib()
    yield
    bd.set_schedule(bd.SCHED_AUTO)


@pytest.fixture(params=[bd.SCHED_POINTS, bd.SCHED_AUTO], ids=["points", "auto"])
def schedule(request):
    bd.set_schedule(request.param)
    yield request.param
    bd.set_schedule(bd.SCHED_AUTO)


def _points(seed, N, k, lo=-2, hi=2):
    if k >= 7:
        lo, hi = max(lo, -1), min(hi, 1)
    rng = gen.stream(seed, N * 100 + k, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k] + [[rng.uniform_int(lo, hi) for _ in range(k)] for _ in range(N - 1)]
        if Matrix(P).rank() == k:
            return np.array(P, dtype=np.int64)


def _same(P, H, lo=0, hi=None):
    g = bd.nvol_points(P, H, lo, hi)
    o = oracle.nvol_range(P, H, lo, hi)
    assert (g.nvol, g.cells, g.tie) == (o.nvol, o.cells, o.tie), (g, o)
    return g


SHAPES = [(5, 3, 12), (8, 3, 16), (12, 4, 16), (17, 5, 20), (24, 6, 20), (31, 4, 24), (33, 3, 24), (40, 4, 20),
          (48, 3, 20), (64, 3, 24), (13, 6, 16), (14, 7, 16), (16, 9, 16), (15, 10, 16), (14, 12, 16)]


@pytest.mark.parametrize("N,k,bits", SHAPES)
def test_full_range_both_schedules(schedule, N, k, bits):
    say("schedule", schedule, "full", N, k, bits)
    P = _points(0x5C1 + N, N, k)
    H = gen.random_heights(0x5C2 + N * 7 + k, N, bits)
    _same(P, H)


@pytest.mark.parametrize("N,k", [(37, 10), (29, 8), (64, 5), (40, 6)])
def test_rank_slices_both_schedules(schedule, N, k):
    """Ragged colex slices: units whose prefix fixes one, two or three of the
    last three elements of a candidate."""
    P = _points(0x5C3 + N, N, k, -3, 3)
    H = gen.random_heights(0x5C4 + N, N, 24)
    total = oracle.binom(N, k + 1)
    rng = gen.stream(0x5C5, N * 31 + k, gen.PURPOSE_MATRIX)
    for _ in range(3):
        lo = rng.next() % total
        hi = min(total, lo + 1 + rng.next() % 40000)
        say("schedule", schedule, "slice", N, k, lo, hi)
        _same(P, H, lo, hi)
    for lo, hi in [(0, 1), (total - 1, total), (total - 333, total), (5, 6), (17, 90)]:
        _same(P, H, lo, hi)


@pytest.mark.parametrize("seed", range(4))
def test_ties_both_schedules(schedule, seed):
    """2- and 3-bit heights on grids in Z^3 and Z^4: frequent ties; flag,
    partial sum and cell count equal the oracle's."""
    P3 = np.array([[x, y, z] for x in range(2) for y in range(2) for z in range(3)], dtype=np.int64)
    P4 = np.array([[x, y, z, w] for x in range(2) for y in range(2) for z in range(2) for w in range(2)],
                  dtype=np.int64)
    for bits in (2, 3):
        say("schedule", schedule, "ties", seed, bits)
        _same(P3, gen.random_heights(0x5C6 + seed * 4 + bits, len(P3), bits))
        _same(P4, gen.random_heights(0x5C7 + seed * 4 + bits, len(P4), bits))


def test_schedules_give_identical_degrees():
    """Whole degrees of quiver-like systems (k = 3..9, both lane-group
    packings) are the same under both schedules, attempts and cells included,
    and equal the oracle's."""
    mats = [gen.quiver_matrix(0x5C8, i, 10 + 2 * i, 10 + 2 * i - (3 + i % 7), 2, 3) for i in range(10)]
    try:
        bd.set_schedule(bd.SCHED_POINTS)
        pts = [bd.degree(A, seed=4, lift_bits=20) for A in mats]
        bd.set_schedule(bd.SCHED_AUTO)
        den = [bd.degree(A, seed=4, lift_bits=20) for A in mats]
    finally:
        bd.set_schedule(bd.SCHED_AUTO)
    for A, a, b in zip(mats, pts, den):
        assert (a["k"], a["comps"], a["nvol"], a["attempts"], a["cells"]) == \
            (b["k"], b["comps"], b["nvol"], b["attempts"], b["cells"])
    for A, b in zip(mats[:6], den[:6]):
        o = oracle.oracle_degree(A, bits=20)
        assert (b["k"], b["comps"], b["nvol"]) == (o["k"], o["comps"], o["nvol"])


def test_cells_under_both_schedules():
    """The emitting variant of each kernel lists the same cells (as a set,
    with the same exact inner normals) as the oracle."""
    P = _points(0x5C9, 14, 5)
    H = gen.random_heights(0x5CA, 14, 16)
    want = oracle.cells_range(P, H).as_set()
    try:
        for s in (bd.SCHED_POINTS, bd.SCHED_AUTO):
            bd.set_schedule(s)
            say("cells schedule", s)
            got = bd.cells_points(P, H)
            assert not got.tie and got.as_set() == want
    finally:
        bd.set_schedule(bd.SCHED_AUTO)
