"""The no-allocation entry point (bdeg_nvol_points_noalloc, for callers that
cannot allocate device memory) against bdeg_nvol_points through the C ABI:
the same volume sum, cell count and tie flag (exact integers), on calls in a
row that reuse the library's static device array, the later ones smaller
than the first."""
import numpy as np
import pytest

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


def _pair(P, H, lo=0, hi=None):
    a = bd.nvol_points_noalloc(P, H, lo, hi)
    b = bd.nvol_points(P, H, lo, hi)
    assert (a.nvol, a.cells, a.tie) == (b.nvol, b.cells, b.tie), (a, b)
    return a


def test_noalloc_two_calls_second_smaller():
    """First the n = 28 quiver system's points (10,015,005 candidates, tens of
    thousands of work units in the array), then a 13-point system (1716
    candidates): the second call must not see the first one's sums, counters
    or units."""
    k1, _, _, P1 = bd.kernel_points(gen.cfg2_system().A)
    H1 = gen.random_heights(0x0A11, len(P1), 20)
    say("noalloc call 1: N", len(P1), "k", k1)
    g1 = _pair(P1, H1)
    assert g1.nvol > 0 and not g1.tie
    k2, _, _, P2 = bd.kernel_points(gen.cfg1_system().A)
    H2 = gen.random_heights(0x0A12, len(P2), 16)
    say("noalloc call 2: N", len(P2), "k", k2)
    g2 = _pair(P2, H2)
    o2 = oracle.nvol_range(P2, H2)
    assert (g2.nvol, g2.cells, g2.tie) == (o2.nvol, o2.cells, o2.tie)


def test_noalloc_rank_slices_ties_and_empty_ranges():
    """Rank slices with ragged edges, an empty range, and a tie-prone 3-bit
    lifting (the tie flag must come back cleared on the next call)."""
    P = np.array([[x, y] for x in range(3) for y in range(3)], dtype=np.int64)
    saw_tie = False
    for a in range(6):
        H = gen.random_heights(0x7E0 + a, 9, 3)
        say("noalloc ties", a)
        saw_tie |= _pair(P, H).tie
    assert saw_tie
    Q = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 1], [-1, 2, 0], [2, -1, 1]], dtype=np.int64)
    Hq = gen.random_heights(0x7F1, len(Q), 12)
    total = oracle.binom(len(Q), 4)
    for lo, hi in [(0, total), (3, 17), (total - 1, total), (5, 5)]:
        say("noalloc slice", lo, hi)
        _pair(Q, Hq, lo, hi)
    assert bd.nvol_points_noalloc(Q, Hq, 5, 5).nvol == 0


def test_noalloc_rejects_plans_beyond_the_array():
    """A range that needs more than BDEG_NOALLOC_MAX_UNITS units even at the
    largest unit size is refused with BDEG_E_TOO_LARGE before any device work
    (W_{2,8}: 49 points in Z^18, 1.9e13 candidates)."""
    k, _, _, P = bd.kernel_points(gen.master_space_matrix(2, 8))
    assert k == 18
    H = gen.random_heights(0x7F2, len(P), 20)
    with pytest.raises(bd.BdegError) as e:
        bd.nvol_points_noalloc(P, H)
    assert e.value.code == bd.BDEG_E_TOO_LARGE
    # a slice of the same point set that fits runs and equals the allocating path
    _pair(P, H, 0, 3_000_000)
