"""Pin of the oracle's colex numbering (CPU only).

A rank slice [rho, rho + 1) of the oracle must visit exactly the (k+1)-subset
whose colex rank sum_i C(c_i, i+1) is rho, and a slice [0, rho + 1) must visit
exactly the subsets of ranks 0..rho.  The expected subset comes from a listing
of itertools.combinations sorted by that rank, with no oracle code involved.

Which subset the oracle visited is made observable with a lifting built for
it: points on the moment curve (t, t^2, ..., t^k) are in general position, so
every (k+1)-subset spans a simplex, and heights 0 on the subset S and positive
heights elsewhere make S a lower facet (Section 4, eq. "lower-face": the
hyperplane of height 0 has every other lifted point strictly above it).  Its
normalized volume is |det| of the difference rows, computed here in exact
rationals."""
import itertools
import math
from fractions import Fraction

import numpy as np
import pytest


def moment_points(N, k):
    return [[(t + 1) ** (q + 1) for q in range(k)] for t in range(N)]


def colex_listing(N, k):
    subsets = list(itertools.combinations(range(N), k + 1))
    subsets.sort(key=lambda c: sum(math.comb(ci, i + 1) for i, ci in enumerate(c)))
    return subsets


def exact_det(rows):
    a = [[Fraction(x) for x in r] for r in rows]
    n, det = len(a), Fraction(1)
    for t in range(n):
        p = next((i for i in range(t, n) if a[i][t] != 0), None)
        if p is None:
            return Fraction(0)
        if p != t:
            a[t], a[p] = a[p], a[t]
            det = -det
        det *= a[t][t]
        for i in range(t + 1, n):
            f = a[i][t] / a[t][t]
            for j in range(t, n):
                a[i][j] -= f * a[t][j]
    return det


def heights_for(S, N):
    return np.array([0 if i in S else 1000 + 7 * i for i in range(N)], dtype=np.int64)


def mask(S):
    return sum(1 << i for i in S)


@pytest.mark.parametrize("N,k", [(6, 1), (7, 2), (8, 3), (8, 4), (9, 2)])
def test_single_rank_slices_follow_the_colex_definition(oracle_mod, N, k):
    P = moment_points(N, k)
    listing = colex_listing(N, k)
    assert len(listing) == math.comb(N, k + 1)
    for rho, S in enumerate(listing):
        H = heights_for(S, N)
        cl = oracle_mod.cells_range(P, H, rho, rho + 1, threads=1)
        assert [int(m) for m in cl.masks] == [mask(S)], (rho, S)
        vol = abs(exact_det([[P[c][q] - P[S[0]][q] for q in range(k)] for c in S[1:]]))
        assert int(cl.den[0]) == vol
        part = oracle_mod.nvol_range(P, H, rho, rho + 1, threads=1)
        assert (part.nvol, part.cells, part.dzero, part.tie) == (vol, 1, 0, False)


@pytest.mark.parametrize("N,k", [(7, 2), (8, 3)])
def test_prefix_slices_visit_ranks_in_order(oracle_mod, N, k):
    """[0, rho+1) minus [0, rho) is exactly the subset of rank rho, for every
    rho: the successor walk from rank 0 follows the colex order."""
    P = moment_points(N, k)
    listing = colex_listing(N, k)
    for rho, S in enumerate(listing):
        H = heights_for(S, N)
        with_s = {int(m) for m in oracle_mod.cells_range(P, H, 0, rho + 1, threads=1).masks}
        without = {int(m) for m in oracle_mod.cells_range(P, H, 0, rho, threads=1).masks}
        assert with_s - without == {mask(S)}, (rho, S)
        # every subset the slice [0, rho) can list lies among ranks 0..rho-1
        assert without <= {mask(T) for T in listing[:rho]}


def test_multithreaded_chunks_cover_the_same_subsets(oracle_mod):
    """Worker chunks start by unranking and continue by successor: with many
    threads and small chunks the visited set is still ranks [lo, hi)."""
    N, k = 10, 3
    P = moment_points(N, k)
    listing = colex_listing(N, k)
    lo, hi = 17, 151
    for rho in (lo, lo + 1, 60, 99, hi - 1):
        S = listing[rho]
        H = heights_for(S, N)
        got = {int(m) for m in oracle_mod.cells_range(P, H, lo, hi, threads=8).masks}
        assert mask(S) in got
        assert got <= {mask(T) for T in listing[lo:hi]}
    # outside the slice the built facet is never visited
    S = listing[hi]
    got = {int(m) for m in oracle_mod.cells_range(P, heights_for(S, N), lo, hi, threads=8).masks}
    assert mask(S) not in got
