"""Pins of the oracle's consistency check (Section 2, eq. ``consistency``).

x^A = b (A: m x n, one row per binomial) has solutions in (C*)^n exactly when
b^q = 1 for every q in the integer left kernel of A.  Pinned against closed
forms that need the saturated basis (x = b1, x = b2 with b1 = -b2 is
inconsistent, which a doubled relation would miss), against right-hand sides
built as b = x0^A from a chosen point x0 (consistent by construction) and
their perturbations, and against sympy for the rank, the relations q^T A = 0
and the saturation of the basis (gcd of its maximal minors is 1).
"""
import itertools
import math
from fractions import Fraction as F

import numpy as np
import pytest
from sympy import Matrix

import gen
import oracle
from oracle import algebra


def _c(x):
    """A rational or Gaussian-rational number as an exact (re, im) pair."""
    if isinstance(x, tuple):
        return (F(x[0]), F(x[1]))
    return (F(x), F(0))


def _exact(b):
    return [_c(x) for x in b]


@pytest.mark.parametrize("b,ok", [((2, 2), True), ((3, 3), True), ((1, -1), False), ((2, 3), False)])
def test_same_monomial_twice(oracle_mod, b, ok):
    r = oracle.oracle_consistency([[1], [1]], _exact(b))
    assert r["relations"] == 1 and r["consistent"] == ok


@pytest.mark.parametrize("b,ok", [((-1, 1), True), ((2, 4), True), ((2, -4), False), (((0, 1), -1), True),
                                  (((0, 1), 1), False)])
def test_square_and_fourth_power(oracle_mod, b, ok):
    # x^2 = b1, x^4 = b2: consistent iff b1^2 = b2
    assert oracle.oracle_consistency([[2], [4]], _exact(b))["consistent"] == ok


def test_sum_of_rows(oracle_mod):
    A = [[2, 1], [1, 2], [3, 3]]  # row 3 = row 1 + row 2: b1 b2 = b3
    assert oracle.oracle_consistency(A, _exact([2, 3, 6]))["consistent"]
    assert not oracle.oracle_consistency(A, _exact([2, 3, F(1, 6)]))["consistent"]
    assert oracle.oracle_consistency(A, _exact([(0, 1), 3, (0, 3)]))["consistent"]


def test_full_rank_has_no_relations(oracle_mod):
    r = oracle.oracle_consistency([[1, 2], [3, 5]], _exact([7, F(1, 3)]))
    assert r == dict(consistent=True, residual=0.0, relations=0)


def _rank_deficient(seed, m, n, r):
    rng = gen.stream(0xC0C0 + seed, m * 100 + n, gen.PURPOSE_MATRIX)
    while True:
        B = [[rng.uniform_int(-2, 2) for _ in range(n)] for _ in range(r)]
        C = [[rng.uniform_int(-2, 2) for _ in range(r)] for _ in range(m)]
        A = (Matrix(C) * Matrix(B)).tolist()
        if Matrix(A).rank() == r:
            return [[int(x) for x in row] for row in A], rng


@pytest.mark.parametrize("seed,m,n,r", [(0, 3, 3, 2), (1, 4, 3, 2), (2, 5, 4, 3), (3, 6, 5, 2), (4, 5, 6, 3)])
def test_left_kernel_basis_is_a_saturated_basis(oracle_mod, seed, m, n, r):
    A, _ = _rank_deficient(seed, m, n, r)
    Q = algebra.left_kernel_basis(A)
    assert len(Q) == m - Matrix(A).rank()
    for q in Q:
        assert all(v == 0 for v in (Matrix([q]) * Matrix(A)).tolist()[0])
    minors = [Matrix([[Q[i][j] for j in cols] for i in range(len(Q))]).det()
              for cols in itertools.combinations(range(m), len(Q))]
    assert math.gcd(*[int(x) for x in minors]) == 1


@pytest.mark.parametrize("seed,m,n,r", [(10, 3, 2, 1), (11, 4, 3, 2), (12, 5, 4, 2), (13, 6, 4, 3)])
def test_images_of_points_are_consistent(oracle_mod, seed, m, n, r):
    A, rng = _rank_deficient(seed, m, n, r)
    # x0: Gaussian rationals; b = x0^A exactly
    x0 = [(F(rng.uniform_int(1, 5), rng.uniform_int(1, 4)), F(rng.uniform_int(-3, 3), 2)) for _ in range(n)]
    b = []
    for row in A:
        v = (F(1), F(0))
        for xj, e in zip(x0, row):
            p = oracle._cpow_exact(xj, e)
            v = (v[0] * p[0] - v[1] * p[1], v[0] * p[1] + v[1] * p[0])
        b.append(v)
    assert oracle.oracle_consistency(A, b)["consistent"]
    # scaling a b_i that some relation involves breaks consistency
    Q = algebra.left_kernel_basis(A)
    i = next(i for i in range(m) if any(q[i] for q in Q))
    b2 = list(b)
    b2[i] = (2 * b[i][0], 2 * b[i][1])
    assert not oracle.oracle_consistency(A, b2)["consistent"]


def test_floating_point_path_agrees_with_exact(oracle_mod):
    A = [[2, 1], [1, 2], [3, 3], [1, -1]]
    x0 = [complex(0.6, 0.8), complex(-0.3, 1.1)]
    b = [np.prod([x0[j] ** A[i][j] for j in range(2)]) for i in range(4)]
    r = oracle.oracle_consistency(A, b)
    assert r["consistent"] and r["residual"] < 1e-12 and r["relations"] == 2
    b[3] *= complex(np.cos(0.5), np.sin(0.5))
    assert not oracle.oracle_consistency(A, b)["consistent"]
