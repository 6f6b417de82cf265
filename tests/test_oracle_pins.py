"""Pins for the oracle (CPU only): every oracle function is checked against
something other than itself -- closed forms, lattice-point counting, library
routines of other provenance (sympy's Smith form and determinants, qhull's
volume), invariances that the mathematics fixes, and the paper's values."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest
from sympy import Matrix, ZZ
from sympy.matrices.normalforms import smith_normal_form

import gen
import oracle
from oracle import algebra

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def nvol(points, seed=1, bits=20):
    return oracle.oracle_nvol_points(points, seed=seed, bits=bits)[0]


# ---------------------------------------------------------------- worked examples
def test_unit_square_example(oracle_mod):
    g = GOLDEN["unit_square"]  # Section 4, Example (two triangles under a generic lifting)
    assert nvol(g["points"]) == g["nvol"]


def test_parabola_degree_two(oracle_mod):
    g = GOLDEN["parabola"]  # Section 2: y - x^2 = 0 defines a curve of degree 2
    r = oracle.oracle_degree(g["A"])
    assert (r["k"], r["comps"], r["nvol"]) == (g["k"], g["comps"], g["nvol"])


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("k", [1, 2, 3, 4, 5])
def test_unit_cube_is_k_factorial(oracle_mod, k):
    pts = [list(v) for v in itertools.product([0, 1], repeat=k)]
    assert nvol(pts) == math.factorial(k)


@pytest.mark.parametrize("k", [1, 2, 3, 4, 5, 6])
def test_cross_polytope_is_two_to_k(oracle_mod, k):
    pts = [[0] * k]
    for i in range(k):
        for s in (1, -1):
            v = [0] * k
            v[i] = s
            pts.append(v)
    assert nvol(pts) == 2 ** k


@pytest.mark.parametrize("k,c", [(2, 3), (3, 2), (4, 3), (5, 2)])
def test_scaled_simplex(oracle_mod, k, c):
    pts = [[0] * k] + [[c * (i == j) for j in range(k)] for i in range(k)]
    assert nvol(pts) == c ** k


def _primitive_kernel_vector(A):
    """Generator of ker_Z of an (n-1) x n rank n-1 integer matrix: signed
    maximal minors (sympy determinants) divided by their gcd."""
    M = Matrix(A)
    n = M.shape[1]
    v = [(-1) ** i * M[:, [j for j in range(n) if j != i]].det() for i in range(n)]
    g = 0
    for x in v:
        g = math.gcd(g, int(x))
    return [int(x) // g for x in v]


@pytest.mark.parametrize("idx", range(12))
def test_k1_closed_form(oracle_mod, idx):
    """k = 1: nvol = max(0, v_i) - min(0, v_i) for the kernel generator v."""
    n = 3 + idx % 5
    A = gen.dense_matrix(0x5EED0001, idx, n - 1, n, -2, 2)
    v = _primitive_kernel_vector(A.tolist())
    r = oracle.oracle_degree(A)
    assert r["k"] == 1
    assert r["nvol"] == max(0, max(v)) - min(0, min(v))


def test_zero_matrix_gives_standard_simplex(oracle_mod):
    r = oracle.oracle_degree(np.zeros((1, 5), dtype=np.int64))
    assert (r["k"], r["rank"], r["comps"], r["nvol"]) == (5, 0, 1, 1)


def _unimodular(n, seed, steps=30):
    rng = gen.stream(seed, n, gen.PURPOSE_MATRIX)
    U = np.eye(n, dtype=object)
    for _ in range(steps):
        i, j = rng.bounded(n), rng.bounded(n)
        if i == j:
            continue
        q = rng.uniform_int(-2, 2)
        U[i] = U[i] + q * U[j]
        if rng.bounded(4) == 0:
            U[[i, j]] = U[[j, i]]
    return U


@pytest.mark.parametrize("n", [2, 4, 6])
def test_unimodular_square_system(oracle_mod, n):
    U = _unimodular(n, 11)
    r = oracle.oracle_degree(np.array(U, dtype=np.int64))
    assert (r["k"], r["comps"], r["nvol"]) == (0, 1, 1)


def test_diagonal_components(oracle_mod):
    A = np.zeros((3, 5), dtype=np.int64)
    A[0, 0], A[1, 1], A[2, 2] = 2, -3, 5
    r = oracle.oracle_degree(A)
    assert (r["k"], r["rank"], r["comps"]) == (2, 3, 30)
    assert r["nvol"] == 1  # ker = span(e_4, e_5): points 0 and the standard simplex


# ---------------------------------------------------------------- Smith form and kernel
def _determinantal_divisor(A, r):
    """gcd of all r x r minors: |prod d_j| for a rank-r matrix."""
    M = Matrix(A)
    g = 0
    for rows in itertools.combinations(range(M.shape[0]), r):
        for cols in itertools.combinations(range(M.shape[1]), r):
            g = math.gcd(g, int(M.extract(list(rows), list(cols)).det()))
    return g


@pytest.mark.parametrize("idx", range(10))
def test_components_match_sympy_and_minors(oracle_mod, idx):
    rng = gen.stream(0x5EED0002, idx, gen.PURPOSE_MATRIX)
    m, n = 2 + idx % 3, 3 + idx % 4
    A = [[rng.uniform_int(-3, 3) for _ in range(n)] for _ in range(m)]
    if idx % 3 == 0:  # make it rank deficient
        A.append([a + b for a, b in zip(A[0], A[1])])
    r, d, P = algebra.smith_with_left_transform(A)
    assert r == Matrix(A).rank()
    if r:
        assert algebra.components(d) == _determinantal_divisor(A, r)
        snf = smith_normal_form(Matrix(A), domain=ZZ)
        prod = 1
        for i in range(min(snf.shape)):
            if snf[i, i] != 0:
                prod *= int(snf[i, i])
        assert algebra.components(d) == abs(prod)
    # P is unimodular and P A^T Q = D has zero rows below r
    assert abs(Matrix(P).det()) == 1
    PA = Matrix(P) * Matrix(A).T
    assert all(PA[i, j] == 0 for i in range(r, PA.shape[0]) for j in range(PA.shape[1]))


@pytest.mark.parametrize("idx", range(8))
def test_kernel_basis_is_saturated(oracle_mod, idx):
    n = 8 + idx
    k = 2 + idx % 3
    A = gen.quiver_matrix(0x5EED0003, idx, n, n - k, 2, 3)
    kk, comps, pts = algebra.kernel_points(A.tolist())
    assert kk == k
    V = Matrix(pts[1:])  # n x k, row i = point of variable i
    assert (Matrix(A) * V).is_zero_matrix
    assert V.rank() == k
    g = 0
    for rows in itertools.combinations(range(n), k):
        g = math.gcd(g, int(V.extract(list(rows), list(range(k))).det()))
        if g == 1:
            break
    assert g == 1  # saturated: the gcd of maximal minors is 1


def test_lll_keeps_the_lattice(oracle_mod):
    B = [[1, 0, 0, 12345], [0, 1, 0, 6789], [0, 0, 1, 1011]]
    R = algebra.lll_reduce(B)
    # same lattice: the reduced rows are integer combinations and vice versa
    MB, MR = Matrix(B), Matrix(R)
    X = MR * MB.T * (MB * MB.T).inv()
    Y = MB * MR.T * (MR * MR.T).inv()
    assert all(x.is_integer for x in X) and all(y.is_integer for y in Y)
    assert abs(X.det()) == 1


# ---------------------------------------------------------------- lattice-point counting
def _ehrhart_nvol(points):
    """k! times the leading Ehrhart coefficient, from exact lattice-point counts
    of t*P (t = 0..k) and Lagrange interpolation; facets from qhull."""
    from scipy.spatial import ConvexHull

    P = np.array(points, dtype=float)
    k = P.shape[1]
    hull = ConvexHull(P)
    eq = hull.equations  # a.x + b <= 0 inside
    lo, hi = P.min(axis=0), P.max(axis=0)
    counts = []
    for t in range(k + 1):
        rngs = [range(int(math.floor(t * lo[i])), int(math.ceil(t * hi[i])) + 1) for i in range(k)]
        c = 0
        for x in itertools.product(*rngs):
            if np.all(eq[:, :k] @ np.array(x, dtype=float) + t * eq[:, k] <= 1e-9):
                c += 1
        counts.append(c)
    # Lagrange: leading coefficient of the degree-k interpolant through (t, counts[t])
    lead = Fraction(0)
    for t in range(k + 1):
        den = 1
        for s in range(k + 1):
            if s != t:
                den *= t - s
        lead += Fraction(counts[t], den)
    return lead * math.factorial(k)


@pytest.mark.parametrize("idx", range(10))
def test_ehrhart_matches_volume(oracle_mod, idx):
    rng = gen.stream(0x5EED0004, idx, gen.PURPOSE_MATRIX)
    k = 2 + idx % 2
    while True:
        pts = [[0] * k] + [[rng.uniform_int(-2, 2) for _ in range(k)] for _ in range(3 + k)]
        if Matrix(pts).rank() == k:
            break
    assert _ehrhart_nvol(pts) == nvol(pts)


@pytest.mark.parametrize("idx", range(10))
def test_qhull_volume_rounds_to_nvol(oracle_mod, idx):
    """The Remark of Section 4: a float volume within 1/2 rounds to nvol."""
    from scipy.spatial import ConvexHull

    rng = gen.stream(0x5EED0005, idx, gen.PURPOSE_MATRIX)
    k = 2 + idx % 5
    while True:
        pts = [[0] * k] + [[rng.uniform_int(-3, 3) for _ in range(k)] for _ in range(k + 4)]
        if Matrix(pts).rank() == k:
            break
    v = ConvexHull(np.array(pts, dtype=float)).volume * math.factorial(k)
    assert abs(v - round(v)) < 1e-6
    assert nvol(pts) == round(v)


# ---------------------------------------------------------------- invariances
@pytest.mark.parametrize("idx", range(6))
def test_unimodular_change_of_basis(oracle_mod, idx):
    rng = gen.stream(0x5EED0006, idx, gen.PURPOSE_MATRIX)
    k = 2 + idx % 4
    while True:
        pts = [[0] * k] + [[rng.uniform_int(-2, 2) for _ in range(k)] for _ in range(k + 3)]
        if Matrix(pts).rank() == k:
            break
    U = _unimodular(k, 100 + idx, steps=12)
    pts2 = [[int(x) for x in (np.array(U, dtype=object) @ np.array(p, dtype=object))] for p in pts]
    assert nvol(pts) == nvol(pts2)


@pytest.mark.parametrize("idx", range(4))
def test_row_ops_and_variable_permutation(oracle_mod, idx):
    n = 10 + idx
    A = gen.quiver_matrix(0x5EED0007, idx, n, n - 4, 2, 3)
    r0 = oracle.oracle_degree(A)
    W = np.array(_unimodular(A.shape[0], 200 + idx, steps=10), dtype=np.int64)
    perm = list(reversed(range(n)))
    r1 = oracle.oracle_degree(W @ A)
    r2 = oracle.oracle_degree(A[:, perm])
    for r in (r1, r2):
        assert (r["k"], r["comps"], r["nvol"]) == (r0["k"], r0["comps"], r0["nvol"])


@pytest.mark.parametrize("idx", range(3))
def test_lifting_independence(oracle_mod, idx):
    A = gen.quiver_matrix(0x5EED0008, idx, 14, 9, 2, 3)
    _, _, pts = algebra.kernel_points(A.tolist())
    vals = set()
    for seed, bits in [(1, 24), (2, 16), (3, 8), (4, 20), (5, 12)]:
        vals.add(oracle.oracle_nvol_points(pts, seed=seed, bits=bits)[0])
    assert len(vals) == 1


def test_ties_are_detected_and_redrawn(oracle_mod):
    # 2-bit heights on a 3x3 grid: many draws are non-generic; every accepted
    # draw must still give the exact area 8 (nvol of the 2x2 square)
    pts = [[x, y] for x in range(3) for y in range(3)]
    ties = 0
    for s in range(20):
        h = oracle.oracle_heights(s, 0, 9, 2)
        part = oracle.nvol_range(pts, h)
        if part.tie:
            ties += 1
        else:
            assert part.nvol == 8
    assert ties > 0
    v, attempts = oracle.oracle_nvol_points(pts, seed=7, bits=2, max_attempts=64)
    assert v == 8


def test_pyramid_rule(oracle_mod):
    """nvol_k(conv{0, (q_i, 1)}) = nvol_{k-1}(conv{q_i})."""
    rng = gen.stream(0x5EED0009, 0, gen.PURPOSE_MATRIX)
    for k in (3, 4):
        while True:
            q = [[rng.uniform_int(-2, 2) for _ in range(k - 1)] for _ in range(k + 2)]
            if Matrix([x + [1] for x in q]).rank() == k:
                break
        base = nvol(q)
        apex = nvol([[0] * k] + [x + [1] for x in q])
        assert base == apex


def test_cells_bounded_by_nvol(oracle_mod):
    s = gen.cfg1_system()
    _, _, pts = algebra.kernel_points(s.A.tolist())
    part = oracle.nvol_range(pts, oracle.oracle_heights(9, 0, len(pts), 16))
    assert not part.tie
    assert 0 < part.cells <= part.nvol


def test_rank_ranges_partition_the_sum(oracle_mod):
    s = gen.cfg1_system()
    _, _, pts = algebra.kernel_points(s.A.tolist())
    h = oracle.oracle_heights(3, 0, len(pts), 16)
    total = oracle.binom(len(pts), len(pts[0]) + 1)
    whole = oracle.nvol_range(pts, h)
    cuts = [0, 1, 17, 400, 401, 1000, total]
    parts = [oracle.nvol_range(pts, h, a, b) for a, b in zip(cuts, cuts[1:])]
    assert sum(p.nvol for p in parts) == whole.nvol
    assert sum(p.cells for p in parts) == whole.cells


def test_dropping_the_origin_breaks_the_paper_value(oracle_mod):
    """Reading check: the point set must include 0 (eq. deg-vol).  Without it
    the homogeneous master-space points are affinely degenerate."""
    A = gen.master_space_matrix(2, 2)
    k, _, pts = algebra.kernel_points(A.tolist())
    assert Matrix(pts[1:]).rank() == k
    with_origin = nvol(pts)
    assert with_origin == GOLDEN["table4_degrees"]["2,2"]
    # without 0, conv{v_i} lies in an affine hyperplane: no full-dimensional cell
    part = oracle.nvol_range(pts[1:], oracle.oracle_heights(1, 0, len(pts) - 1, 20))
    assert part.nvol == 0


# ---------------------------------------------------------------- paper values
@pytest.mark.parametrize("mk", ["1,2", "1,3", "1,4", "1,5", "1,6", "2,1", "2,2", "2,3", "3,2", "3,1", "1,7"])
def test_master_space_degrees(oracle_mod, mk):
    m, k = map(int, mk.split(","))
    r = oracle.oracle_degree(gen.master_space_matrix(m, k))
    assert r["comps"] == 1
    assert r["nvol"] == GOLDEN["table4_degrees"][mk]
    assert r["k"] == GOLDEN["table2_dims"][str(m)][k - 1]


def test_master_space_degree_2_4(oracle_mod):
    r = oracle.oracle_degree(gen.master_space_matrix(2, 4))
    assert r["nvol"] == GOLDEN["table4_degrees"]["2,4"] == 6 * 92 + 2 ** 5  # conjectured recurrence


@pytest.mark.parametrize("m,k", [(m, k) for m in range(1, 5) for k in range(1, 5) if (m, k) != (1, 1)])
def test_master_space_dimensions(oracle_mod, m, k):
    r, _, _ = algebra.smith_with_left_transform(gen.master_space_matrix(m, k).tolist())
    assert 3 * m * k - r == GOLDEN["table2_dims"][str(m)][k - 1] == m * k + 2
