"""Oracle: exact integer algebra for the degree of a binomial system.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this file;
only tests, the smoke check and the benchmark's CPU-baseline leg use it.

Everything here is exact (Python integers, Fractions), plain and slow.

Notation follows the paper (Section 2): the paper's exponent matrix has one
*column* per binomial, A_paper in Z^{n x m}.  Callers hand in A with one *row*
per binomial (m x n); ``smith_with_left_transform`` works on A_paper = A^T.

* ``smith_with_left_transform``: Smith-type diagonalisation P A_paper Q = D by
  repeated unimodular 2x2 row and column reductions built from Bezout's
  identity (Section 3, the 2x2 matrices P and Q), with row/column swaps.
  Divisibility d_1 | d_2 | ... is not enforced; Section 3 notes it is not
  needed for binomial systems.  Returns r = rank, the d_j and P.
* ``components``: |prod d_j| (Proposition ``topological``).
* ``kernel_points``: the paper's point set: the columns of P_0, the bottom
  n - r rows of P (Section 4, the matrix P^0 in eq. ``deg-vol2``), after an LLL
  reduction of the rows of P_0.  The reduction is a unimodular change of basis
  of the kernel lattice (P_0 -> U P_0 with det U = +-1), which maps the point
  set by a unimodular linear map and so leaves the normalized volume unchanged;
  it only keeps coordinates small enough for the exact volume code.
"""
from __future__ import annotations

from fractions import Fraction


def _egcd(a: int, b: int) -> tuple[int, int, int]:
    """(g, s, t) with g = s*a + t*b = gcd(a, b) >= 0."""
    s0, s1, t0, t1 = 1, 0, 0, 1
    x, y = a, b
    while y != 0:
        q = x // y
        x, y = y, x - q * y
        s0, s1 = s1, s0 - q * s1
        t0, t1 = t1, t0 - q * t1
    if x < 0:
        x, s0, t0 = -x, -s0, -t0
    return x, s0, t0


def _bezout(a1: int, a2: int) -> tuple[int, int, int]:
    """Bezout data (d, s, t) with d = s*a1 + t*a2 dividing both a1 and a2.

    When a1 divides a2 the choice s = 1, t = 0, d = a1 is taken (the 2x2
    reduction is then an ordinary elimination step); otherwise d = gcd."""
    if a2 % a1 == 0:
        return a1, 1, 0
    return _egcd(a1, a2)


def smith_with_left_transform(A_rows: list[list[int]]) -> tuple[int, list[int], list[list[int]]]:
    """P A_paper Q = diag(d_1..d_r, 0..) for A_paper = transpose(A_rows).

    Returns (r, [d_1..d_r], P) with P unimodular n x n (n = number of
    variables = columns of A_rows)."""
    m = len(A_rows)
    n = len(A_rows[0]) if m else 0
    M = [[int(A_rows[j][i]) for j in range(m)] for i in range(n)]  # n x m
    P = [[int(i == j) for j in range(n)] for i in range(n)]

    def row_reduce(t: int, i: int) -> None:
        # rows (t, i) <- [[s, tt], [-a2/d, a1/d]] (rows t, i): kills M[i][t]
        a1, a2 = M[t][t], M[i][t]
        d, s, tt = _bezout(a1, a2)
        u, v = -a2 // d, a1 // d
        for X in (M, P):
            rt, ri = X[t], X[i]
            X[t] = [s * x + tt * y for x, y in zip(rt, ri)]
            X[i] = [u * x + v * y for x, y in zip(rt, ri)]

    def col_reduce(t: int, j: int) -> None:
        # cols (t, j) <- cols (t, j) [[s, -a2/d], [tt, a1/d]]: kills M[t][j]
        a1, a2 = M[t][t], M[t][j]
        d, s, tt = _bezout(a1, a2)
        u, v = -a2 // d, a1 // d
        for row in M:
            x, y = row[t], row[j]
            row[t] = s * x + tt * y
            row[j] = u * x + v * y

    r = 0
    for t in range(min(n, m)):
        # pivot: a nonzero entry of smallest magnitude in the trailing block
        best = None
        for i in range(t, n):
            for j in range(t, m):
                if M[i][j] != 0 and (best is None or abs(M[i][j]) < best[0]):
                    best = (abs(M[i][j]), i, j)
        if best is None:
            break
        _, pi, pj = best
        if pi != t:
            M[t], M[pi] = M[pi], M[t]
            P[t], P[pi] = P[pi], P[t]
        if pj != t:
            for row in M:
                row[t], row[pj] = row[pj], row[t]
        while True:
            for i in range(t + 1, n):
                if M[i][t] != 0:
                    row_reduce(t, i)
            for j in range(t + 1, m):
                if M[t][j] != 0:
                    col_reduce(t, j)
            if all(M[i][t] == 0 for i in range(t + 1, n)):
                break
        r = t + 1
    d = [M[j][j] for j in range(r)]
    return r, d, P


def components(d: list[int]) -> int:
    """Number of components |prod d_j| (Proposition ``topological``)."""
    prod = 1
    for x in d:
        prod *= x
    return abs(prod)


def lll_reduce(B: list[list[int]], delta: Fraction = Fraction(3, 4)) -> list[list[int]]:
    """LLL reduction of the rows of B (A. K. Lenstra, H. W. Lenstra, L. Lovasz,
    Math. Ann. 261, 1982) in exact rational arithmetic: size-reduce against the
    Gram-Schmidt vectors, swap on the Lovasz condition, recompute.  Plain and
    slow on purpose; returns a basis of the same lattice."""
    B = [list(map(int, b)) for b in B]
    k = len(B)
    if k <= 1:
        return B

    def dot(u, v):
        return sum(a * b for a, b in zip(u, v))

    def gram_schmidt():
        Bs, Bn = [], []
        mu = [[Fraction(0)] * k for _ in range(k)]
        for i in range(k):
            v = [Fraction(x) for x in B[i]]
            for j in range(i):
                mu[i][j] = Fraction(dot(B[i], Bs[j])) / Bn[j] if Bn[j] else Fraction(0)
                v = [a - mu[i][j] * b for a, b in zip(v, Bs[j])]
            Bs.append(v)
            Bn.append(dot(v, v))
        return Bs, Bn, mu

    Bs, Bn, mu = gram_schmidt()
    i = 1
    while i < k:
        for j in range(i - 1, -1, -1):
            q = round(mu[i][j])
            if q:
                B[i] = [a - q * b for a, b in zip(B[i], B[j])]
                Bs, Bn, mu = gram_schmidt()
        if Bn[i] >= (delta - mu[i][i - 1] ** 2) * Bn[i - 1]:
            i += 1
        else:
            B[i], B[i - 1] = B[i - 1], B[i]
            Bs, Bn, mu = gram_schmidt()
            i = max(i - 1, 1)
    return B


def kernel_points(A_rows, reduce: bool = True) -> tuple[int, int, list[list[int]]]:
    """(k, comps, points): k = n - rank, comps = |prod d_j|, and the point set
    {0} + {columns of P_0} in Z^k as a list of N = n + 1 integer k-vectors,
    the origin first (Proposition ``degree``, eq. ``deg-vol``)."""
    rows = [[int(x) for x in r] for r in A_rows]
    n = len(rows[0])
    r, d, P = smith_with_left_transform(rows)
    k = n - r
    P0 = [P[i][:] for i in range(r, n)]  # k x n
    if reduce and k > 1:
        P0 = lll_reduce(P0)
    pts = [[0] * k] + [[P0[i][j] for i in range(k)] for j in range(n)]
    return k, components(d), pts


def left_kernel_basis(A_rows) -> list[list[int]]:
    """A basis of the integer left kernel {q in Z^m : q^T A = 0} of the m x n
    exponent matrix A (one row per binomial): the rows r..m-1 of the
    unimodular left transform of the Smith form of A, i.e. the columns of Q_0
    in the paper's orientation (Section 2, eq. ``rank-decomp``), LLL-reduced.
    Being rows of a unimodular matrix they span the whole lattice (a
    saturated basis)."""
    rows = [[int(x) for x in r] for r in A_rows]
    m, n = len(rows), len(rows[0])
    transposed = [[rows[i][j] for i in range(m)] for j in range(n)]  # n x m
    r, _d, Pm = smith_with_left_transform(transposed)  # Pm: m x m with Pm A Q = D
    Q0 = [Pm[i][:] for i in range(r, m)]
    # The condition concerns the lattice, not the basis: LLL (a unimodular
    # change of basis) keeps it saturated and keeps the exponents of b^q small
    # (the raw transform rows reach millions on 12 x 9 systems).
    return lll_reduce(Q0) if len(Q0) > 1 else Q0
