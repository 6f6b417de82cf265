"""Oracle for the degree of a binomial system's C*-solution set.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the product library (``paper_1501_02237_amd``) and never imports
it; the two meet only in the seeded input generators of ``gen``.

What it computes, plainly and exactly (paper Sections 2 and 4):

* ``oracle_degree(A)`` -> {k, rank, comps, nvol, attempts}
    - rank r and comps = |prod d_j| from a Smith diagonalisation by Bezout 2x2
      reductions (``algebra``; Proposition ``topological``);
    - k = n - r; the point set {0} + columns of P_0 (Proposition ``degree``);
    - nvol = k! Vol_k(conv of the points), by summing |det| over the lower
      facets of a generic integer lifting, visiting every (k+1)-subset
      (``volume.c``; eqs. ``lower-face``, ``simplex-vol``); a lifting that
      produces a non-generic lower face is redrawn (at most 16 draws);
    - k = 0: nvol = 1 (a finite set of points, each of degree 1).
* ``oracle_nvol_points(points, heights)`` -> the same volume sum for a caller's
  point set and explicit heights, optionally over a colex rank range.
* ``oracle_consistency(A, b)`` -> whether x^A = b has solutions when
  rank A < m: b^q = 1 for every q of a saturated basis of the left kernel
  (Section 2, eq. ``consistency``); exact for rational or Gaussian-rational b
  (``fractions.Fraction`` pairs), complex double otherwise.
* ``cells_range(points, heights)`` -> the lower facets themselves (the cells of
  the regular subdivision) with their inner normals (alpha, 1), alpha exact
  rationals num / den (eq. ``lower-d-face-again``; the start data of the
  polyhedral homotopy of Section 5).

Parity unpinned: nothing.  Every function is pinned by the tests in
``tests/test_oracle_*.py`` against closed forms, brute-force lattice-point
counts, library routines of other provenance and the paper's printed values.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from fractions import Fraction

import numpy as np

from gen import MASK64, PURPOSE_HEIGHTS, stream
from . import algebra

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "volume.c")
_LIB = os.path.join(_HERE, "liboracle_volume.so")

# tag mixed into the oracle's own lifting stream (distinct from the library's)
ORACLE_TAG = 0x0AC1E0AC1E0AC1E0
MAX_ATTEMPTS = 16

ORACLE_OK = 0
ORACLE_E_ARG = -1
ORACLE_E_OVERFLOW = -2


class OracleError(RuntimeError):
    pass


def build(force: bool = True) -> str:
    """Compile volume.c into liboracle_volume.so (plain gcc, no GPU)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared", "-pthread", _SRC, "-o", tmp],
            check=True,
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_nvol_range.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_int, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
        ]
        lib.oracle_nvol_range.restype = ctypes.c_int
        lib.oracle_cells_range.argtypes = [
            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint64,
            ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_int),
        ]
        lib.oracle_cells_range.restype = ctypes.c_int
        lib.oracle_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        lib.oracle_binom.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def binom(n: int, r: int) -> int:
    return int(_load().oracle_binom(n, r))


@dataclass
class VolumePart:
    nvol: int
    tie: bool
    cells: int
    dzero: int


def nvol_range(points, heights, rank_lo: int = 0, rank_hi: int | None = None, threads: int | None = None) -> VolumePart:
    """Sum of |D| over lower facets among candidates with colex rank in
    [rank_lo, rank_hi), for explicit heights (one per point)."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    if H.shape != (N,):
        raise OracleError("one height per point")
    lo, hi, tie = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int()
    cells, dz = ctypes.c_uint64(), ctypes.c_uint64()
    rh = MASK64 if rank_hi is None else int(rank_hi)
    rc = _load().oracle_nvol_range(
        P.ctypes.data, H.ctypes.data, N, k, int(rank_lo), rh, threads or default_threads(),
        ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(tie), ctypes.byref(cells), ctypes.byref(dz),
    )
    if rc == ORACLE_E_OVERFLOW:
        raise OracleError("int128 overflow in the oracle volume")
    if rc != ORACLE_OK:
        raise OracleError(f"oracle_nvol_range: bad arguments (N={N}, k={k})")
    v = (hi.value << 64) | lo.value
    if v >= 1 << 127:
        v -= 1 << 128
    return VolumePart(v, bool(tie.value), cells.value, dz.value)


@dataclass
class Cells:
    masks: np.ndarray  # uint64 [c]: bit i set for vertex i
    num: np.ndarray    # int64 [c, k]: inner normal numerators
    den: np.ndarray    # uint64 [c]: denominators = normalized volumes |D|
    tie: bool

    def as_set(self) -> set:
        return {(int(m), tuple(int(x) for x in n), int(d)) for m, n, d in zip(self.masks, self.num, self.den)}


def cells_range(points, heights, rank_lo: int = 0, rank_hi: int | None = None,
                threads: int | None = None, cap: int = 1024) -> Cells:
    """The lower facets (cells of the regular subdivision) among candidates
    with colex rank in [rank_lo, rank_hi), each with its inner normal
    (alpha, 1), alpha = num / den (eq. ``lower-d-face-again``)."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int64))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    if H.shape != (N,):
        raise OracleError("one height per point")
    rh = MASK64 if rank_hi is None else int(rank_hi)
    while True:
        masks = np.zeros(cap, dtype=np.uint64)
        num = np.zeros((cap, k), dtype=np.int64)
        den = np.zeros(cap, dtype=np.uint64)
        cnt, tie = ctypes.c_uint64(), ctypes.c_int()
        rc = _load().oracle_cells_range(
            P.ctypes.data, H.ctypes.data, N, k, int(rank_lo), rh, threads or default_threads(), cap,
            masks.ctypes.data, num.ctypes.data, den.ctypes.data, ctypes.byref(cnt), ctypes.byref(tie),
        )
        if rc == ORACLE_E_OVERFLOW:
            raise OracleError("overflow in the oracle cell list")
        if rc != ORACLE_OK:
            raise OracleError(f"oracle_cells_range: bad arguments (N={N}, k={k})")
        if cnt.value <= cap:
            c = cnt.value
            return Cells(masks[:c].copy(), num[:c].copy(), den[:c].copy(), bool(tie.value))
        cap = int(cnt.value)


def oracle_heights(seed: int, attempt: int, N: int, bits: int) -> np.ndarray:
    """The oracle's own lifting: heights uniform in [0, 2^bits) from a
    SplitMix64 stream keyed by (seed, attempt), tagged apart from the library's."""
    rng = stream(seed ^ ORACLE_TAG, attempt, PURPOSE_HEIGHTS)
    return np.array([rng.next() >> (64 - bits) for _ in range(N)], dtype=np.int64)


def oracle_nvol_points(points, seed: int = 1, bits: int = 20, threads: int | None = None,
                       max_attempts: int = MAX_ATTEMPTS) -> tuple[int, int]:
    """(nvol, attempts) of conv(points) for a point set that spans Z^k affinely;
    the lifting is redrawn while it is not generic."""
    P = np.asarray(points, dtype=np.int64)
    N, k = P.shape
    if k == 0:
        return 1, 0
    for attempt in range(max_attempts):
        part = nvol_range(P, oracle_heights(seed, attempt, N, bits), threads=threads)
        if not part.tie:
            return part.nvol, attempt + 1
    raise OracleError(f"no generic lifting in {max_attempts} draws")


def oracle_degree(A, seed: int = 1, bits: int = 20, threads: int | None = None) -> dict:
    """{k, rank, comps, nvol, attempts, points} for the binomial system with
    exponent matrix A (m x n, one row per binomial)."""
    A = np.asarray(A, dtype=np.int64)
    m, n = A.shape
    k, comps, pts = algebra.kernel_points(A.tolist())
    rank = n - k
    if k == 0:
        return dict(k=0, rank=rank, comps=comps, nvol=1, attempts=0, points=pts)
    nvol, attempts = oracle_nvol_points(pts, seed=seed, bits=bits, threads=threads)
    return dict(k=k, rank=rank, comps=comps, nvol=nvol, attempts=attempts, points=pts)


def _cpow_exact(base, e: int):
    """(re, im) Fraction pair raised to the integer power e (exact)."""
    re, im = base
    if e < 0:
        n2 = re * re + im * im
        re, im, e = re / n2, -im / n2, -e
    acc = (Fraction(1), Fraction(0))
    for _ in range(e):
        acc = (acc[0] * re - acc[1] * im, acc[0] * im + acc[1] * re)
    return acc


def oracle_consistency(A, b, tol: float = 1e-9) -> dict:
    """{consistent, residual, relations} of x^A = b (Section 2, eq.
    ``consistency``): b^q for each q of a saturated left-kernel basis.

    b: m entries, each a Python complex (evaluated in complex double) or a
    pair (re, im) of Fractions (evaluated exactly; then residual is 0.0 or
    the double value of the largest |b^q - 1|)."""
    rows = [[int(x) for x in r] for r in np.asarray(A, dtype=np.int64).tolist()]
    basis = algebra.left_kernel_basis(rows)
    exact = all(isinstance(x, tuple) for x in b)
    worst = 0.0
    for q in basis:
        if exact:
            prod = (Fraction(1), Fraction(0))
            for bi, qi in zip(b, q):
                if qi:
                    p = _cpow_exact((Fraction(bi[0]), Fraction(bi[1])), qi)
                    prod = (prod[0] * p[0] - prod[1] * p[1], prod[0] * p[1] + prod[1] * p[0])
            dev = abs(complex(float(prod[0] - 1), float(prod[1])))
        else:
            prod = complex(1.0)
            for bi, qi in zip(b, q):
                if qi:
                    prod *= complex(bi) ** qi
            dev = abs(prod - 1.0)
        worst = max(worst, dev)
    return dict(consistent=worst <= tol, residual=worst, relations=len(basis))
