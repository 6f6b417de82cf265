"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only *draws inputs*: integer exponent matrices A (m x n, one row
per binomial x^(alpha-beta) = b, one column per variable), explicit lifting
heights for tests, and request arrival times for the serving trace.  It holds
none of the degree method's arithmetic (no Smith form, no kernel basis, no
volume).  The only linear algebra here is a rank filter modulo a prime, used
to redraw matrices until they have full row rank as the workload recipes ask.

Random numbers come from SplitMix64 (G. L. Steele, D. Lea, C. H. Flood,
"Fast splittable pseudorandom number generators", OOPSLA 2014), used as a
counter-based generator, and bounded integers from Lemire's multiply-shift
method with rejection (D. Lemire, "Fast random integer generation in an
interval", ACM TOMACS 2019).

The master-space system of the paper's Section 6 (eq. ``superpotential``) is
also built here: it is a formula-defined input, not part of the method.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# bump whenever a recipe below changes: stored expected values record it
GEN_VERSION = 1

MASK64 = (1 << 64) - 1
GOLDEN_GAMMA = 0x9E3779B97F4A7C15

# stream purposes (xor-ed into the stream key)
PURPOSE_MATRIX = 0x4D41545249580000  # "MATRIX"
PURPOSE_HEIGHTS = 0x4845494748540000  # "HEIGHT"
PURPOSE_ARRIVAL = 0x4152524956000000  # "ARRIV"
PURPOSE_SIZES = 0x53495A4553000000  # "SIZES"
PURPOSE_PHASE = 0x5048415345000000  # "PHASE"

# per-workload seeds
SEED_CFG = {1: 0xB0E60001, 2: 0xB0E60002, 3: 0xB0E60003, 4: 0xB0E60004, 5: 0xB0E60005}


def splitmix64_mix(z: int) -> int:
    """The SplitMix64 output function (finaliser) on a 64-bit word."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64: state advances by the golden gamma each draw."""

    __slots__ = ("state",)

    def __init__(self, state: int):
        self.state = state & MASK64

    def next(self) -> int:
        self.state = (self.state + GOLDEN_GAMMA) & MASK64
        return splitmix64_mix(self.state)

    def bounded(self, s: int) -> int:
        """Uniform integer in [0, s) for 0 < s < 2^32 (Lemire 2019)."""
        assert 0 < s < (1 << 32)
        x = self.next() >> 32
        m = x * s
        low = m & 0xFFFFFFFF
        if low < s:
            t = ((1 << 32) - s) % s
            while low < t:
                x = self.next() >> 32
                m = x * s
                low = m & 0xFFFFFFFF
        return m >> 32

    def uniform_int(self, lo: int, hi: int) -> int:
        """Uniform integer in the closed range [lo, hi]."""
        return lo + self.bounded(hi - lo + 1)

    def unit(self) -> float:
        """Uniform double in [0, 1) from the top 53 bits (harness use only)."""
        return (self.next() >> 11) * (1.0 / (1 << 53))


def stream(seed_cfg: int, index: int, purpose: int) -> SplitMix64:
    key = splitmix64_mix((seed_cfg ^ ((index * GOLDEN_GAMMA) & MASK64) ^ purpose) & MASK64)
    return SplitMix64(key)


# --------------------------------------------------------------------------
# rank filter (generator-side only)
# --------------------------------------------------------------------------
_P31 = 2147483647  # 2^31 - 1, prime


def rank_mod_p(A: np.ndarray) -> int:
    """Rank of A over GF(2^31-1).  rank_p(A) <= rank_Q(A), so a matrix with
    rank_p == m has full row rank m over Q; a matrix that fails is redrawn."""
    M = np.array(A, dtype=np.int64) % _P31
    rows, cols = M.shape
    r = 0
    for c in range(cols):
        if r == rows:
            break
        nz = np.nonzero(M[r:, c])[0]
        if nz.size == 0:
            continue
        piv = r + int(nz[0])
        if piv != r:
            M[[r, piv]] = M[[piv, r]]
        inv = pow(int(M[r, c]), _P31 - 2, _P31)
        M[r] = (M[r] * inv) % _P31
        f = M[:, c].copy()
        f[r] = 0
        nzr = np.nonzero(f)[0]
        if nzr.size:
            M[nzr] = (M[nzr] - (f[nzr, None] * M[r][None, :]) % _P31) % _P31
        r += 1
    return r


# --------------------------------------------------------------------------
# matrix recipes
# --------------------------------------------------------------------------
def _sample_subset(rng: SplitMix64, pool: list[int], w: int) -> list[int]:
    """Uniform w-subset of pool by a partial Fisher-Yates shuffle."""
    pool = list(pool)
    for i in range(w):
        j = i + rng.bounded(len(pool) - i)
        pool[i], pool[j] = pool[j], pool[i]
    return pool[:w]


def quiver_row(rng: SplitMix64, n: int, wlo: int, whi: int) -> list[int]:
    """a = p - q with p, q disjoint 0/1 vectors of weights drawn in [wlo, whi]."""
    wp = rng.uniform_int(wlo, whi)
    wq = rng.uniform_int(wlo, whi)
    sp = _sample_subset(rng, list(range(n)), wp)
    rest = [i for i in range(n) if i not in set(sp)]
    sq = _sample_subset(rng, rest, wq)
    row = [0] * n
    for i in sp:
        row[i] += 1
    for i in sq:
        row[i] -= 1
    return row


def quiver_matrix(seed_cfg: int, index: int, n: int, m: int, wlo: int, whi: int) -> np.ndarray:
    """m x n quiver-like exponent matrix, the whole matrix redrawn until rank m."""
    rng = stream(seed_cfg, index, PURPOSE_MATRIX)
    while True:
        A = np.array([quiver_row(rng, n, wlo, whi) for _ in range(m)], dtype=np.int64)
        if rank_mod_p(A) == m:
            return A


def dense_matrix(seed_cfg: int, index: int, m: int, n: int, lo: int, hi: int) -> np.ndarray:
    """m x n matrix with entries uniform in [lo, hi], redrawn until rank m."""
    rng = stream(seed_cfg, index, PURPOSE_MATRIX)
    while True:
        A = np.array([[rng.uniform_int(lo, hi) for _ in range(n)] for _ in range(m)], dtype=np.int64)
        if rank_mod_p(A) == m:
            return A


@dataclass
class System:
    """One binomial system of a workload: exponent matrix and lifting width."""

    A: np.ndarray  # m x n int64
    lift_bits: int
    index: int = 0

    @property
    def m(self) -> int:
        return int(self.A.shape[0])

    @property
    def n(self) -> int:
        return int(self.A.shape[1])


def cfg1_system() -> System:
    """Plain single system: A 6x12, entries uniform in {-2..2}, rank 6 (k=6, N=13), B=16."""
    return System(dense_matrix(SEED_CFG[1], 0, 6, 12, -2, 2), 16, 0)


def cfg1_b_phases() -> list[float]:
    """The random nonzero complex b of the plain 6x12 workload, as unit-circle
    phases in [0, 1).  The degree does not depend on b; kept for completeness."""
    rng = stream(SEED_CFG[1], 0, PURPOSE_PHASE)
    return [rng.unit() for _ in range(6)]


def cfg2_system() -> System:
    """Quiver-like single system: n=28, 20 rows of weight 2-3, k=8, N=29, B=20."""
    return System(quiver_matrix(SEED_CFG[2], 0, 28, 20, 2, 3), 20, 0)


def cfg3_systems(count: int = 4096) -> list[System]:
    """Batch of quiver-like systems, n ~ U[10,24], k ~ U[3,7], weights 2-3, B=20."""
    out = []
    for i in range(count):
        rng = stream(SEED_CFG[3], i, PURPOSE_SIZES)
        n = rng.uniform_int(10, 24)
        k = rng.uniform_int(3, 7)
        out.append(System(quiver_matrix(SEED_CFG[3], i, n, n - k, 2, 3), 20, i))
    return out


def cfg4_system() -> System:
    """Large single system: n=36, 26 rows of weight 2-4, k=10, N=37, B=24."""
    return System(quiver_matrix(SEED_CFG[4], 0, 36, 26, 2, 4), 24, 0)


@dataclass
class Request:
    arrival_s: float
    system: System


def cfg5_trace(count: int = 4000, rate_hz: float = 200.0) -> list[Request]:
    """Serving trace: Poisson arrivals (exponential gaps, mean 1/rate) of
    quiver-like systems with n ~ U[12,32], k ~ U[4,9], weights 2-3, B=20."""
    arr = stream(SEED_CFG[5], 0, PURPOSE_ARRIVAL)
    t = 0.0
    out = []
    for i in range(count):
        u = arr.unit()
        t += -math.log1p(-u) / rate_hz
        rng = stream(SEED_CFG[5], i, PURPOSE_SIZES)
        n = rng.uniform_int(12, 32)
        k = rng.uniform_int(4, 9)
        out.append(Request(t, System(quiver_matrix(SEED_CFG[5], i, n, n - k, 2, 3), 20, i)))
    return out


def random_heights(seed: int, N: int, bits: int) -> np.ndarray:
    """Explicit lifting heights, uniform in [0, 2^bits), for tests that hand the
    same heights to both the oracle and the device path."""
    rng = stream(seed, N, PURPOSE_HEIGHTS)
    return np.array([rng.next() >> (64 - bits) for _ in range(N)], dtype=np.int64)


# --------------------------------------------------------------------------
# master space system (paper Section 6, eq. superpotential)
# --------------------------------------------------------------------------
def master_space_matrix(m: int, k: int) -> np.ndarray:
    """Exponent matrix of the binomial system dW_{m,k} = 0.

    W_{m,k} = sum_{i<m, j<k} x_{i,j} y_{i+1,j} z_{i+1,j+1} - y_{i,j} x_{i,j+1} z_{i+1,j+1}
    with the first index periodic mod m and the second mod k.  Every variable
    lies in exactly two monomials, so each partial derivative is a binomial
    c1 x^alpha + c2 x^beta; its row of A is alpha - beta.  Variables are
    ordered x_{i,j}, y_{i,j}, z_{i,j} with flat index 3*(i*k + j) + {0,1,2}.
    """
    nv = 3 * m * k

    def var(kind: int, i: int, j: int) -> int:
        return 3 * ((i % m) * k + (j % k)) + kind

    terms = []  # list of (coef, [variables])
    for i in range(m):
        for j in range(k):
            terms.append((+1, [var(0, i, j), var(1, i + 1, j), var(2, i + 1, j + 1)]))
            terms.append((-1, [var(1, i, j), var(0, i, j + 1), var(2, i + 1, j + 1)]))
    rows = []
    for v in range(nv):
        occ = []
        for coef, vs in terms:
            if v in vs:
                e = [0] * nv
                for u in vs:
                    e[u] += 1
                e[v] -= 1
                occ.append(e)
        if len(occ) != 2:
            raise ValueError(f"variable {v} of W_{m},{k} lies in {len(occ)} monomials")
        rows.append([a - b for a, b in zip(occ[0], occ[1])])
    return np.array(rows, dtype=np.int64)
