"""CPU-only checks of the product library: it loads, exports every symbol the
header declares, and its host prologue (rank, components, kernel points,
argument checks, tiling bounds) agrees with the oracle and with mathematics.
No device compute is called here."""
import itertools
import math

import numpy as np
import pytest
from sympy import Matrix

import gen
import oracle
from oracle import algebra
import paper_1501_02237_amd as bd


def test_library_exports_every_header_symbol():
    L = bd.lib()
    names = bd.header_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_binding_constants_equal_the_header():
    """Every numeric #define of include/bdeg.h that the binding repeats has the
    header's value (the binding parses nothing at run time)."""
    import re

    src = open(bd.HEADER).read()
    defs = {}
    for name, val in re.findall(r"^#define (BDEG_\w+) (.+?)(?:\s*/\*.*)?$", src, flags=re.M):
        val = val.strip().rstrip("u")
        val = val.replace("ull", "").replace("(", "").replace(")", "")
        try:
            defs[name] = eval(val, {})
        except Exception:
            continue
    binding = {
        "BDEG_OK": bd.BDEG_OK, "BDEG_PENDING": bd.BDEG_PENDING, "BDEG_E_ARG": bd.BDEG_E_ARG,
        "BDEG_E_OVERFLOW": bd.BDEG_E_OVERFLOW, "BDEG_E_TOO_LARGE": bd.BDEG_E_TOO_LARGE,
        "BDEG_E_TIE": bd.BDEG_E_TIE, "BDEG_E_DEVICE": bd.BDEG_E_DEVICE, "BDEG_E_NOMEM": bd.BDEG_E_NOMEM,
        "BDEG_E_STATE": bd.BDEG_E_STATE, "BDEG_F_NEEDS_CONSISTENCY": bd.BDEG_F_NEEDS_CONSISTENCY,
        "BDEG_MAX_N": bd.MAX_N, "BDEG_MAX_K": bd.MAX_K, "BDEG_MAX_ATTEMPTS": bd.MAX_ATTEMPTS,
        "BDEG_PIVOT_MAX_K": bd.PIVOT_MAX_K, "BDEG_PRUNE_MAX_PREFIXES": bd.PRUNE_MAX_PREFIXES,
        "BDEG_NOALLOC_MAX_UNITS": bd.NOALLOC_MAX_UNITS, "BDEG_SCHED_AUTO": bd.SCHED_AUTO,
        "BDEG_SCHED_POINTS": bd.SCHED_POINTS, "BDEG_F_PRUNED": bd.BDEG_F_PRUNED,
        "BDEG_PRUNE_MIN_CANDIDATES": bd.PRUNE_MIN_CANDIDATES,
    }
    for name, v in binding.items():
        assert name in defs, name
        assert defs[name] == v, (name, defs[name], v)


def test_degree_batch_raises_on_a_failing_system():
    """A system over the size limit fails before any device work: the batch
    call raises unless asked for per-system statuses (no GPU needed)."""
    too_wide = np.zeros((1, bd.MAX_N + 1), dtype=np.int64)
    with pytest.raises(bd.BdegError):
        bd.degree_batch([too_wide])


def test_strerror_covers_codes():
    for c in (0, 1, -1, -2, -3, -4, -5, -6, -7):
        assert bd.strerror(c) and "unknown" not in bd.strerror(c)


def _check_kernel(A, k, rank, comps, P):
    A = np.asarray(A)
    m, n = A.shape
    assert P.shape == (n + 1, k)
    assert (P[0] == 0).all()
    V = Matrix(P[1:].tolist())
    assert (Matrix(A.tolist()) * V).is_zero_matrix
    if k:
        assert V.rank() == k
        g = 0
        for rows in itertools.combinations(range(n), k):
            g = math.gcd(g, int(V.extract(list(rows), list(range(k))).det()))
            if g == 1:
                break
        assert g == 1


@pytest.mark.parametrize("idx", range(10))
def test_kernel_points_vs_oracle(idx):
    n = 8 + idx
    k = 1 + idx % 5
    A = gen.quiver_matrix(0x5EED0101, idx, n, n - k, 2, 3)
    kk, rank, comps, P = bd.kernel_points(A)
    ok, ocomps, _ = algebra.kernel_points(A.tolist())
    assert (kk, comps) == (ok, ocomps)
    assert rank == n - kk
    _check_kernel(A, kk, rank, comps, P)


@pytest.mark.parametrize("idx", range(8))
def test_components_dense_and_rank_deficient(idx):
    rng = gen.stream(0x5EED0102, idx, gen.PURPOSE_MATRIX)
    m, n = 2 + idx % 3, 4 + idx % 3
    A = [[rng.uniform_int(-4, 4) for _ in range(n)] for _ in range(m)]
    if idx % 2:
        A.append([2 * a - b for a, b in zip(A[0], A[1])])
    kk, rank, comps, P = bd.kernel_points(np.array(A))
    r, d, _ = algebra.smith_with_left_transform(A)
    assert rank == r and comps == algebra.components(d)
    _check_kernel(np.array(A), kk, rank, comps, P)


def test_workload_kernels_are_small():
    for s in (gen.cfg1_system(), gen.cfg2_system(), gen.cfg4_system()):
        k, rank, comps, P = bd.kernel_points(s.A)
        assert rank == s.m and comps == 1
        assert np.abs(P).max() <= 8


def test_zero_and_unimodular_systems():
    k, rank, comps, P = bd.kernel_points(np.zeros((2, 4), dtype=np.int64))
    assert (k, rank, comps) == (4, 0, 1)
    assert abs(Matrix(P[1:].tolist()).det()) == 1
    U = np.array([[1, 2, 0], [0, 1, 3], [0, 0, 1]], dtype=np.int64)
    assert bd.kernel_points(U)[:3] == (0, 3, 1)


def test_argument_errors():
    with pytest.raises(bd.BdegError) as e:
        bd.kernel_points(np.zeros((1, 64), dtype=np.int64))
    assert e.value.code == bd.BDEG_E_ARG


def test_pruned_argument_errors_before_any_device_work():
    P = np.array([[0, 0], [1, 0], [0, 1], [1, 1]], dtype=np.int32)
    H = np.array([0, 1, 2, 5], dtype=np.int64)
    for width in (3, 9):  # wider than k, wider than the widest prefix state
        with pytest.raises(bd.BdegError) as e:
            bd.nvol_points_pruned(P, H, width=width)
        assert e.value.code == bd.BDEG_E_ARG
    # C(64 - 8, 11) prefixes exceed the limit even at the widest state
    P = np.zeros((64, 18), dtype=np.int32)  # unit vectors: every minor is 0 or +-1
    P[np.arange(64), np.arange(64) % 18] = 1
    with pytest.raises(bd.BdegError) as e:
        bd.nvol_points_pruned(P, np.arange(64, dtype=np.int64))
    assert e.value.code == bd.BDEG_E_TOO_LARGE


def test_host_overflow_is_reported():
    # kernel vector of [1, -2^40]: entries around 2^40 fit int64 but not the int32 point format
    A = np.array([[1, -(1 << 40)]], dtype=np.int64)
    with pytest.raises(bd.BdegError) as e:
        bd.kernel_points(A)
    assert e.value.code == bd.BDEG_E_OVERFLOW


def test_degree_without_device_fails_loudly():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the gpu tests")
    r = bd.degree(gen.cfg1_system().A, check=False)
    assert r["status"] == bd.BDEG_E_DEVICE
    assert r["k"] == 6  # host prologue still reported


def test_degree_k0_needs_no_device():
    # k = 0 is answered on the host (a finite set of points, nvol = 1)
    r = bd.degree(np.array([[2, 1], [1, 1]], dtype=np.int64), check=False)
    assert (r["status"], r["k"], r["comps"], r["nvol"]) == (0, 0, 1, 1)


@pytest.mark.parametrize("N,k,cap", [(13, 6, 256), (29, 8, 1000), (29, 8, 5000), (37, 10, 200000), (64, 3, 1000),
                                     (20, 1, 256), (17, 12, 256), (40, 5, 777), (64, 12, 1 << 40)])
def test_work_units_cover_every_candidate_once(N, k, cap):
    """Units of the full candidate space tile [0, C(N, k+1)) exactly."""
    iv = bd.plan_units(N, k, 0, None, cap)
    total = math.comb(N, k + 1)
    order = np.argsort(iv[:, 0], kind="stable")
    s, e = iv[order, 0].astype(object), iv[order, 1].astype(object)
    assert s[0] == 0 and e[-1] == total
    assert all(e[i] == s[i + 1] for i in range(len(s) - 1))
    assert all(e[i] > s[i] for i in range(len(s)))


@pytest.mark.parametrize("seed", range(12))
def test_work_units_cover_rank_ranges(seed):
    rng = gen.stream(0x5EED0103, seed, gen.PURPOSE_MATRIX)
    N = rng.uniform_int(6, 64)
    k = rng.uniform_int(1, min(12, N - 1))
    total = math.comb(N, k + 1)
    lo = rng.next() % total
    hi = lo + 1 + rng.next() % (total - lo)
    cap = max((hi - lo) // 20000, 1) + rng.next() % 5000
    iv = bd.plan_units(N, k, lo, hi, cap)
    order = np.argsort(iv[:, 0], kind="stable")
    s, e = iv[order, 0].astype(object), iv[order, 1].astype(object)
    assert s[0] == lo and e[-1] == hi
    assert all(e[i] == s[i + 1] for i in range(len(s) - 1))


# ------------------------------------------------------------------ consistency (host only)
def _deficient(seed, m, n, r):
    rng = gen.stream(0xC0C1 + seed, m * 100 + n, gen.PURPOSE_MATRIX)
    while True:
        B = [[rng.uniform_int(-2, 2) for _ in range(n)] for _ in range(r)]
        C = [[rng.uniform_int(-2, 2) for _ in range(r)] for _ in range(m)]
        A = np.array((Matrix(C) * Matrix(B)).tolist(), dtype=np.int64)
        if Matrix(A.tolist()).rank() == r:
            return A, rng


@pytest.mark.parametrize("seed,m,n,r", [(0, 2, 1, 1), (1, 3, 2, 1), (2, 4, 3, 2), (3, 5, 4, 3), (4, 6, 4, 2),
                                        (5, 8, 6, 4), (6, 7, 7, 5), (7, 12, 9, 6)])
def test_consistency_vs_oracle(seed, m, n, r):
    """Same decision and relation count as the oracle for images b = x0^A
    (consistent) and for one b_i rotated by 0.5 rad (inconsistent when a
    relation involves it)."""
    A, rng = _deficient(seed, m, n, r)
    angles = [rng.uniform_int(0, 10**6) / 10**6 * 2 * math.pi for _ in range(n)]
    radii = [0.5 + rng.uniform_int(0, 1000) / 1000 for _ in range(n)]
    x0 = [r_ * complex(math.cos(a), math.sin(a)) for r_, a in zip(radii, angles)]
    b = [complex(np.prod([x0[j] ** int(A[i, j]) for j in range(n)])) for i in range(m)]
    lib = bd.consistency(A, b, tol=1e-8)
    ora = oracle.oracle_consistency(A, b, tol=1e-8)
    assert lib["relations"] == ora["relations"] == m - r
    assert lib["consistent"] and ora["consistent"]
    involved = [i for i in range(m) if any(q[i] for q in algebra.left_kernel_basis(A.tolist()))]
    for i in involved[:3]:
        b2 = list(b)
        b2[i] *= complex(math.cos(0.5), math.sin(0.5))
        lib2 = bd.consistency(A, b2, tol=1e-8)
        ora2 = oracle.oracle_consistency(A, b2, tol=1e-8)
        assert not lib2["consistent"] and not ora2["consistent"]
        assert lib2["residual"] > 0.1


def test_consistency_needs_the_saturated_relation():
    # x = b1, x = b2 with b1 = -b2: b1^2 = b2^2 holds, b1 = b2 does not
    assert not bd.consistency([[1], [1]], [1, -1])["consistent"]
    assert bd.consistency([[1], [1]], [1j, 1j])["consistent"]
    assert bd.consistency([[2], [4]], [1j, -1])["consistent"]


def test_consistency_full_rank_and_errors():
    assert bd.consistency([[1, 2], [3, 5]], [7, 0.25]) == dict(consistent=True, residual=0.0, relations=0)
    with pytest.raises(bd.BdegError):
        bd.consistency([[1], [1]], [0, 1])  # a zero right-hand side is outside (C*)^m
    with pytest.raises(bd.BdegError):
        bd.consistency([[1], [1]], [1, 1], tol=-1.0)


def _cert_margin(P, span):
    """log2 slack of the device width certificate (positive: inside): spatial
    Hadamard bound Hs below 2^31 and (k+1) * span * Hs below 2^60."""
    P = np.asarray(P, dtype=np.int64)
    N, k = P.shape
    rows = sorted((1 + int((r * r).sum()) for r in P), reverse=True)[: k + 1]
    h2 = min(math.prod(rows), (k + 1) ** (k + 1) * math.prod(max(1, int(abs(P[:, i]).max())) ** 2 for i in range(k)))
    return min(62 - math.log2(h2), 120 - math.log2(((k + 1) * max(span, 1)) ** 2 * h2)) / 2


@pytest.mark.parametrize("k,c,bits", [(4, 12, 36), (4, 40, 32), (6, 3, 39), (6, 2, 39), (3, 12, 39)])
def test_width_certificate_edge_on_the_host(k, c, bits):
    """The host certificate decides before any device work: a point set just
    outside it returns BDEG_E_OVERFLOW, one just inside passes the host
    checks (and, with no GPU here, stops at BDEG_E_DEVICE); heights of
    magnitude 2^40 are rejected as arguments."""
    N = 3 * k + 4
    rng = gen.stream(0xCE27, k * 100 + c, gen.PURPOSE_MATRIX)
    while True:
        P = [[0] * k] + [[rng.uniform_int(-c, c) for _ in range(k)] for _ in range(N - 1)]
        if Matrix(P).rank() == k:
            break
    P = np.array(P, dtype=np.int64)
    H = gen.random_heights(0xCE28 + k, N, bits) - (1 << (bits - 1))
    H[0] = -(1 << bits) + 1
    margin = _cert_margin(P, int(H.max() - H.min()))
    code = bd.BDEG_OK
    try:
        bd.nvol_points(P, H)
    except bd.BdegError as err:
        code = err.code
    if margin > 0:
        assert code in (bd.BDEG_OK, bd.BDEG_E_DEVICE)  # computed, or no GPU here
    else:
        assert code == bd.BDEG_E_OVERFLOW
    H2 = H.copy()
    H2[1] = 1 << 40
    with pytest.raises(bd.BdegError) as e:
        bd.nvol_points(P, H2)
    assert e.value.code == bd.BDEG_E_ARG
