"""Python binding of libbdeg (include/bdeg.h): argument marshalling only.

Every step of the degree path runs inside the C-ABI library (host algebra in
C++, enumeration in HIP kernels on the GPU).  There is no Python or CPU
fallback: if the library is missing, importing the functions raises.
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbdeg.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "bdeg.h")

BDEG_OK = 0
BDEG_PENDING = 1
BDEG_E_ARG = -1
BDEG_E_OVERFLOW = -2
BDEG_E_TOO_LARGE = -3
BDEG_E_TIE = -4
BDEG_E_DEVICE = -5
BDEG_E_NOMEM = -6
BDEG_E_STATE = -7
BDEG_F_NEEDS_CONSISTENCY = 1
BDEG_F_PRUNED = 2
PRUNE_MIN_CANDIDATES = 1 << 27
MAX_N = 63
MAX_K = 18
MAX_ATTEMPTS = 16
PIVOT_MAX_K = 24
PRUNE_MAX_PREFIXES = 1 << 24
NOALLOC_MAX_UNITS = 1 << 17
SCHED_AUTO = 0
SCHED_POINTS = 1
NOALLOC_SCRATCH_BYTES = NOALLOC_MAX_UNITS * 16 + 32768
U64_MAX = (1 << 64) - 1


class BdegError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


class U128(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64)]

    @property
    def value(self) -> int:
        return (self.hi << 64) | self.lo


class Result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32), ("k", ctypes.c_int32), ("rank", ctypes.c_int32), ("attempts", ctypes.c_int32),
        ("flags", ctypes.c_uint32), ("reserved", ctypes.c_uint32), ("components", U128), ("nvol", U128),
        ("candidates", ctypes.c_uint64), ("cells", ctypes.c_uint64),
    ]

    def as_dict(self) -> dict:
        return dict(status=self.status, k=self.k, rank=self.rank, attempts=self.attempts, flags=self.flags,
                    comps=self.components.value, nvol=self.nvol.value, candidates=self.candidates, cells=self.cells)


class Stats(ctypes.Structure):
    _fields_ = [
        ("ridges", ctypes.c_uint64), ("inner_nodes", ctypes.c_uint64), ("spatial_updates", ctypes.c_uint64),
        ("pruned", ctypes.c_uint64), ("leaves", ctypes.c_uint64), ("tiles", ctypes.c_uint64),
        ("ridge_steps", ctypes.c_uint64), ("leaf_steps", ctypes.c_uint64), ("empty_steps", ctypes.c_uint64),
        ("point_inner", ctypes.c_uint64), ("point_spatial", ctypes.c_uint64), ("point_ridges", ctypes.c_uint64),
        ("leaf_points", ctypes.c_uint64), ("triples", ctypes.c_uint64), ("dense_units", ctypes.c_uint64), ("quads", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_float), ("total_ms", ctypes.c_float),
        ("captured", ctypes.c_int32), ("redraws", ctypes.c_int32),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libbdeg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1501_02237_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, U64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t
    sig = {
        "bdeg_init": ([I32], ctypes.c_int),
        "bdeg_set_schedule": ([I32], ctypes.c_int),
        "bdeg_degree": ([P, I32, I32, U64, I32, P], ctypes.c_int),
        "bdeg_degree_batch": ([P, P, P, I32, U64, I32, P], ctypes.c_int),
        "bdeg_batch_create": ([P, P, P, I32, U64, I32, P], ctypes.c_int),
        "bdeg_batch_run": ([P], ctypes.c_int),
        "bdeg_batch_results": ([P, P], ctypes.c_int),
        "bdeg_batch_stats": ([P, P], ctypes.c_int),
        "bdeg_batch_profile": ([P], ctypes.c_int),
        "bdeg_batch_destroy": ([P], ctypes.c_int),
        "bdeg_batch_tune": ([P, ctypes.c_char_p, I32], ctypes.c_int),
        "bdeg_nvol_points": ([P, P, I32, I32, U64, U64, P, P, P], ctypes.c_int),
        "bdeg_nvol_points_noalloc": ([P, P, I32, I32, U64, U64, P, P, P], ctypes.c_int),
        "bdeg_nvol_points_pruned": ([P, P, I32, I32, I32, P, P, P, P], ctypes.c_int),
        "bdeg_kernel_points": ([P, I32, I32, P, P, P, P], ctypes.c_int),
        "bdeg_consistency": ([P, I32, I32, P, ctypes.c_double, P, P, P], ctypes.c_int),
        "bdeg_pivot_points": ([P, P, I32, I32, U64, U64, P, P, P, P], ctypes.c_int),
        "bdeg_degree_pivot": ([P, I32, I32, U64, I32, P], ctypes.c_int),
        "bdeg_extend_points": ([P, P, I32, I32, P, P], ctypes.c_int),
        "bdeg_pivot_cells": ([P, P, I32, I32, U64, U64, P, P, P, P, P, P], ctypes.c_int),
        "bdeg_cells_points": ([P, P, I32, I32, U64, U64, U64, P, P, P, P, P], ctypes.c_int),
        "bdeg_subdivision": ([P, I32, I32, U64, I32, U64, P, P, P, P, P, P, P], ctypes.c_int),
        "bdeg_serve_open": ([SZ, P], ctypes.c_int),
        "bdeg_serve_submit": ([P, P, I32, I32, U64, I32, P], ctypes.c_int),
        "bdeg_serve_poll": ([P, U64, P], ctypes.c_int),
        "bdeg_serve_wait": ([P, U64, P], ctypes.c_int),
        "bdeg_serve_latency": ([P, U64, P], ctypes.c_int),
        "bdeg_serve_close": ([P], ctypes.c_int),
        "bdeg_plan_units": ([I32, I32, U64, U64, U64, P, SZ, P], ctypes.c_int),
        "bdeg_strerror": ([ctypes.c_int], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _ = I64
    _lib = L
    return L


def header_functions() -> list[str]:
    """Names of the functions declared in include/bdeg.h."""
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(bdeg_\w+)\s*\(", src, flags=re.M)))


def strerror(code: int) -> str:
    try:
        return lib().bdeg_strerror(code).decode()
    except ImportError:
        return f"error {code}"


def _mat(A) -> np.ndarray:
    A = np.ascontiguousarray(np.asarray(A, dtype=np.int64))
    if A.ndim != 2:
        raise ValueError("A must be a 2-D integer matrix (m x n)")
    return A


def set_schedule(schedule: int) -> None:
    """bdeg_set_schedule: SCHED_AUTO (lane-dense kernel for certified k >= 3
    systems) or SCHED_POINTS (lanes as points everywhere)."""
    rc = lib().bdeg_set_schedule(schedule)
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_set_schedule")


def degree(A, seed: int = 1, lift_bits: int = 20, check: bool = True) -> dict:
    """{status, k, rank, comps, nvol, attempts, flags, candidates, cells} of x^A = b."""
    A = _mat(A)
    r = Result()
    rc = lib().bdeg_degree(A.ctypes.data, A.shape[0], A.shape[1], seed & U64_MAX, lift_bits, ctypes.byref(r))
    if check and rc != BDEG_OK:
        raise BdegError(rc, "bdeg_degree")
    d = r.as_dict()
    d["status"] = rc if rc != BDEG_OK else d["status"]
    return d


def _pack(mats):
    mats = [_mat(A) for A in mats]
    m = np.array([A.shape[0] for A in mats], dtype=np.int32)
    n = np.array([A.shape[1] for A in mats], dtype=np.int32)
    cat = np.ascontiguousarray(np.concatenate([A.ravel() for A in mats]).astype(np.int64))
    return cat, m, n


def degree_pivot(A, seed: int = 1, lift_bits: int = 20, check: bool = True) -> dict:
    """Degree data of x^A = b computed by the cell walk (simplicial pivoting), k <= 24."""
    A = _mat(A)
    r = Result()
    rc = lib().bdeg_degree_pivot(A.ctypes.data, A.shape[0], A.shape[1], seed & U64_MAX, lift_bits, ctypes.byref(r))
    if check and rc != BDEG_OK:
        raise BdegError(rc, "bdeg_degree_pivot")
    d = r.as_dict()
    d["status"] = rc if rc != BDEG_OK else d["status"]
    return d


def pivot_points(points, heights, start_mask: int, cap: int = 0) -> dict:
    """The cell walk from a caller's start cell: {nvol, cells, tie, masks}."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    masks = np.zeros(max(cap, 1), dtype=np.uint64)
    n, nv, tie = ctypes.c_uint64(), U128(), ctypes.c_int32()
    rc = lib().bdeg_pivot_points(P.ctypes.data, H.ctypes.data, N, k, int(start_mask) & U64_MAX, cap,
                                 masks.ctypes.data, ctypes.byref(n), ctypes.byref(nv), ctypes.byref(tie))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_pivot_points")
    return dict(nvol=nv.value, cells=n.value, tie=bool(tie.value), masks=masks[: min(cap, n.value)].copy())


def extend_points(points, heights) -> dict:
    """Extend: a lower facet of the lifted points, {mask, tie}."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    m, tie = ctypes.c_uint64(), ctypes.c_int32()
    rc = lib().bdeg_extend_points(P.ctypes.data, H.ctypes.data, N, k, ctypes.byref(m), ctypes.byref(tie))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_extend_points")
    return dict(mask=m.value, tie=bool(tie.value))


def pivot_cells(points, heights, start_mask: int = 0, cap: int = 1 << 16) -> dict:
    """The cell walk (start_mask 0: from Extend's facet) with the cells'
    inner normals: {nvol, cells, tie, cell_list (Cells)}."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    while True:
        masks, num, den = np.zeros(max(cap, 1), dtype=np.uint64), np.zeros((max(cap, 1), k), dtype=np.int64), \
            np.zeros(max(cap, 1), dtype=np.uint64)
        n, nv, tie = ctypes.c_uint64(), U128(), ctypes.c_int32()
        rc = lib().bdeg_pivot_cells(P.ctypes.data, H.ctypes.data, N, k, int(start_mask) & U64_MAX, cap,
                                    masks.ctypes.data, num.ctypes.data, den.ctypes.data, ctypes.byref(n),
                                    ctypes.byref(nv), ctypes.byref(tie))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_pivot_cells")
        c = n.value
        if c <= cap:
            break
        cap = c
    return dict(nvol=nv.value, cells=c, tie=bool(tie.value),
                cell_list=Cells(masks[:c].copy(), num[:c].copy(), den[:c].copy(), bool(tie.value)))


class PruneStats(ctypes.Structure):
    _fields_ = [
        ("prefixes", ctypes.c_uint64), ("degenerate", ctypes.c_uint64), ("pruned", ctypes.c_uint64),
        ("units", ctypes.c_uint64), ("pivots", ctypes.c_uint64), ("prefix_size", ctypes.c_int32),
        ("width", ctypes.c_int32), ("filter_ms", ctypes.c_float), ("enum_ms", ctypes.c_float),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def nvol_points_pruned(points, heights, width: int = 0) -> dict:
    """bdeg_nvol_points over all candidates with prefix pruning: {nvol, tie, cells, stats}."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    nv, tie, cells, ps = U128(), ctypes.c_int32(), ctypes.c_uint64(), PruneStats()
    rc = lib().bdeg_nvol_points_pruned(P.ctypes.data, H.ctypes.data, N, k, width, ctypes.byref(nv),
                                       ctypes.byref(tie), ctypes.byref(cells), ctypes.byref(ps))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_nvol_points_pruned")
    return dict(nvol=nv.value, tie=bool(tie.value), cells=cells.value, stats=ps.as_dict())


def degree_batch(mats, seed: int = 1, lift_bits: int = 20, check: bool = True) -> list[dict]:
    """Many systems in one device launch; raises on the first failing system's
    code unless check=False (then every result carries its own status)."""
    cat, m, n = _pack(mats)
    out = (Result * len(m))()
    rc = lib().bdeg_degree_batch(cat.ctypes.data, m.ctypes.data, n.ctypes.data, len(m), seed & U64_MAX, lift_bits,
                                 out)
    if check and rc != BDEG_OK:
        raise BdegError(rc, "bdeg_degree_batch")
    return [r.as_dict() for r in out]


def consistency(A, b, tol: float = 1e-9) -> dict:
    """Host only: {consistent, residual, relations} of x^A = b (b: m complex values)."""
    A = _mat(A)
    m, n = A.shape
    bb = np.asarray(b, dtype=np.complex128).reshape(m)
    pairs = np.ascontiguousarray(np.stack([bb.real, bb.imag], axis=1).astype(np.float64))
    ok, res, rel = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    rc = lib().bdeg_consistency(A.ctypes.data, m, n, pairs.ctypes.data, float(tol), ctypes.byref(ok),
                                ctypes.byref(res), ctypes.byref(rel))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_consistency")
    return dict(consistent=bool(ok.value), residual=res.value, relations=rel.value)


def kernel_points(A) -> tuple[int, int, int, np.ndarray]:
    """Host prologue only: (k, rank, comps, points (n+1) x k int32)."""
    A = _mat(A)
    m, n = A.shape
    k, rank, comps = ctypes.c_int32(), ctypes.c_int32(), U128()
    pts = np.zeros((n + 1) * max(n, 1), dtype=np.int32)
    rc = lib().bdeg_kernel_points(A.ctypes.data, m, n, ctypes.byref(k), ctypes.byref(rank), ctypes.byref(comps),
                                  pts.ctypes.data)
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_kernel_points")
    return k.value, rank.value, comps.value, pts[: (n + 1) * k.value].reshape(n + 1, k.value)


def plan_units(N: int, k: int, rank_lo: int = 0, rank_hi: int | None = None, max_cost: int = 256) -> np.ndarray:
    """Host-only: the device work units as colex rank intervals [start, end)."""
    n = ctypes.c_size_t()
    hi = U64_MAX if rank_hi is None else rank_hi
    lib().bdeg_plan_units(N, k, rank_lo, hi, max_cost, None, 0, ctypes.byref(n))
    buf = np.zeros(2 * max(n.value, 1), dtype=np.uint64)
    rc = lib().bdeg_plan_units(N, k, rank_lo, hi, max_cost, buf.ctypes.data, n.value, ctypes.byref(n))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_plan_units")
    return buf[: 2 * n.value].reshape(-1, 2)


@dataclass
class VolumeRange:
    nvol: int
    tie: bool
    cells: int


def nvol_points(points, heights, rank_lo: int = 0, rank_hi: int | None = None) -> VolumeRange:
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    nv, tie, cells = U128(), ctypes.c_int32(), ctypes.c_uint64()
    rc = lib().bdeg_nvol_points(P.ctypes.data, H.ctypes.data, N, k, rank_lo, U64_MAX if rank_hi is None else rank_hi,
                                ctypes.byref(nv), ctypes.byref(tie), ctypes.byref(cells))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_nvol_points")
    return VolumeRange(nv.value, bool(tie.value), cells.value)


def nvol_points_noalloc(points, heights, rank_lo: int = 0, rank_hi: int | None = None) -> VolumeRange:
    """bdeg_nvol_points_noalloc: nvol_points with every device buffer taken
    from the library's static scratch array (no device allocation)."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    nv, tie, cells = U128(), ctypes.c_int32(), ctypes.c_uint64()
    rc = lib().bdeg_nvol_points_noalloc(P.ctypes.data, H.ctypes.data, N, k, rank_lo,
                                        U64_MAX if rank_hi is None else rank_hi, ctypes.byref(nv),
                                        ctypes.byref(tie), ctypes.byref(cells))
    if rc != BDEG_OK:
        raise BdegError(rc, "bdeg_nvol_points_noalloc")
    return VolumeRange(nv.value, bool(tie.value), cells.value)


@dataclass
class Cells:
    """Lower facets with inner normals (alpha, 1), alpha = num / den."""
    masks: np.ndarray  # uint64 [c]: bit i set for vertex i
    num: np.ndarray    # int64 [c, k]
    den: np.ndarray    # uint64 [c]: the cells' normalized volumes
    tie: bool

    def as_set(self) -> set:
        return {(int(m), tuple(int(x) for x in n), int(d)) for m, n, d in zip(self.masks, self.num, self.den)}


def _cell_arrays(cap: int, k: int):
    return (np.zeros(max(cap, 1), dtype=np.uint64), np.zeros((max(cap, 1), max(k, 1)), dtype=np.int64),
            np.zeros(max(cap, 1), dtype=np.uint64))


def cells_points(points, heights, rank_lo: int = 0, rank_hi: int | None = None, cap: int = 65536) -> Cells:
    """Cells of the regular subdivision among candidates of colex rank in
    [rank_lo, rank_hi), with exact inner normals (a second call with a larger
    buffer when more than cap cells exist)."""
    P = np.ascontiguousarray(np.asarray(points, dtype=np.int32))
    H = np.ascontiguousarray(np.asarray(heights, dtype=np.int64))
    N, k = P.shape
    hi = U64_MAX if rank_hi is None else rank_hi
    while True:
        masks, num, den = _cell_arrays(cap, k)
        cnt, tie = ctypes.c_uint64(), ctypes.c_int32()
        rc = lib().bdeg_cells_points(P.ctypes.data, H.ctypes.data, N, k, rank_lo, hi, cap, masks.ctypes.data,
                                     num.ctypes.data, den.ctypes.data, ctypes.byref(cnt), ctypes.byref(tie))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_cells_points")
        c = cnt.value
        if c <= cap:
            return Cells(masks[:c].copy(), num[:c, :k].copy(), den[:c].copy(), bool(tie.value))
        cap = c


def subdivision(A, seed: int = 1, lift_bits: int = 20, cap: int = 65536) -> dict:
    """The regular subdivision behind degree(A, seed, lift_bits): the degree
    result plus "points", "heights" (the lifting used) and "cell_list"."""
    A = _mat(A)
    m, n = A.shape
    while True:
        pts = np.zeros((n + 1) * n, dtype=np.int32)
        hts = np.zeros(n + 1, dtype=np.int64)
        masks, num_full, den = np.zeros(max(cap, 1), dtype=np.uint64), np.zeros(max(cap, 1) * n, dtype=np.int64), \
            np.zeros(max(cap, 1), dtype=np.uint64)
        cnt, r = ctypes.c_uint64(), Result()
        rc = lib().bdeg_subdivision(A.ctypes.data, m, n, seed & U64_MAX, lift_bits, cap, pts.ctypes.data,
                                    hts.ctypes.data, masks.ctypes.data, num_full.ctypes.data, den.ctypes.data,
                                    ctypes.byref(cnt), ctypes.byref(r))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_subdivision")
        c = cnt.value
        if c <= cap:
            break
        cap = c
    d = r.as_dict()
    k = d["k"]
    d["points"] = pts[: (n + 1) * k].reshape(n + 1, k)
    d["heights"] = hts
    d["cell_list"] = Cells(masks[:c].copy(), num_full[: c * k].reshape(c, k).copy(), den[:c].copy(), False)
    return d


class Batch:
    """Prepared, device-resident batch with a captured device pass."""

    def __init__(self, mats, seed: int = 1, lift_bits: int = 20):
        cat, m, n = _pack(mats)
        self.count = len(m)
        self._h = ctypes.c_void_p()
        rc = lib().bdeg_batch_create(cat.ctypes.data, m.ctypes.data, n.ctypes.data, self.count, seed & U64_MAX,
                                     lift_bits, ctypes.byref(self._h))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_batch_create")

    def run(self) -> None:
        rc = lib().bdeg_batch_run(self._h)
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_batch_run")

    def results(self) -> list[dict]:
        out = (Result * self.count)()
        lib().bdeg_batch_results(self._h, out)
        return [r.as_dict() for r in out]

    def stats(self) -> dict:
        s = Stats()
        lib().bdeg_batch_stats(self._h, ctypes.byref(s))
        return s.as_dict()

    def tune(self, table_path: str | None = None, reps: int = 3) -> None:
        """Autotune the work schedule per (k, lane-group width) bucket on this
        batch's systems; write the table to table_path (None: not written)
        and apply it (bdeg_batch_tune)."""
        path = None if table_path is None else os.fsencode(table_path)
        rc = lib().bdeg_batch_tune(self._h, path, reps)
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_batch_tune")

    def profile(self) -> dict:
        """One extra device pass with the work-counting kernel variant."""
        rc = lib().bdeg_batch_profile(self._h)
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_batch_profile")
        return self.stats()

    def close(self) -> None:
        if self._h:
            lib().bdeg_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching request engine (bdeg_serve_*)."""

    def __init__(self, device_mem_budget: int = 256 << 20):
        self._h = ctypes.c_void_p()
        rc = lib().bdeg_serve_open(device_mem_budget, ctypes.byref(self._h))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_serve_open")

    def submit(self, A, seed: int = 1, lift_bits: int = 20) -> int:
        A = _mat(A)
        t = ctypes.c_uint64()
        rc = lib().bdeg_serve_submit(self._h, A.ctypes.data, A.shape[0], A.shape[1], seed & U64_MAX, lift_bits,
                                     ctypes.byref(t))
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_serve_submit")
        return t.value

    def poll(self, ticket: int):
        r = Result()
        rc = lib().bdeg_serve_poll(self._h, ticket, ctypes.byref(r))
        if rc == BDEG_PENDING:
            return None
        if rc != BDEG_OK and rc != r.status:
            raise BdegError(rc, "bdeg_serve_poll")
        return r.as_dict()

    def wait(self, ticket: int) -> dict:
        r = Result()
        rc = lib().bdeg_serve_wait(self._h, ticket, ctypes.byref(r))
        if rc != BDEG_OK and rc != r.status:
            raise BdegError(rc, "bdeg_serve_wait")
        return r.as_dict()

    def latency_ms(self, ticket: int) -> float | None:
        """Submit-to-completion time of a finished request (engine clock)."""
        ns = ctypes.c_uint64()
        rc = lib().bdeg_serve_latency(self._h, ticket, ctypes.byref(ns))
        if rc == BDEG_PENDING:
            return None
        if rc != BDEG_OK:
            raise BdegError(rc, "bdeg_serve_latency")
        return ns.value * 1e-6

    def close(self) -> None:
        if self._h:
            lib().bdeg_serve_close(self._h)
            self._h = ctypes.c_void_p()
