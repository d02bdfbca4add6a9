"""Plain CPU oracle for Fast CoveringLSH (arXiv:1602.02620) -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never does, and the
oracle imports nothing from it: the two share no code.

The arithmetic lives in ``fclsh_oracle.c`` (plain loops, one function per
definition of the paper, each citing its passage); this module only compiles it
with gcc and marshals numpy arrays through ctypes.

    derive_params   Alg. 1 partitioning + Alg. 2 random draws (SplitMix64)
    replicate       Alg. 1 replication (the copies of a point concatenated)
    masks           basic CoveringLSH masks g_v, Eq. (2) / Eq. (5)
    keys            Eq. (1) universal hash of g_v AND x  (O(d L) per point)
    tables          hash tables of non-empty buckets, sorted by (key, id)
    query_batch     Strategy 2 with S1-S3 of Sec. 4.1 and an n-bit bitmap
    brute_force     linear scan ground truth (Sec. 4.2)
    keys_sparse     Eq. (1) keys of points given by their nonzero coordinates
                    (O(nnz L) per point)
    brute_force_sparse  linear scan over such points
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fclsh_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MERSENNE31 = (1 << 31) - 1


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP across host cores)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
             _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_parts_for_radius.restype = i32
        L.orc_parts_for_radius.argtypes = [i32, i32]
        L.orc_derive_params.restype = i32
        L.orc_derive_params.argtypes = [i32, i32, u64, i32, u64, i32, vp, vp, vp, vp, vp]
        L.orc_masks.restype = None
        L.orc_masks.argtypes = [i32, i32, i32, vp, vp, vp]
        L.orc_keys.restype = None
        L.orc_keys.argtypes = [vp, i32, vp, i64, i32, vp, vp, u64, vp]
        L.orc_tables.restype = None
        L.orc_tables.argtypes = [vp, i64, i32, vp, vp]
        L.orc_query_batch.restype = None
        L.orc_query_batch.argtypes = [vp, i64, i32, vp, vp, i32, vp, i64, vp, i32, i64,
                                      vp, vp, vp, vp]
        L.orc_brute_force.restype = None
        L.orc_brute_force.argtypes = [vp, i64, i32, vp, i64, i32, i64, vp, vp]
        L.orc_keys_sparse.restype = None
        L.orc_keys_sparse.argtypes = [vp, vp, i64, i32, i32, vp, vp, vp, u64, vp]
        L.orc_brute_force_sparse.restype = None
        L.orc_brute_force_sparse.argtypes = [vp, vp, i64, vp, vp, i64, i32, i32, i64, vp, vp]
        L.orc_num_threads.restype = i32
        L.orc_num_threads.argtypes = []
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Params:
    """Index parameters: t parts, per-part radius r', D = 2^(r'+1) columns,
    part[c], col[c] (Hadamard column of coordinate c) and b[c] (Eq. (1) seed
    vector), prime P."""

    d: int
    r: int
    t: int
    rpart: int
    part: np.ndarray  # int32 [d]
    col: np.ndarray  # int32 [d]
    b: np.ndarray  # uint64 [d]
    P: int

    @property
    def D(self) -> int:
        return 1 << (self.rpart + 1)

    @property
    def Lp(self) -> int:
        return self.D - 1

    @property
    def L(self) -> int:
        return self.t * self.Lp


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed & (2**64 - 1), k))


def parts_for_radius(r: int, override_t: int = 0) -> int:
    return int(lib().orc_parts_for_radius(r, override_t))


def derive_params(d: int, r: int, seed: int, override_t: int = 0, P: int = MERSENNE31,
                  exclude_column0: bool = False) -> Params:
    part = np.zeros(d, np.int32)
    col = np.zeros(d, np.int32)
    b = np.zeros(d, np.uint64)
    t = ctypes.c_int32()
    rp = ctypes.c_int32()
    rc = lib().orc_derive_params(d, r, seed & (2**64 - 1), override_t, P, int(bool(exclude_column0)), ctypes.byref(t),
                                 ctypes.byref(rp), _p(part), _p(col), _p(b))
    if rc != 0:
        raise ValueError(f"oracle refused parameters d={d} r={r} t={override_t}")
    return Params(d, r, t.value, rp.value, part, col, b, P)


def preprocessing(n: int, r: int, c: float) -> tuple[int, int]:
    """Alg. 1's branch for n points, radius r and approximation ratio c, log
    base 2: (copies, parts) = (floor(log n / cr), 1) when cr < log n,
    (1, ceil(cr / log n)) when cr > log n, else (1, 1)."""
    logn = math.log2(n)
    cr = c * r
    if cr < logn:
        return math.floor(logn / cr), 1
    if cr > logn:
        return 1, math.ceil(cr / logn)
    return 1, 1


def replicate(points: np.ndarray, d: int, times: int) -> np.ndarray:
    """Alg. 1, first branch: every point repeated `times` times, the copies
    concatenated (coordinate i*d + c of the result is coordinate c).  A
    distance of k between two points becomes times * k.  uint64 [n, W] with d
    coordinates -> uint64 [n, W'] with times * d coordinates."""
    points = np.ascontiguousarray(points, np.uint64)
    n = points.shape[0]
    bits = np.unpackbits(points.view(np.uint8).reshape(n, -1), axis=1, bitorder="little")[:, :d]
    rep = np.tile(bits, (1, times))
    dd = times * d
    W2 = (dd + 63) // 64
    padded = np.zeros((n, W2 * 64), np.uint8)
    padded[:, :dd] = rep
    return np.packbits(padded, axis=1, bitorder="little").view(np.uint64).reshape(n, W2)


def explicit_params(d: int, rpart: int, part, col, b, P: int = MERSENNE31, r: int | None = None) -> Params:
    part = np.ascontiguousarray(part, np.int32)
    t = int(part.max()) + 1 if d else 1
    return Params(d, rpart if r is None else r, t, rpart, part,
                  np.ascontiguousarray(col, np.int32), np.ascontiguousarray(b, np.uint64), P)


def masks(pr: Params) -> np.ndarray:
    """uint8 [L, d]: row T = p*(D-1)+(v-1) is the mask g_v of part p."""
    m = np.zeros((pr.L, pr.d), np.uint8)
    lib().orc_masks(pr.d, pr.t, pr.rpart, _p(pr.part), _p(pr.col), _p(m))
    return m


def keys(points: np.ndarray, pr: Params, which=None, mask: np.ndarray | None = None) -> np.ndarray:
    """uint32 [L, npick]: Eq. (1) key of each (listed) point in every table."""
    points = np.ascontiguousarray(points, np.uint64)
    if mask is None:
        mask = masks(pr)
    if which is None:
        npick = points.shape[0]
        wp = None
    else:
        which = np.ascontiguousarray(which, np.int64)
        npick = which.shape[0]
        wp = _p(which)
    out = np.zeros((pr.L, npick), np.uint32)
    if npick:
        lib().orc_keys(_p(points), pr.d, wp, npick, pr.L, _p(mask), _p(pr.b), pr.P, _p(out))
    return out


def tables(keys_: np.ndarray):
    """Per table, the (key, id) pairs sorted by key then id."""
    keys_ = np.ascontiguousarray(keys_, np.uint32)
    ntab, n = keys_.shape
    tk = np.zeros_like(keys_)
    ti = np.zeros((ntab, n), np.uint32)
    lib().orc_tables(_p(keys_), n, ntab, _p(tk), _p(ti))
    return tk, ti


@dataclass
class QueryResult:
    counts: np.ndarray  # int64 [nq]
    ids: list  # per query uint32 array, ascending
    collisions: np.ndarray | None = None
    candidates: np.ndarray | None = None


def query_batch(points, d, tk, ti, queries, qkeys, rq, cap=None) -> QueryResult:
    points = np.ascontiguousarray(points, np.uint64)
    queries = np.ascontiguousarray(queries, np.uint64)
    qkeys = np.ascontiguousarray(qkeys, np.uint32)
    ntab, n = tk.shape
    nq = queries.shape[0]
    cap = n if cap is None else cap
    out = np.zeros((max(nq, 1), max(cap, 1)), np.uint32)
    counts = np.zeros(max(nq, 1), np.int64)
    coll = np.zeros(max(nq, 1), np.int64)
    cand = np.zeros(max(nq, 1), np.int64)
    lib().orc_query_batch(_p(points), n, d, _p(tk), _p(ti), ntab, _p(queries), nq, _p(qkeys), rq,
                          max(cap, 1), _p(out), _p(counts), _p(coll), _p(cand))
    ids = [out[i, :min(counts[i], cap)].copy() for i in range(nq)]
    return QueryResult(counts[:nq], ids, coll[:nq], cand[:nq])


def brute_force(points, d, queries, rq, cap=None) -> QueryResult:
    points = np.ascontiguousarray(points, np.uint64)
    queries = np.ascontiguousarray(queries, np.uint64)
    n = points.shape[0]
    nq = queries.shape[0]
    cap = n if cap is None else cap
    out = np.zeros((max(nq, 1), max(cap, 1)), np.uint32)
    counts = np.zeros(max(nq, 1), np.int64)
    lib().orc_brute_force(_p(points), n, d, _p(queries), nq, rq, max(cap, 1), _p(out), _p(counts))
    ids = [out[i, :min(counts[i], cap)].copy() for i in range(nq)]
    return QueryResult(counts[:nq], ids)


def _csr(ptr, cols, d: int | None = None):
    ptr = np.ascontiguousarray(ptr, np.int64)
    cols = np.ascontiguousarray(cols, np.int32)
    if ptr.ndim != 1 or ptr.size < 1 or ptr[0] != 0 or ptr[-1] != cols.size or np.any(np.diff(ptr) < 0):
        raise ValueError("ptr must run from 0 to len(cols), non-decreasing")
    if d is not None and cols.size and (cols.min() < 0 or cols.max() >= d):
        raise ValueError("column outside [0, d)")
    return ptr, cols


def keys_sparse(ptr, cols, pr: Params) -> np.ndarray:
    """uint32 [L, m]: Eq. (1) keys of the m points whose nonzero coordinates
    are cols[ptr[i]:ptr[i+1]] (no repeats within a point)."""
    ptr, cols = _csr(ptr, cols, pr.d)
    m = ptr.size - 1
    out = np.zeros((pr.L, m), np.uint32)
    if m:
        lib().orc_keys_sparse(_p(ptr), _p(cols), m, pr.t, pr.rpart, _p(pr.part), _p(pr.col), _p(pr.b), pr.P,
                              _p(out))
    return out


def brute_force_sparse(ptr, cols, qptr, qcols, d: int, rq: int, cap=None) -> QueryResult:
    """Linear scan over points and queries given by their nonzero
    coordinates (d coordinates)."""
    ptr, cols = _csr(ptr, cols, d)
    qptr, qcols = _csr(qptr, qcols, d)
    n = ptr.size - 1
    nq = qptr.size - 1
    cap = n if cap is None else cap
    out = np.zeros((max(nq, 1), max(cap, 1)), np.uint32)
    counts = np.zeros(max(nq, 1), np.int64)
    lib().orc_brute_force_sparse(_p(ptr), _p(cols), n, _p(qptr), _p(qcols), nq, d, rq, max(cap, 1), _p(out),
                                 _p(counts))
    ids = [out[i, :min(counts[i], cap)].copy() for i in range(nq)]
    return QueryResult(counts[:nq], ids)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(k: int) -> None:
    lib().orc_set_num_threads(k)
