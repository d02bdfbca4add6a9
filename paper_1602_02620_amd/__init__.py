"""Python binding of the gfx950 Fast CoveringLSH library (libfclsh.so).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch supplies device memory (tensors) and the stream.  There
is no CPU fallback: if the library is not built, importing works but every
call raises.

    idx = Index(points, d=256, r=8, seed=3002)       # points: int64 [n, W] on the GPU
    offsets, ids = idx.query(queries, r=8)           # CSR: ids of query i in ids[offsets[i]:offsets[i+1]]
    keys = idx.hash(points)                          # [L, n] uint32 keys (as int32 storage)

    sidx = SparseIndex(ptr, cols, d=28102, r=29)     # rows of nonzero coordinates (int64 / int32 on the GPU)
    offsets, ids = sidx.query(qptr, qcols, r=29)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfclsh.so")

FCLSH_OK = 0
FCLSH_EINVAL = -1
FCLSH_ERADIUS = -2
FCLSH_ENOMEM = -3
FCLSH_ECAPACITY = -4
FCLSH_EDEVICE = -5
FCLSH_EUNSUPPORTED = -6

# Every C-ABI entry point declared in include/fclsh.h.
EXPORTS = [
    "fclsh_derive_params", "fclsh_build_index", "fclsh_build_index_with_params", "fclsh_query_batch",
    "fclsh_index_free", "fclsh_last_error", "fclsh_index_info", "fclsh_index_params", "fclsh_hash",
    "fclsh_index_tables", "fclsh_index_rebuild", "fclsh_index_rebuild_timed", "fclsh_query_collisions", "fclsh_query_plain",
    "fclsh_query_batch_radii", "fclsh_query_reserve", "fclsh_query_batch_async", "fclsh_query_graph_create",
    "fclsh_graph_launch", "fclsh_graph_free", "fclsh_index_set_tuning", "fclsh_index_get_tuning",
    "fclsh_autotune", "fclsh_query_batch_finish", "fclsh_index_rebuild_async", "fclsh_index_build_mode",
    "fclsh_preprocessing", "fclsh_index_memory", "fclsh_query_cost",
    "fclsh_query_batch_noalloc", "fclsh_linear_scan", "fclsh_build_index_sparse", "fclsh_hash_sparse",
    "fclsh_query_batch_sparse", "fclsh_index_set_schedule", "fclsh_index_get_schedule",
    "fclsh_query_cost_sparse", "fclsh_index_table_keys",
]

# status bits of the device result of fclsh_query_batch_async
QUERY_PAIR_OVERFLOW = 1
QUERY_SPILL_OVERFLOW = 2
QUERY_IDS_OVERFLOW = 4


class FclshError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"fclsh status {status}: {msg}")
        self.status = status


class BuildOpts(ctypes.Structure):
    """fclsh_build_opts; struct_size is filled in by make()."""
    _fields_ = [("struct_size", ctypes.c_uint32), ("partitions", ctypes.c_int32),
                ("replicate", ctypes.c_int32), ("exclude_column0", ctypes.c_int32),
                ("prime", ctypes.c_uint64), ("mem_budget_bytes", ctypes.c_uint64),
                ("keep_build_scratch", ctypes.c_int32), ("test_flags", ctypes.c_int32)]

    @classmethod
    def make(cls, partitions=0, replicate=0, exclude_column0=False, mem_budget_bytes=0,
             keep_build_scratch=False, test_flags=0):
        return cls(ctypes.sizeof(cls), partitions, replicate, int(bool(exclude_column0)), 0,
                   mem_budget_bytes, int(bool(keep_build_scratch)), int(test_flags))


_lib = None


def lib():
    """Load libfclsh.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_1602_02620_amd/build.py` (there is no CPU fallback)")
        L = ctypes.CDLL(LIB_PATH)
        i32, i64, u64, vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p
        P = ctypes.POINTER
        sig = {
            "fclsh_derive_params": [i32, i32, u64, P(BuildOpts), P(i32), P(i32), vp, vp, vp],
            "fclsh_build_index": [vp, i64, i32, i32, u64, P(BuildOpts), vp, P(vp)],
            "fclsh_build_index_with_params": [vp, i64, i32, i32, i32, i32, vp, vp, vp, u64, vp, P(vp)],
            "fclsh_query_batch": [vp, vp, i64, i32, vp, vp, vp, i64, P(i64)],
            "fclsh_query_plain": [vp, vp, i64, i32, vp, vp, vp, i64, P(i64)],
            "fclsh_index_info": [vp, P(i32), P(i32), P(i32), P(i32), P(i64), P(i32), P(i32), P(i32)],
            "fclsh_index_memory": [vp, P(u64), P(u64), P(u64)],
            "fclsh_index_params": [vp, vp, vp, vp],
            "fclsh_hash": [vp, vp, i64, vp, vp],
            "fclsh_index_tables": [vp, P(vp), P(i32), P(vp), P(vp), P(vp)],
            "fclsh_index_table_keys": [vp, i32, i32, vp, vp],
            "fclsh_index_rebuild": [vp, vp],
            "fclsh_index_rebuild_async": [vp, vp],
            "fclsh_index_rebuild_timed": [vp, vp, P(ctypes.c_float), i32],
            "fclsh_index_build_mode": [vp, P(i32)],
            "fclsh_preprocessing": [i64, i32, ctypes.c_double, P(i32), P(i32)],
            "fclsh_query_collisions": [vp, vp, i64, vp, vp],
            "fclsh_query_cost": [vp, vp, i64, vp, vp, vp],
            "fclsh_linear_scan": [vp, i64, i32, vp, i64, i32, vp, vp, vp, i64, P(i64)],
            "fclsh_query_batch_radii": [vp, vp, i64, vp, i32, vp, vp, vp, i64, P(i64)],
            "fclsh_query_batch_finish": [vp, vp, vp, vp, i64, P(i64)],
            "fclsh_query_reserve": [vp, i64, i64, i64, vp],
            "fclsh_query_batch_async": [vp, vp, i64, i32, vp, vp, vp, vp, i64, vp],
            "fclsh_query_batch_noalloc": [vp, vp, i64, i32, vp, vp, vp, vp, i64, vp],
            "fclsh_query_graph_create": [vp, vp, i64, i32, vp, vp, vp, i64, vp, vp, P(vp)],
            "fclsh_graph_launch": [vp, vp],
            "fclsh_index_set_tuning": [vp, i32, i32],
            "fclsh_index_get_tuning": [vp, P(i32), P(i32)],
            "fclsh_autotune": [vp, vp, i64, i32, vp, P(i32), P(i32), P(ctypes.c_float)],
            "fclsh_build_index_sparse": [vp, vp, i64, i64, i32, i32, u64, P(BuildOpts), vp, P(vp)],
            "fclsh_hash_sparse": [vp, vp, vp, i64, i64, vp, vp],
            "fclsh_query_batch_sparse": [vp, vp, vp, i64, i64, i32, vp, vp, vp, i64, P(i64)],
            "fclsh_index_set_schedule": [vp, i32],
            "fclsh_query_cost_sparse": [vp, vp, vp, i64, i64, vp, vp, vp],
            "fclsh_index_get_schedule": [vp, P(i32)],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = i32
        L.fclsh_index_free.argtypes = [vp]
        L.fclsh_index_free.restype = None
        L.fclsh_graph_free.argtypes = [vp]
        L.fclsh_graph_free.restype = None
        L.fclsh_last_error.argtypes = []
        L.fclsh_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int):
    if status != FCLSH_OK:
        raise FclshError(status, lib().fclsh_last_error().decode())


def words(d: int) -> int:
    return (d + 63) // 64


def preprocessing(n: int, r: int, c: float) -> dict:
    """Alg. 1's choice for n points, radius r, ratio c: dict(replicate, partitions)."""
    rep, t = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().fclsh_preprocessing(n, r, c, ctypes.byref(rep), ctypes.byref(t)))
    return {"replicate": rep.value, "partitions": t.value}


def derive_params(d: int, r: int, seed: int, partitions: int = 0, replicate: int = 0,
                  exclude_column0: bool = False):
    """Host-only parameter draw: returns dict(t, r_part, part, col, b), the
    arrays over the d * replicate coordinates of the replicated point."""
    dd = d * max(1, replicate)
    part = np.zeros(dd, np.int32)
    col = np.zeros(dd, np.int32)
    b = np.zeros(dd, np.uint64)
    t = ctypes.c_int32()
    rp = ctypes.c_int32()
    opts = BuildOpts.make(partitions, replicate, exclude_column0)
    _check(lib().fclsh_derive_params(d, r, seed & (2**64 - 1), ctypes.byref(opts), ctypes.byref(t),
                                     ctypes.byref(rp), part.ctypes.data, col.ctypes.data, b.ctypes.data))
    return {"t": t.value, "r_part": rp.value, "part": part, "col": col, "b": b}


def linear_scan(points, d: int, queries, r: int, stream=None):
    """fclsh_linear_scan: every point within r of each query, without an
    index (offsets int64 [nq+1], ids int32 [total])."""
    torch = _torch()
    pts = _dev_words(points, d, "points")
    q = _dev_words(queries, d, "queries")
    offsets = torch.empty(q.shape[0] + 1, dtype=torch.int64, device=q.device)
    total = ctypes.c_int64()
    cap = max(1024, 16 * q.shape[0])
    for _ in range(2):
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=q.device)
        st = lib().fclsh_linear_scan(ctypes.c_void_p(pts.data_ptr()), pts.shape[0], d, ctypes.c_void_p(q.data_ptr()),
                                     q.shape[0], r, _stream_ptr(stream), ctypes.c_void_p(offsets.data_ptr()),
                                     ctypes.c_void_p(ids.data_ptr()), cap, ctypes.byref(total))
        if st == FCLSH_ECAPACITY:
            cap = total.value
            continue
        _check(st)
        return offsets, ids[:total.value]
    raise FclshError(FCLSH_ECAPACITY, "result did not fit after resizing")


def _torch():
    import torch
    return torch


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_words(x, d: int, what: str):
    """A contiguous int64 [m, W] CUDA tensor holding packed bit vectors."""
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{what} must be a CUDA tensor")
    if x.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{what} must hold 64-bit words")
    x = x.contiguous()
    if x.dim() != 2 or x.shape[1] != words(d):
        raise ValueError(f"{what} must have shape [m, {words(d)}]")
    return x


def to_device_words(arr: np.ndarray, device="cuda"):
    """numpy uint64 [m, W] -> int64 CUDA tensor with the same bits."""
    torch = _torch()
    return torch.from_numpy(np.ascontiguousarray(arr, np.uint64).view(np.int64)).to(device)


class Index:
    """An exact r-NN index (Def. 2) built on the GPU.  Immutable."""

    def __init__(self, points, d: int, r: int, seed: int = 0, partitions: int = 0,
                 mem_budget_bytes: int = 0, stream=None, *, replicate: int = 0,
                 exclude_column0: bool = False, keep_build_scratch: bool = False, _params=None,
                 _test_flags: int = 0):
        torch = _torch()
        pts = _dev_words(points, d, "points")
        n = pts.shape[0]
        h = ctypes.c_void_p()
        st = _stream_ptr(stream)
        if _params is None:
            opts = BuildOpts.make(partitions, replicate, exclude_column0, mem_budget_bytes, keep_build_scratch,
                                  _test_flags)
            _check(lib().fclsh_build_index(ctypes.c_void_p(pts.data_ptr()), n, d, r, seed & (2**64 - 1),
                                           ctypes.byref(opts), st, ctypes.byref(h)))
        else:
            t, rp, part, col, b = _params
            part = np.ascontiguousarray(part, np.int32)
            col = np.ascontiguousarray(col, np.int32)
            b = np.ascontiguousarray(b, np.uint64)
            _check(lib().fclsh_build_index_with_params(ctypes.c_void_p(pts.data_ptr()), n, d, r, t, rp,
                                                       part.ctypes.data, col.ctypes.data, b.ctypes.data,
                                                       0, st, ctypes.byref(h)))
        self._h = h
        self.d = d
        self.replicate = max(1, replicate) if _params is None else 1  # copies per point of the family
        self.device = pts.device
        self._ids_per_query = 64.0  # sizes the id buffer of the next batch
        del torch

    @classmethod
    def with_params(cls, points, d: int, r: int, t: int, r_part: int, part, col, b, stream=None):
        return cls(points, d, r, stream=stream, _params=(t, r_part, part, col, b))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().fclsh_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self) -> dict:
        d, r, t, rp, L, db, gb = (ctypes.c_int32() for _ in range(7))
        n = ctypes.c_int64()
        _check(lib().fclsh_index_info(self._h, ctypes.byref(d), ctypes.byref(r), ctypes.byref(t),
                                      ctypes.byref(rp), ctypes.byref(n), ctypes.byref(L), ctypes.byref(db),
                                      ctypes.byref(gb)))
        return {"d": d.value, "r": r.value, "t": t.value, "r_part": rp.value, "n": n.value, "L": L.value,
                "dir_bits": db.value, "group_bits": gb.value}

    def memory(self) -> dict:
        """fclsh_index_memory: device bytes of the index, its kept build
        scratch and its query workspaces."""
        a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().fclsh_index_memory(self._h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return {"index_bytes": a.value, "build_scratch_bytes": b.value, "workspace_bytes": c.value}

    def params(self) -> dict:
        d = self.d * self.replicate  # the family's coordinates
        part = np.zeros(d, np.int32)
        col = np.zeros(d, np.int32)
        b = np.zeros(d, np.uint64)
        _check(lib().fclsh_index_params(self._h, part.ctypes.data, col.ctypes.data, b.ctypes.data))
        return {"part": part, "col": col, "b": b}

    def hash(self, points, out=None, stream=None):
        """[L, m] keys (int32 storage of the uint32 keys) of m points."""
        torch = _torch()
        pts = _dev_words(points, self.d, "points")
        m = pts.shape[0]
        L = self.info["L"]
        if out is None:
            out = torch.empty((L, m), dtype=torch.int32, device=pts.device)
        _check(lib().fclsh_hash(self._h, ctypes.c_void_p(pts.data_ptr()), m, ctypes.c_void_p(out.data_ptr()),
                                _stream_ptr(stream)))
        return out

    def rebuild(self, stream=None):
        _check(lib().fclsh_index_rebuild(self._h, _stream_ptr(stream)))

    def rebuild_async(self, stream=None):
        """fclsh_index_rebuild_async: enqueue the rebuild on the stream."""
        _check(lib().fclsh_index_rebuild_async(self._h, _stream_ptr(stream)))

    BUILD_MODES = ("full", "slot_only", "slot_all")

    @property
    def build_mode(self) -> str:
        """fclsh_index_build_mode: pass 2's form in the next rebuild."""
        m = ctypes.c_int32()
        _check(lib().fclsh_index_build_mode(self._h, ctypes.byref(m)))
        return self.BUILD_MODES[m.value]

    REBUILD_PHASES = ("fht_hash_kernel", "p1_hist_kernel", "p1_scan_kernel", "p1_scatter_kernel",
                      "p1b_split_kernel", "p2_fast_kernel", "p2_rest_kernel")

    def rebuild_timed(self, stream=None) -> dict:
        """Rebuild with HIP events between the kernels: kernel name -> ms."""
        ms = (ctypes.c_float * len(self.REBUILD_PHASES))()
        _check(lib().fclsh_index_rebuild_timed(self._h, _stream_ptr(stream), ms, len(self.REBUILD_PHASES)))
        return dict(zip(self.REBUILD_PHASES, (float(x) for x in ms)))

    def table_pointers(self):
        """(keys, ids, directory, points) device addresses and the bytes per stored key."""
        k, i, dr, p = (ctypes.c_void_p() for _ in range(4))
        kb = ctypes.c_int32()
        _check(lib().fclsh_index_tables(self._h, ctypes.byref(k), ctypes.byref(kb), ctypes.byref(i),
                                        ctypes.byref(dr), ctypes.byref(p)))
        return k.value, i.value, dr.value, p.value, kb.value

    def tables(self, T0: int = 0, T1: int | None = None):
        """Copies of tables [T0, T1): (whole keys, ids) as int32 CUDA tensors [T1-T0, n]."""
        torch = _torch()
        inf = self.info
        n, L = inf["n"], inf["L"]
        T1 = L if T1 is None else T1
        _, ip, _, _, _ = self.table_pointers()
        keys = torch.empty((T1 - T0, n), dtype=torch.int32, device=self.device)
        ids = torch.empty_like(keys)
        _check(lib().fclsh_index_table_keys(self._h, T0, T1, ctypes.c_void_p(keys.data_ptr()),
                                            _stream_ptr(None)))
        _memcpy_d2d(ids.data_ptr(), ip + T0 * n * 4, (T1 - T0) * n * 4)
        return keys, ids

    def directory(self):
        torch = _torch()
        inf = self.info
        nb = (1 << inf["dir_bits"]) + 1
        _, _, dp, _, _ = self.table_pointers()
        out = torch.empty((inf["L"], nb), dtype=torch.int32, device=self.device)
        _memcpy_d2d(out.data_ptr(), dp, inf["L"] * nb * 4)
        return out

    def _default_capacity(self, nq: int) -> int:
        # ids per query seen in the last batch, with a margin, at least 64
        return max(1024, int(nq * self._ids_per_query) + 1)

    def _collect(self, st, offsets, ids, total, nq, stream, finish: bool, explicit: bool):
        """Result of a batch call: on FCLSH_ECAPACITY with a library-sized
        buffer, the pending batch is finished into a buffer of the reported
        size (no recomputation)."""
        torch = _torch()
        if st == FCLSH_ECAPACITY and not explicit:
            if not finish:
                return None
            ids = torch.empty(max(total.value, 1), dtype=torch.int32, device=offsets.device)
            st = lib().fclsh_query_batch_finish(self._h, _stream_ptr(stream), ctypes.c_void_p(offsets.data_ptr()),
                                                ctypes.c_void_p(ids.data_ptr()), ids.numel(), ctypes.byref(total))
        _check(st)
        if nq:
            self._ids_per_query = max(64.0, 1.25 * total.value / nq)
        return offsets, ids[:total.value]

    def _run_query(self, fn, queries, r: int, ids_capacity=None, stream=None, finish=True):
        torch = _torch()
        q = _dev_words(queries, self.d, "queries")
        nq = q.shape[0]
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=q.device)
        cap = int(ids_capacity) if ids_capacity is not None else self._default_capacity(nq)
        total = ctypes.c_int64()
        for _ in range(2):
            ids = torch.empty(max(cap, 1), dtype=torch.int32, device=q.device)
            st = fn(self._h, ctypes.c_void_p(q.data_ptr()), nq, r, _stream_ptr(stream),
                    ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(ids.data_ptr()), cap,
                    ctypes.byref(total))
            res = self._collect(st, offsets, ids, total, nq, stream, finish, ids_capacity is not None)
            if res is not None:
                return res
            cap = total.value  # the plain path answers again into a larger buffer
        raise FclshError(FCLSH_ECAPACITY, "result did not fit after resizing")

    def query(self, queries, r: int, ids_capacity=None, stream=None):
        """Exact r-NN reporting for a batch: (offsets int64 [nq+1], ids int32 [total])."""
        return self._run_query(lib().fclsh_query_batch, queries, r, ids_capacity, stream)

    def query_plain(self, queries, r: int, ids_capacity=None, stream=None):
        """Same answers via one launch sequence per query (the unbatched baseline)."""
        return self._run_query(lib().fclsh_query_plain, queries, r, ids_capacity, stream, finish=False)

    def query_radii(self, queries, radii, ids_capacity=None, stream=None):
        """Exact r-NN reporting with one radius per query (int32 CUDA tensor)."""
        torch = _torch()
        q = _dev_words(queries, self.d, "queries")
        rad = radii.to(device=q.device, dtype=torch.int32).contiguous()
        nq = q.shape[0]
        if rad.shape != (nq,):
            raise ValueError("one radius per query")
        rmax = int(rad.max().item()) if nq else 0
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=q.device)
        cap = int(ids_capacity) if ids_capacity is not None else self._default_capacity(nq)
        total = ctypes.c_int64()
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=q.device)
        st = lib().fclsh_query_batch_radii(self._h, ctypes.c_void_p(q.data_ptr()), nq,
                                           ctypes.c_void_p(rad.data_ptr()), rmax, _stream_ptr(stream),
                                           ctypes.c_void_p(offsets.data_ptr()),
                                           ctypes.c_void_p(ids.data_ptr()), cap, ctypes.byref(total))
        return self._collect(st, offsets, ids, total, nq, stream, True, ids_capacity is not None)

    def query_finish(self, offsets, ids, stream=None) -> int:
        """fclsh_query_batch_finish: after a batch call with an explicit
        ids_capacity failed with FCLSH_ECAPACITY, writes its ids into `ids`
        (int32 CUDA tensor); returns the total."""
        total = ctypes.c_int64()
        _check(lib().fclsh_query_batch_finish(self._h, _stream_ptr(stream), ctypes.c_void_p(offsets.data_ptr()),
                                              ctypes.c_void_p(ids.data_ptr()), ids.numel(), ctypes.byref(total)))
        return total.value

    def reserve(self, max_nq: int, pair_capacity: int, spill_capacity: int = 1 << 16, stream=None):
        """Size the stream's query workspace for the asynchronous / graph path."""
        _check(lib().fclsh_query_reserve(self._h, max_nq, pair_capacity, spill_capacity, _stream_ptr(stream)))

    def query_async(self, queries, r: int, offsets, ids, result, radii=None, stream=None):
        """Enqueue a batch without host synchronisation.  offsets: int64
        [nq+1], ids: int32 [capacity], result: int64 [2] (total, status bits),
        all CUDA tensors owned by the caller."""
        q = _dev_words(queries, self.d, "queries")
        rp = ctypes.c_void_p(radii.data_ptr()) if radii is not None else ctypes.c_void_p()
        _check(lib().fclsh_query_batch_async(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0], r, rp,
                                             _stream_ptr(stream), ctypes.c_void_p(offsets.data_ptr()),
                                             ctypes.c_void_p(ids.data_ptr()), ids.numel(),
                                             ctypes.c_void_p(result.data_ptr())))

    def query_graph(self, queries, r: int, offsets, ids, result, radii=None, stream=None):
        """Capture query_async on these buffers into a replayable HIP graph."""
        q = _dev_words(queries, self.d, "queries")
        rp = ctypes.c_void_p(radii.data_ptr()) if radii is not None else ctypes.c_void_p()
        g = ctypes.c_void_p()
        _check(lib().fclsh_query_graph_create(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0], r, rp,
                                              ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                                              ids.numel(), ctypes.c_void_p(result.data_ptr()),
                                              _stream_ptr(stream), ctypes.byref(g)))
        return QueryGraph(g)

    def set_tuning(self, tile: int, blocks_per_cu: int):
        _check(lib().fclsh_index_set_tuning(self._h, tile, blocks_per_cu))

    SCHEDULES = ("static", "claim")

    def set_schedule(self, schedule: str):
        """fclsh_index_set_schedule: "static" or "claim"."""
        _check(lib().fclsh_index_set_schedule(self._h, self.SCHEDULES.index(schedule)))

    def get_tuning(self):
        t, b, sc = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().fclsh_index_get_tuning(self._h, ctypes.byref(t), ctypes.byref(b)))
        _check(lib().fclsh_index_get_schedule(self._h, ctypes.byref(sc)))
        return {"tile": t.value, "blocks_per_cu": b.value, "schedule": self.SCHEDULES[sc.value]}

    def autotune(self, queries, r: int, stream=None):
        """Pick the batched launch shape on a sample batch; returns it with its time."""
        q = _dev_words(queries, self.d, "queries")
        t, b, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float()
        _check(lib().fclsh_autotune(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0], r, _stream_ptr(stream),
                                    ctypes.byref(t), ctypes.byref(b), ctypes.byref(ms)))
        return {"tile": t.value, "blocks_per_cu": b.value, "schedule": self.get_tuning()["schedule"],
                "ms": ms.value}

    def collisions(self, queries, stream=None):
        """#Collisions (Sec. 4.1) per query, int64 [nq]."""
        torch = _torch()
        q = _dev_words(queries, self.d, "queries")
        out = torch.empty(q.shape[0], dtype=torch.int64, device=q.device)
        _check(lib().fclsh_query_collisions(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0],
                                            _stream_ptr(stream), ctypes.c_void_p(out.data_ptr())))
        return out


    def cost(self, queries, stream=None):
        """Sec. 4.1's #Collisions and #Candidates per query: (int64 [nq], int64 [nq])."""
        torch = _torch()
        q = _dev_words(queries, self.d, "queries")
        coll = torch.empty(q.shape[0], dtype=torch.int64, device=q.device)
        cand = torch.empty_like(coll)
        _check(lib().fclsh_query_cost(self._h, ctypes.c_void_p(q.data_ptr()), q.shape[0], _stream_ptr(stream),
                                      ctypes.c_void_p(coll.data_ptr()), ctypes.c_void_p(cand.data_ptr())))
        return coll, cand


def to_device_rows(ptr: np.ndarray, cols: np.ndarray, device="cuda"):
    """numpy CSR rows -> (int64 [m+1], int32 [nnz]) CUDA tensors."""
    torch = _torch()
    return (torch.from_numpy(np.ascontiguousarray(ptr, np.int64)).to(device),
            torch.from_numpy(np.ascontiguousarray(cols, np.int32)).to(device))


def _dev_rows(ptr, cols, what: str):
    torch = _torch()
    for x, dt, nm in ((ptr, torch.int64, "ptr"), (cols, torch.int32, "cols")):
        if not isinstance(x, torch.Tensor) or not x.is_cuda or x.dtype != dt or x.dim() != 1:
            raise TypeError(f"{what} {nm} must be a 1-D {dt} CUDA tensor")
    if ptr.numel() < 1:
        raise ValueError(f"{what} ptr needs m+1 >= 1 entries")
    return ptr.contiguous(), cols.contiguous()


class SparseIndex(Index):
    """An exact r-NN index over points given as rows of nonzero coordinates
    (fclsh_build_index_sparse): ptr int64 [n+1], cols int32 [nnz] CUDA
    tensors, d up to 2^19.  Queries are rows too."""

    def __init__(self, ptr, cols, d: int, r: int, seed: int = 0, partitions: int = 0, mem_budget_bytes: int = 0,
                 stream=None, *, exclude_column0: bool = False, keep_build_scratch: bool = False):
        ptr, cols = _dev_rows(ptr, cols, "points")
        h = ctypes.c_void_p()
        opts = BuildOpts.make(partitions, 0, exclude_column0, mem_budget_bytes, keep_build_scratch)
        _check(lib().fclsh_build_index_sparse(ctypes.c_void_p(ptr.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
                                              ptr.numel() - 1, cols.numel(), d, r, seed & (2**64 - 1),
                                              ctypes.byref(opts), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.d = d
        self.replicate = 1
        self.device = ptr.device
        self._ids_per_query = 64.0

    def hash(self, ptr, cols, out=None, stream=None):
        """[L, m] keys (int32 storage) of m rows."""
        torch = _torch()
        ptr, cols = _dev_rows(ptr, cols, "points")
        m = ptr.numel() - 1
        if out is None:
            out = torch.empty((self.info["L"], m), dtype=torch.int32, device=ptr.device)
        _check(lib().fclsh_hash_sparse(self._h, ctypes.c_void_p(ptr.data_ptr()), ctypes.c_void_p(cols.data_ptr()), m,
                                       cols.numel(), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def query(self, ptr, cols, r: int, ids_capacity=None, stream=None):
        """Exact r-NN reporting for a batch of query rows: (offsets int64
        [nq+1], ids int32 [total])."""
        torch = _torch()
        ptr, cols = _dev_rows(ptr, cols, "queries")
        nq = ptr.numel() - 1
        offsets = torch.empty(nq + 1, dtype=torch.int64, device=ptr.device)
        cap = int(ids_capacity) if ids_capacity is not None else self._default_capacity(nq)
        total = ctypes.c_int64()
        ids = torch.empty(max(cap, 1), dtype=torch.int32, device=ptr.device)
        st = lib().fclsh_query_batch_sparse(self._h, ctypes.c_void_p(ptr.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
                                            nq, cols.numel(), r, _stream_ptr(stream),
                                            ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(ids.data_ptr()),
                                            cap, ctypes.byref(total))
        return self._collect(st, offsets, ids, total, nq, stream, True, ids_capacity is not None)

    def cost(self, ptr, cols, stream=None):
        """Sec. 4.1's #Collisions and #Candidates per query row: (int64 [nq], int64 [nq])."""
        torch = _torch()
        ptr, cols = _dev_rows(ptr, cols, "queries")
        nq = ptr.numel() - 1
        coll = torch.empty(nq, dtype=torch.int64, device=ptr.device)
        cand = torch.empty_like(coll)
        _check(lib().fclsh_query_cost_sparse(self._h, ctypes.c_void_p(ptr.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
                                             nq, cols.numel(), _stream_ptr(stream), ctypes.c_void_p(coll.data_ptr()),
                                             ctypes.c_void_p(cand.data_ptr())))
        return coll, cand


class QueryGraph:
    """A captured batched query; launch() replays it on a stream."""

    def __init__(self, handle):
        self._g = handle

    def launch(self, stream=None):
        _check(lib().fclsh_graph_launch(self._g, _stream_ptr(stream)))

    def close(self):
        if self._g and self._g.value:
            lib().fclsh_graph_free(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_hip = None


def _memcpy_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy on torch's current stream, through the HIP runtime."""
    global _hip
    torch = _torch()
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                        ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    rc = _hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3,
                             ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")


def split_csr(offsets, ids):
    """CSR (torch tensors) -> list of numpy uint32 arrays."""
    o = offsets.cpu().numpy()
    v = ids.cpu().numpy().view(np.uint32)
    return [v[o[i]:o[i + 1]] for i in range(len(o) - 1)]
