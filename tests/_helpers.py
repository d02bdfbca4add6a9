"""Shared helpers of the GPU parity tests: oracle-side expected values and
GPU-side marshalling.  Expected values come only from `oracle`."""
from __future__ import annotations

import numpy as np

import oracle


def oracle_derive(d, r, seed, t=0):
    return oracle.derive_params(d, r, seed, override_t=t)


class OracleIndex:
    """The oracle's view of an index: masks, keys of every point, tables."""

    def __init__(self, points: np.ndarray, pr: oracle.Params, with_tables: bool = True):
        self.points = points
        self.pr = pr
        self.mask = oracle.masks(pr)
        self.keys = oracle.keys(points, pr, mask=self.mask)
        if with_tables:
            self.tk, self.ti = oracle.tables(self.keys)

    def binned_tables(self, dir_bits: int):
        """The table layout of the index: per table the oracle's (key, id)
        pairs ordered by directory bin (top dir_bits of the 31-bit key), ids
        ascending inside a bin."""
        L, n = self.keys.shape
        ids = np.arange(n, dtype=np.uint32)
        tk = np.empty_like(self.keys)
        ti = np.empty((L, n), np.uint32)
        for T in range(L):
            order = np.lexsort((ids, self.keys[T] >> np.uint32(31 - dir_bits)))
            tk[T] = self.keys[T][order]
            ti[T] = ids[order]
        return tk, ti

    def query_keys(self, queries):
        return oracle.keys(queries, self.pr, mask=self.mask)

    def strategy2(self, queries, rq):
        return oracle.query_batch(self.points, self.pr.d, self.tk, self.ti, queries, self.query_keys(queries), rq)


def as_u32(t):
    return t.cpu().numpy().view(np.uint32)


def csr_lists(offsets, ids):
    o = offsets.cpu().numpy()
    v = ids.cpu().numpy().view(np.uint32)
    assert o[0] == 0 and np.all(np.diff(o) >= 0) and o[-1] == v.size
    return [v[o[i]:o[i + 1]] for i in range(len(o) - 1)]


def assert_same_lists(got, want, what="query"):
    assert len(got) == len(want)
    for i, (g, w) in enumerate(zip(got, want)):
        assert np.array_equal(np.asarray(g, np.uint32), np.asarray(w, np.uint32)), \
            f"{what} {i}: got {list(g)[:10]} ({len(g)}) want {list(w)[:10]} ({len(w)})"
