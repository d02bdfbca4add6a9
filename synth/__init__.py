"""Seeded synthetic Hamming-space workloads shaped like the paper's data.

This module only draws random bit vectors; it holds none of Fast
CoveringLSH's arithmetic and is the one piece of code shared by the test
oracle side and the GPU side (both read the same arrays).

Layout of every point set: uint64 [n, W], W = ceil(d/64); coordinate c is bit
(c & 63) of word (c >> 6); bits beyond d in the last word are zero.

Workloads (the paper's datasets are not available; these stand in for their
shapes, see the design notes for which stands in for what):

  uniform_with_planted   i.i.d. uniform bits (the paper's synthetic sets,
                         Sec. 4.2) with neighbours planted around each query
  mixture                points drawn from random centres with independent
                         per-bit flip noise (learned binary codes / document
                         fingerprints, Table 2 shapes)
  hamming_balls          the synthetic sets of the precision/recall study
                         (Sec. 4.3): around each uniform query, points at
                         distances spread uniformly over 1..max_radius
  sparse_planted         very high-dimensional sparse binary vectors (the
                         bag-of-words and user-rating shapes of Table 2) as
                         CSR rows of ascending nonzero coordinates, with
                         neighbours planted around some queries

Sparse layout: ptr int64 [n+1] (ptr[0] = 0), cols int32 [ptr[n]]; point i has
the coordinates cols[ptr[i]:ptr[i+1]] set, ascending and distinct.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def words(d: int) -> int:
    return (d + 63) // 64


def _pack_bits(bits: np.ndarray, d: int) -> np.ndarray:
    """bool/uint8 [n, d] -> uint64 [n, W], coordinate c = bit c&63 of word c>>6."""
    n = bits.shape[0]
    W = words(d)
    padded = np.zeros((n, W * 64), np.uint8)
    padded[:, :d] = bits
    packed = np.packbits(padded, axis=1, bitorder="little")  # [n, W*8] bytes
    return np.ascontiguousarray(packed).view("<u8").reshape(n, W)


def _pad_mask(d: int) -> np.ndarray:
    W = words(d)
    m = np.full(W, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64)
    if d % 64:
        m[-1] = np.uint64((1 << (d % 64)) - 1)
    return m


def uniform_points(n: int, d: int, rng: np.random.Generator) -> np.ndarray:
    x = rng.integers(0, np.iinfo(np.uint64).max, size=(n, words(d)), dtype=np.uint64,
                     endpoint=True)
    return x & _pad_mask(d)


def flip_distinct(x: np.ndarray, d: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """Copy of point x (uint64 [W]) with k distinct uniformly chosen bits flipped."""
    y = x.copy()
    if k:
        pos = rng.choice(d, size=k, replace=False)
        for c in pos:
            y[c >> 6] ^= np.uint64(1) << np.uint64(c & 63)
    return y


def bernoulli_bits(n: int, d: int, p, rng: np.random.Generator, chunk: int = 1 << 17) -> np.ndarray:
    """uint64 [n, W] noise words whose bits are independently 1 with probability
    p (scalar, or one value per row).  p is quantised to multiples of 2^-16."""
    out = np.empty((n, words(d)), np.uint64)
    p = np.broadcast_to(np.asarray(p, np.float64), (n,))
    thr = np.round(p * 65536.0).astype(np.uint32)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = rng.integers(0, 65536, size=(e - s, d), dtype=np.uint16)
        out[s:e] = _pack_bits(u < thr[s:e, None], d)
    return out


@dataclass
class Workload:
    name: str
    d: int
    r: int
    points: np.ndarray  # uint64 [n, W]
    queries: np.ndarray  # uint64 [nq, W]
    query_radius: np.ndarray | None = None  # int32 [nq]: per-query radius if mixed
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def nq(self) -> int:
        return int(self.queries.shape[0])


def uniform_with_planted(n: int, d: int, r: int, nq: int, per_query: int, seed: int,
                         name: str = "uniform", query_radius: np.ndarray | None = None) -> Workload:
    """Uniform points; query j is a copy of a random data point a_j, and
    per_query planted points are the query with k ~ U{0..r_j} distinct bits
    flipped (r_j = query_radius[j] if given, else r), written into fresh slots
    disjoint from all anchors."""
    rng = np.random.default_rng(seed)
    pts = uniform_points(n, d, rng)
    need = nq * (1 + per_query)
    if need > n:
        raise ValueError("not enough points to plant neighbours")
    slots = rng.choice(n, size=need, replace=False)
    anchors = slots[:nq]
    planted = slots[nq:].reshape(nq, per_query) if per_query else np.zeros((nq, 0), np.int64)
    queries = pts[anchors].copy()
    for j in range(nq):
        rj = int(query_radius[j]) if query_radius is not None else r
        for s in planted[j]:
            pts[s] = flip_distinct(queries[j], d, int(rng.integers(0, rj + 1)), rng)
    return Workload(name, d, r, pts, queries, query_radius,
                    {"anchors": anchors, "planted": planted, "seed": seed})


def mixture(n: int, d: int, r: int, n_centers: int, p, nq: int, seed: int,
            name: str = "mixture") -> Workload:
    """Points and queries drawn i.i.d. from a mixture of n_centers uniform
    random centres (cluster chosen uniformly), each bit flipped independently
    with the cluster's noise p.  p is a float (all clusters) or a pair
    (lo, hi): then each cluster draws its own p ~ U[lo, hi]."""
    rng = np.random.default_rng(seed)
    centers = uniform_points(n_centers, d, rng)
    if isinstance(p, tuple):
        pc = rng.uniform(p[0], p[1], size=n_centers)
    else:
        pc = np.full(n_centers, float(p))
    mask = _pad_mask(d)

    def draw(m):
        c = rng.integers(0, n_centers, size=m)
        noise = bernoulli_bits(m, d, pc[c], rng)
        return (centers[c] ^ noise) & mask, c

    pts, pc_of = draw(n)
    qs, qc_of = draw(nq)
    return Workload(name, d, r, pts, qs, None,
                    {"centers": n_centers, "p": p, "seed": seed, "cluster": pc_of,
                     "query_cluster": qc_of})


def hamming_balls(n: int, d: int, nq: int, seed: int, max_radius: int | None = None,
                  name: str = "hamming_balls") -> Workload:
    """nq uniform queries; the n points are split evenly among them (point i
    belongs to query i % nq), and each point is its query with k ~ U{1..R}
    distinct uniformly chosen bits flipped, R = max_radius (default d)."""
    rng = np.random.default_rng(seed)
    R = d if max_radius is None else int(max_radius)
    queries = uniform_points(nq, d, rng)
    owner = np.arange(n) % nq
    k = rng.integers(1, R + 1, size=n)
    # the k smallest of d random keys per row pick k distinct coordinates
    order = np.argsort(rng.random((n, d)), axis=1)
    flip = np.zeros((n, d), np.uint8)
    rows = np.repeat(np.arange(n), k)
    cols = order[np.arange(d)[None, :] < k[:, None]]  # row-major: the first k of each row
    flip[rows, cols] = 1
    pts = queries[owner] ^ _pack_bits(flip, d)
    return Workload(name, d, 0, pts, queries, None, {"owner": owner, "flips": k, "seed": seed})


# ---------------------------------------------------------------------------
# The five workload shapes.  `scale` < 1 shrinks n and the query count for
# parity tests that must finish on the CPU oracle in seconds.
# ---------------------------------------------------------------------------

def small(scale: float = 1.0) -> Workload:
    """n = 10,000 uniform 128-bit points, r = 4; 100 queries x 5 planted."""
    n = max(200, int(10_000 * scale))
    nq = max(4, int(100 * scale))
    return uniform_with_planted(n, 128, 4, nq, 5, seed=1001, name="small")


def mid(scale: float = 1.0) -> Workload:
    """n = 1,000,000 uniform 256-bit points, r = 8; 1,000 queries x 10 planted."""
    n = max(2000, int(1_000_000 * scale))
    nq = max(4, int(1000 * scale))
    return uniform_with_planted(n, 256, 8, nq, 10, seed=1002, name="mid")


def learned_code(scale: float = 1.0) -> Workload:
    """n = 10,000,000 64-bit points from 10,000 centres with flip noise 0.05,
    r = 6; 10,000 queries from the same mixture."""
    n = max(2000, int(10_000_000 * scale))
    nq = max(4, int(10_000 * scale))
    nc = max(10, int(10_000 * scale))
    return mixture(n, 64, 6, nc, 0.05, nq, seed=1003, name="learned_code")


def batched(scale: float = 1.0) -> Workload:
    """n = 4,000,000 512-bit points from 1,000 centres with per-cluster noise
    p ~ U[0.02, 0.15], r = 12; 100,000 queries from the same mixture."""
    n = max(2000, int(4_000_000 * scale))
    nq = max(4, int(100_000 * scale))
    nc = max(4, int(1000 * scale))
    return mixture(n, 512, 12, nc, (0.02, 0.15), nq, seed=1004, name="batched")


def served_a(scale: float = 1.0, nq: int = 4096) -> Workload:
    """Index A of the served workload: n = 2,000,000 uniform 256-bit points,
    r = 10, 5 planted per query at per-query radius r_q ~ U{0..10}."""
    n = max(2000, int(2_000_000 * scale))
    rng = np.random.default_rng(2005)
    rq = rng.integers(0, 11, size=nq).astype(np.int32)
    return uniform_with_planted(n, 256, 10, nq, 5, seed=1005, name="served_a", query_radius=rq)


def served_b(scale: float = 1.0, nq: int = 4096) -> Workload:
    """Index B of the served workload: n = 500,000 uniform 1024-bit points,
    r = 20, 5 planted per query at per-query radius r_q ~ U{0..20}."""
    n = max(2000, int(500_000 * scale))
    rng = np.random.default_rng(2006)
    rq = rng.integers(0, 21, size=nq).astype(np.int32)
    return uniform_with_planted(n, 1024, 20, nq, 5, seed=1006, name="served_b", query_radius=rq)


def fig3_replication(scale: float = 1.0) -> Workload:
    """The shape of the paper's pre-processing experiment (Fig. 3): n = 65,536
    uniform 128-bit points, r = 3, the index built on 3 copies of every point
    (L = 1023); 1,000 queries x 10 planted."""
    n = max(2000, int(65_536 * scale))
    nq = max(4, int(1000 * scale))
    w = uniform_with_planted(n, 128, 3, nq, 10, seed=1007, name="fig3_replication")
    w.meta["replicate"] = 3
    return w


# ---------------------------------------------------------------------------
# Sparse high-dimensional workloads
# ---------------------------------------------------------------------------

def csr_to_words(ptr: np.ndarray, cols: np.ndarray, d: int) -> np.ndarray:
    """CSR rows -> packed uint64 [n, W] (coordinate c = bit c&63 of word c>>6)."""
    n = len(ptr) - 1
    W = words(d)
    out = np.zeros((n, W), np.uint64)
    rows = np.repeat(np.arange(n), np.diff(ptr))
    c = np.asarray(cols, np.int64)
    np.bitwise_or.at(out, (rows, c >> 6), np.left_shift(np.uint64(1), (c & 63).astype(np.uint64)))
    return out


def sparse_rows(n: int, d: int, mean_nnz: float, sigma: float, zipf_a: float,
                rng: np.random.Generator) -> tuple[np.ndarray, np.ndarray]:
    """n rows whose lengths are log-normal (mean about mean_nnz, shape sigma,
    at least 1) and whose coordinates follow a Zipf-like popularity
    (probability of the column of popularity rank k proportional to
    (k+1)^-zipf_a, ranks shuffled over the d columns): each row draws twice
    its length with replacement and keeps a random subset of that length of
    its distinct columns (fewer if there are fewer).  Returns (ptr, cols)."""
    mu = np.log(mean_nnz) - sigma * sigma / 2
    k = np.clip(np.rint(rng.lognormal(mu, sigma, size=n)), 1, d).astype(np.int64)
    w = (np.arange(d, dtype=np.float64) + 1.0) ** (-zipf_a)
    cdf = np.cumsum(w[rng.permutation(d)])
    cdf /= cdf[-1]
    # twice the draws, then a random k of each row's distinct columns
    rows = np.repeat(np.arange(n, dtype=np.int64), 2 * k)
    c = np.minimum(np.searchsorted(cdf, rng.random(rows.size), side="right"), d - 1)
    pair = np.unique(rows * d + c)
    r_of, c_of = pair // d, pair % d
    # (pairs are in (row, column) order; rank them within a row at random)
    order = np.argsort(r_of + rng.random(pair.size), kind="stable")
    first = np.searchsorted(r_of, np.arange(n))
    keep = np.empty(pair.size, bool)
    keep[order] = np.arange(pair.size) - first[r_of[order]] < k[r_of[order]]
    r_of, c_of = r_of[keep], c_of[keep]
    ptr = np.zeros(n + 1, np.int64)
    np.add.at(ptr, r_of + 1, 1)
    return np.cumsum(ptr), c_of.astype(np.int32)


def perturb_row(row: np.ndarray, d: int, k: int, rng: np.random.Generator) -> np.ndarray:
    """The row with k distinct coordinates flipped: each flip removes a
    present coordinate or adds an absent one (even odds while both exist)."""
    have = set(int(x) for x in row)
    out = set(have)
    touched = set()
    while len(touched) < k:
        if out & have - touched and (rng.random() < 0.5 or len(touched) >= d - len(have)):
            c = int(rng.choice(sorted(out & have - touched)))
            out.discard(c)
        else:
            c = int(rng.integers(0, d))
            if c in have or c in touched:
                continue
            out.add(c)
        touched.add(c)
    return np.array(sorted(out), np.int32)


@dataclass
class SparseWorkload:
    name: str
    d: int
    r: int
    ptr: np.ndarray    # int64 [n+1]
    cols: np.ndarray   # int32 [nnz]
    qptr: np.ndarray   # int64 [nq+1]
    qcols: np.ndarray  # int32 [qnnz]
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(len(self.ptr) - 1)

    @property
    def nq(self) -> int:
        return int(len(self.qptr) - 1)

    def dense_points(self) -> np.ndarray:
        return csr_to_words(self.ptr, self.cols, self.d)

    def dense_queries(self) -> np.ndarray:
        return csr_to_words(self.qptr, self.qcols, self.d)


def _rows_to_csr(rows) -> tuple[np.ndarray, np.ndarray]:
    ptr = np.zeros(len(rows) + 1, np.int64)
    ptr[1:] = np.cumsum([len(x) for x in rows])
    cols = np.concatenate(rows).astype(np.int32) if rows else np.zeros(0, np.int32)
    return ptr, cols


def sparse_planted(n: int, d: int, r: int, nq: int, mean_nnz: float, sigma: float, zipf_a: float,
                   planted_queries: int, per_query: int, seed: int, name: str = "sparse") -> SparseWorkload:
    """n + nq rows from sparse_rows; the last nq are the queries (held out
    from the data, as the paper draws its queries from the data sets).
    Around each of the first planted_queries queries, per_query data rows
    are replaced by the query with k ~ U{0..r} coordinates flipped."""
    rng = np.random.default_rng(seed)
    ptr, cols = sparse_rows(n + nq, d, mean_nnz, sigma, zipf_a, rng)
    rows = [cols[ptr[i]:ptr[i + 1]] for i in range(n + nq)]
    data, queries = rows[:n], rows[n:]
    need = planted_queries * per_query
    if need > n:
        raise ValueError("not enough points to plant neighbours")
    slots = rng.choice(n, size=need, replace=False).reshape(planted_queries, per_query) if need else \
        np.zeros((planted_queries, 0), np.int64)
    for j in range(planted_queries):
        for s in slots[j]:
            data[int(s)] = perturb_row(queries[j], d, int(rng.integers(0, r + 1)), rng)
    p, c = _rows_to_csr(data)
    qp, qc = _rows_to_csr(queries)
    return SparseWorkload(name, d, r, p, c, qp, qc, {"planted": slots, "seed": seed, "mean_nnz": mean_nnz})


def enron_like(scale: float = 1.0, r: int = 29) -> SparseWorkload:
    """Bag-of-words shape (Table 2's Enron): n = 40,000 documents over
    d = 28,102 words, about 150 distinct words per document (log-normal
    lengths, Zipf word frequencies), 100 queries, 20 of them with 5 planted
    neighbours within r."""
    n = max(500, int(40_000 * scale))
    nq = max(8, int(100 * scale))
    return sparse_planted(n, 28_102, r, nq, 150.0, 0.8, 1.0, min(nq, 20), 5, seed=1101, name="enron_like")


def movielens_like(scale: float = 1.0, r: int = 13) -> SparseWorkload:
    """User-rating shape (Table 2's MovieLens): n = 234,834 users over
    d = 140,214 movies, about 80 positive ratings per user with a heavy tail
    (log-normal, shape 1.2; Zipf movie popularity), 100 queries, 20 of them
    with 5 planted neighbours within r."""
    n = max(500, int(234_834 * scale))
    nq = max(8, int(100 * scale))
    return sparse_planted(n, 140_214, r, nq, 80.0, 1.2, 0.9, min(nq, 20), 5, seed=1102, name="movielens_like")


SPARSE_WORKLOADS = {"enron_like": enron_like, "movielens_like": movielens_like}


WORKLOADS = {"small": small, "mid": mid, "learned_code": learned_code, "batched": batched,
             "served_a": served_a, "served_b": served_b, "fig3_replication": fig3_replication}
