"""GPU parity at sizes the oracle finishes in seconds: every key, every table
entry, the directory, every query answer and the #Collisions counters of the
HIP path against the CPU oracle, plus the edge cases (ragged sizes, d not a
multiple of 64, a single point, no queries, duplicate points, radius limits,
output capacity, 3 parts, the largest Hadamard order)."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import OracleIndex, as_u32, assert_same_lists, csr_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return fc.to_device_words(a)


def build(w: synth.Workload, seed: int, partitions: int = 0):
    _say(f"[build] {w.name} n={w.n} d={w.d} r={w.r} seed={seed} t={partitions}")
    idx = fc.Index(dev(w.points), w.d, w.r, seed=seed, partitions=partitions)
    pr = oracle.derive_params(w.d, w.r, seed, override_t=partitions)
    return idx, pr


CASES = {
    # name: (workload factory, index seed, partitions)
    "small": (lambda: synth.small(0.2), 3001, 0),                       # general, D=32
    "mid": (lambda: synth.uniform_with_planted(4099, 256, 8, 8, 10, 1102, "mid"), 3002, 0),  # specific, D=512
    "learned": (lambda: synth.mixture(5003, 64, 6, 6, 0.05, 12, 1103, "learned"), 3003, 0),  # specific, D=128
    "batched": (lambda: synth.mixture(4001, 512, 12, 8, 0.01, 24, 1104, "batched"), 3004, 0),  # t=2 general D=128
    "served_a": (lambda: synth.uniform_with_planted(3001, 256, 10, 10, 5, 1105, "served_a"), 3005, 0),  # t=2, D=64
    "served_b": (lambda: synth.uniform_with_planted(701, 1024, 20, 6, 5, 1106, "served_b"), 3006, 0),  # t=2, D=2048
    "ragged_d": (lambda: synth.uniform_with_planted(1237, 100, 5, 9, 6, 1107, "ragged_d"), 3007, 0),
    "three_parts": (lambda: synth.uniform_with_planted(1500, 96, 9, 6, 6, 1108, "three_parts"), 3008, 3),
    "general_d256": (lambda: synth.uniform_with_planted(2100, 300, 7, 8, 6, 1109, "general_d256"), 3009, 0),  # D=256
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    make, seed, t = CASES[request.param]
    w = make()
    idx, pr = build(w, seed, t)
    orc = OracleIndex(w.points, pr)
    yield request.param, w, idx, orc
    idx.close()


def test_params_agree(case):
    name, w, idx, orc = case
    p = idx.params()
    assert np.array_equal(p["part"], orc.pr.part) and np.array_equal(p["col"], orc.pr.col)
    assert np.array_equal(p["b"], orc.pr.b)
    assert idx.info["L"] == orc.pr.L


def test_keys_bit_exact(case):
    """Lemma 3: the FHT keys equal the Eq. (1) keys of the basic masks."""
    name, w, idx, orc = case
    _say(f"[keys] {name}")
    got = as_u32(idx.hash(dev(w.points)))
    assert got.shape == orc.keys.shape
    bad = np.argwhere(got != orc.keys)
    assert bad.size == 0, f"{len(bad)} keys differ, first (table, point) {bad[:5].tolist()}"
    # queries through the same kernel
    qk = as_u32(idx.hash(dev(w.queries)))
    assert np.array_equal(qk, orc.query_keys(w.queries))


def test_tables_bit_exact(case):
    name, w, idx, orc = case
    _say(f"[tables] {name}")
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(idx.info["dir_bits"])
    assert np.array_equal(as_u32(tk), wk)
    assert np.array_equal(as_u32(ti), wi)


def test_directory(case):
    name, w, idx, orc = case
    db = idx.info["dir_bits"]
    dr = as_u32(idx.directory())
    bins = np.sort(orc.keys >> np.uint32(31 - db), axis=1)
    for T in range(orc.pr.L):
        want = np.searchsorted(bins[T], np.arange((1 << db) + 1), side="left")
        assert np.array_equal(dr[T], want.astype(np.uint32)), f"table {T}"


def test_queries_exact(case):
    """Def. 2 with delta = 0: every point within r, nothing else."""
    name, w, idx, orc = case
    _say(f"[query] {name} nq={w.nq}")
    bf = oracle.brute_force(w.points, w.d, w.queries, w.r)
    assert sum(len(x) for x in bf.ids) > 0
    got = csr_lists(*idx.query(dev(w.queries), w.r))
    assert_same_lists(got, bf.ids)
    s2 = orc.strategy2(w.queries, w.r)  # the paper's bitmap Strategy 2 agrees too
    assert_same_lists(s2.ids, bf.ids)


def test_collisions_counter(case):
    name, w, idx, orc = case
    s2 = orc.strategy2(w.queries, w.r)
    got = idx.collisions(dev(w.queries)).cpu().numpy()
    assert np.array_equal(got, s2.collisions)


def test_cost_counters(case):
    # Sec. 4.1's #Collisions and #Candidates (bitmap dedupe on the GPU) equal
    # the oracle's Strategy-2 counters
    name, w, idx, orc = case
    s2 = orc.strategy2(w.queries, w.r)
    coll, cand = (x.cpu().numpy() for x in idx.cost(dev(w.queries)))
    assert np.array_equal(coll, s2.collisions)
    assert np.array_equal(cand, s2.candidates)
    assert np.all(cand <= coll) and np.all(cand >= np.array([len(x) for x in s2.ids]))


def test_smaller_radii(case):
    name, w, idx, orc = case
    for rq in sorted({0, 1, w.r // 2, w.r - 1}):
        if rq < 0:
            continue
        bf = oracle.brute_force(w.points, w.d, w.queries, rq)
        assert_same_lists(csr_lists(*idx.query(dev(w.queries), rq)), bf.ids)


def test_plain_path_matches(case):
    name, w, idx, orc = case
    q = w.queries[:4]
    bf = oracle.brute_force(w.points, w.d, q, w.r)
    assert_same_lists(csr_lists(*idx.query_plain(dev(q), w.r)), bf.ids)


# --------------------------------------------------------------------------
# Edge cases
# --------------------------------------------------------------------------

def _p2_params(d, rp, cols):
    return dict(t=1, r_part=rp, part=np.zeros(d, np.int32), col=np.asarray(cols, np.int32),
                b=np.array([1 << c for c in range(d)], np.uint64))


def _str_point(s):
    w = np.zeros(1, np.uint64)
    for k, ch in enumerate(s):
        if ch == "1":
            w[0] |= np.uint64(1) << np.uint64(k)
    return w


def test_worked_example_2_1(golden):
    g = {ln.split()[0]: ln.split()[1:] for ln in golden("example_2_1.txt")}
    p = _p2_params(4, 2, [int(s, 2) for s in g["m"]])
    pts = np.stack([_str_point(g["x"][0]), _str_point(g["q"][0])])
    idx = fc.Index.with_params(dev(pts), 4, 2, p["t"], p["r_part"], p["part"], p["col"], p["b"])
    k = as_u32(idx.hash(dev(pts)))
    v = int(g["collide"][0])
    assert list(np.nonzero(k[:, 0] == k[:, 1])[0]) == [v - 1]
    assert int(k[v - 1, 0]) == sum(1 << i for i, ch in enumerate(g["collide"][1]) if ch == "1")
    idx.close()


def test_worked_example_3_1(golden):
    g = {ln.split()[0]: ln.split()[1:] for ln in golden("example_3_1.txt")}
    p = _p2_params(8, 2, list(range(8)))
    pts = np.stack([_str_point(g[k][0]) for k in ("x", "y", "q")])
    idx = fc.Index.with_params(dev(pts), 8, 2, p["t"], p["r_part"], p["part"], p["col"], p["b"])
    k = as_u32(idx.hash(dev(pts)))
    row = int(g["collide_x"][0])
    assert list(np.nonzero(k[:, 0] == k[:, 2])[0]) == [row - 1]
    assert not np.any(k[:, 1] == k[:, 2])
    # x (distance 2) is reported for q at r = 2, y (distance 3) is not
    offs, ids = idx.query(dev(pts[2:3]), 2)
    assert sorted(csr_lists(offs, ids)[0].tolist()) == [0, 2]
    idx.close()


def test_single_point_and_empty_batch():
    rng = np.random.default_rng(5)
    x = synth.uniform_points(1, 128, rng)
    idx = fc.Index(dev(x), 128, 4, seed=11)
    offs, ids = idx.query(dev(x), 4)
    assert csr_lists(offs, ids)[0].tolist() == [0]
    empty = torch.zeros((0, 2), dtype=torch.int64, device="cuda")
    offs, ids = idx.query(empty, 4)
    assert offs.shape[0] == 1 and int(offs[0]) == 0 and ids.numel() == 0
    idx.close()


def test_empty_super_bins():
    # few distinct points: most directory bins and whole top-8-bit super-bins
    # are empty in every table
    rng = np.random.default_rng(9)
    distinct = synth.uniform_points(3, 128, rng)
    pts = distinct[rng.integers(0, 3, size=5000)]
    pr = oracle.derive_params(128, 4, 79)
    orc = OracleIndex(pts, pr, with_tables=False)
    idx = fc.Index(dev(pts), 128, 4, seed=79)
    db = idx.info["dir_bits"]
    dr = as_u32(idx.directory())
    bins = np.sort(orc.keys >> np.uint32(31 - db), axis=1)
    for T in range(orc.pr.L):
        want = np.searchsorted(bins[T], np.arange((1 << db) + 1), side="left")
        assert np.array_equal(dr[T], want.astype(np.uint32)), f"table {T}"
    bf = oracle.brute_force(pts, 128, distinct, 4)
    assert_same_lists(csr_lists(*idx.query(dev(distinct), 4)), bf.ids)
    idx.close()


def test_duplicates_and_heavy_buckets():
    # many identical points: one bucket holds them in every table
    rng = np.random.default_rng(6)
    base = synth.uniform_points(1, 256, rng)
    pts = synth.uniform_points(3000, 256, rng)
    pts[::3] = base  # 1000 copies
    qs = np.vstack([base, synth.flip_distinct(base[0], 256, 3, rng)[None], pts[1:3]])
    pr = oracle.derive_params(256, 8, 77)
    orc = OracleIndex(pts, pr)
    idx = fc.Index(dev(pts), 256, 8, seed=77)
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(idx.info["dir_bits"])
    assert np.array_equal(as_u32(tk), wk) and np.array_equal(as_u32(ti), wi)
    bf = oracle.brute_force(pts, 256, qs, 8)
    assert len(bf.ids[0]) >= 1000
    assert_same_lists(csr_lists(*idx.query(dev(qs), 8)), bf.ids)
    assert np.array_equal(idx.collisions(dev(qs)).cpu().numpy(), orc.strategy2(qs, 8).collisions)
    idx.close()


@pytest.mark.parametrize("n", [20011, 300_007], ids=["8byte_entries", "6byte_entries"])
def test_all_points_identical(n):
    # every table is one bucket of n entries: the pass-2 workgroup walks it in
    # many chunks; at 300,007 points pass 1 hands pass 2 its 6-byte entries
    # (16-bit stored keys, pass 2 on super-bins)
    rng = np.random.default_rng(8)
    pts = np.repeat(synth.uniform_points(1, 64, rng), n, axis=0)
    pr = oracle.derive_params(64, 3, 78)
    orc = OracleIndex(pts, pr, with_tables=False)
    idx = fc.Index(dev(pts), 64, 3, seed=78)
    _say(f"[identical] n={n}")
    inf = idx.info
    assert idx.table_pointers()[4] == (2 if n > 2 ** 18 else 4)
    assert n < 2 ** 18 or inf["group_bits"] == 8
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(inf["dir_bits"])
    assert np.array_equal(as_u32(tk), wk) and np.array_equal(as_u32(ti), wi)
    offs, ids = idx.query(dev(pts[:1]), 3)
    assert np.array_equal(csr_lists(offs, ids)[0], np.arange(n, dtype=np.uint32))
    idx.close()


def test_radius_and_capacity_errors():
    w = synth.small(0.05)
    idx = fc.Index(dev(w.points), w.d, w.r, seed=3)
    with pytest.raises(fc.FclshError) as e:
        idx.query(dev(w.queries), w.r + 1)
    assert e.value.status == fc.FCLSH_ERADIUS
    bf = oracle.brute_force(w.points, w.d, w.queries, w.r)
    total = sum(len(x) for x in bf.ids)
    assert total > 2
    with pytest.raises(fc.FclshError) as e:
        idx.query(dev(w.queries), w.r, ids_capacity=total - 1)
    assert e.value.status == fc.FCLSH_ECAPACITY
    # exact capacity is enough
    offs, ids = idx.query(dev(w.queries), w.r, ids_capacity=total)
    assert_same_lists(csr_lists(offs, ids), bf.ids)
    idx.close()


@pytest.mark.parametrize("n,group_bits,mode,flags", [(300000, 8, "slot_all", 0), (300000, 8, "slot_only", 1),
                                                     (20000, 4, "full", 0)],
                         ids=["ordered_slots", "forced_fallbacks", "u32_keys"])
def test_rebuild_slot_only_with_large_bins(n, group_bits, mode, flags):
    """Here 60 copies of one point put one large bin in every table: at
    300000 points that is 1 of 256 groups, at 20000 points (32-bit stored
    keys, 16 super-bins merged per group) one group in 16.
    With 16-bit stored keys the group kernel places every group by per-wave
    slots and checks the id order, which holds, so every group stays on the
    slot branch and rebuilds take the slot-all form.  With the check forced
    to fail (a test flag), the first build's group with the large bin takes
    the ballot branch; a first build that sent at most 1 % of the groups off
    the slot branch makes the rebuilds take the slot-only form, which leaves
    those groups to the second kernel.  With 32-bit stored keys the group
    kernel ranks by slot and id walk, the bin's group takes the ballot
    branch, and the rebuilds keep the full form.  Every build equals the
    oracle."""
    rng = np.random.default_rng(41)
    d, r = 64, 4
    pts = synth.uniform_points(n, d, rng)
    pts[1:61] = pts[0]  # 61 equal points: equal keys in every table
    idx = fc.Index(dev(pts), d, r, seed=41, _test_flags=flags)
    orc = OracleIndex(pts, oracle.derive_params(d, r, 41), with_tables=False)
    db = idx.info["dir_bits"]
    assert idx.info["group_bits"] == group_bits
    wk, wi = orc.binned_tables(db)
    assert idx.build_mode == mode
    for build in ("first build", "rebuild", "second rebuild", "async rebuilds"):
        if build == "async rebuilds":
            # enqueued without host waits; the table reads follow on the stream
            idx.rebuild_async()
            idx.rebuild_async()
        elif build != "first build":
            idx.rebuild()
        _say(f"[slot-only n={n}] {build}")
        tk, ti = idx.tables()
        assert np.array_equal(as_u32(tk), wk), build
        assert np.array_equal(as_u32(ti), wi), build
        assert idx.build_mode == mode, build
    # a query enqueued right after an asynchronous rebuild sees the new tables
    qs = pts[[0, 100, 5000]]
    idx.rebuild_async()
    offs, ids = idx.query(dev(qs), r)
    assert_same_lists(csr_lists(offs, ids), oracle.brute_force(pts, d, qs, r).ids)
    idx.close()


@pytest.mark.parametrize("n,flags", [(300_000, 0), (300_000, 1), (8192 * 3 + 77, 0)],
                         ids=["many_tiles", "many_tiles_forced_walk", "ragged"])
def test_rebuild_slot_all(n, flags):
    """Uniform keys: the first build sends no group off the slot branch, so
    rebuilds take pass 2's slot branch for every group without checking bin
    sizes (with the test flag, every group's id-order check counts as
    failed and the id walk places it).  Tables and directory equal the
    oracle's after each of them, synchronous or not, and so do query
    answers."""
    rng = np.random.default_rng(43 + n % 5)
    d, r, seed = 64, 4, 43
    pts = synth.uniform_points(n, d, rng)
    idx = fc.Index(dev(pts), d, r, seed=seed, _test_flags=flags)
    pr = oracle.derive_params(d, r, seed)
    orc = OracleIndex(pts, pr, with_tables=False)
    db = idx.info["dir_bits"]
    wk, wi = orc.binned_tables(db)
    assert idx.build_mode == "slot_all"
    for build in ("rebuild", "second rebuild", "async rebuilds"):
        if build == "async rebuilds":
            idx.rebuild_async()
            idx.rebuild_async()
        else:
            idx.rebuild()
        _say(f"[slot-all] n={n} {build}")
        tk, ti = idx.tables()
        assert np.array_equal(as_u32(tk), wk), build
        assert np.array_equal(as_u32(ti), wi), build
        assert idx.build_mode == "slot_all", build
    dr = as_u32(idx.directory())
    for T in range(pr.L):
        bins = np.sort(orc.keys[T] >> np.uint32(31 - db))
        assert np.array_equal(dr[T], np.searchsorted(bins, np.arange((1 << db) + 1)).astype(np.uint32)), f"table {T}"
    qs = pts[rng.choice(n, size=5, replace=False)]
    idx.rebuild_async()
    assert_same_lists(csr_lists(*idx.query(dev(qs), r)), oracle.brute_force(pts, d, qs, r).ids)
    idx.close()


def test_finish_after_capacity_error():
    """A batch whose ids overflow the buffer is finished into a larger one
    from the pairs it already found (fclsh_query_batch_finish)."""
    import ctypes
    w = synth.learned_code(0.001)  # 10,000 points in 10 clusters: hundreds of neighbours per query
    idx = fc.Index(dev(w.points), w.d, w.r, seed=5)
    bf = oracle.brute_force(w.points, w.d, w.queries, w.r)
    total_want = sum(len(x) for x in bf.ids)
    assert total_want > 64 * len(w.queries)
    # the binding's first buffer (64 ids per query) overflows; it finishes
    offs, ids = idx.query(dev(w.queries), w.r)
    assert_same_lists(csr_lists(offs, ids), bf.ids)
    # through the C-ABI: too small, still too small, then large enough
    L = fc.lib()
    q = dev(w.queries)
    nq = q.shape[0]
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    offsets = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    small = torch.empty(8, dtype=torch.int32, device="cuda")
    total = ctypes.c_int64()
    st = L.fclsh_query_batch(idx._h, ctypes.c_void_p(q.data_ptr()), nq, w.r, stream,
                             ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(small.data_ptr()), 8,
                             ctypes.byref(total))
    assert st == fc.FCLSH_ECAPACITY and total.value == total_want
    st = L.fclsh_query_batch_finish(idx._h, stream, ctypes.c_void_p(offsets.data_ptr()),
                                    ctypes.c_void_p(small.data_ptr()), 8, ctypes.byref(total))
    assert st == fc.FCLSH_ECAPACITY
    other = torch.empty(nq + 1, dtype=torch.int64, device="cuda")
    big = torch.full((total_want,), -1, dtype=torch.int32, device="cuda")
    st = L.fclsh_query_batch_finish(idx._h, stream, ctypes.c_void_p(other.data_ptr()),
                                    ctypes.c_void_p(big.data_ptr()), total_want, ctypes.byref(total))
    assert st == fc.FCLSH_EINVAL
    assert idx.query_finish(offsets, big) == total_want
    assert_same_lists(csr_lists(offsets, big), bf.ids)
    # nothing is pending any more
    with pytest.raises(fc.FclshError) as e:
        idx.query_finish(offsets, big)
    assert e.value.status == fc.FCLSH_EINVAL
    # another call on the stream discards a pending batch
    st = L.fclsh_query_batch(idx._h, ctypes.c_void_p(q.data_ptr()), nq, w.r, stream,
                             ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(small.data_ptr()), 8,
                             ctypes.byref(total))
    assert st == fc.FCLSH_ECAPACITY
    idx.query(q[:1], w.r)
    with pytest.raises(fc.FclshError) as e:
        idx.query_finish(offsets, big)
    assert e.value.status == fc.FCLSH_EINVAL
    idx.close()


def test_bad_build_arguments():
    x = dev(synth.uniform_points(10, 64, np.random.default_rng(1)))
    with pytest.raises(fc.FclshError) as e:
        fc.Index(x, 64, 24, seed=1, partitions=1)  # 2^13 columns
    assert e.value.status == fc.FCLSH_EUNSUPPORTED
    with pytest.raises(fc.FclshError) as e:
        fc.Index(x, 64, 4, seed=1, mem_budget_bytes=1024)
    assert e.value.status == fc.FCLSH_ENOMEM


def test_largest_hadamard_order():
    # r' = 11: D = 4096 columns, 64 lanes per point
    w = synth.uniform_with_planted(300, 128, 11, 3, 4, 1109, "big_D")
    idx, pr = build(w, 3009, partitions=1)
    assert pr.D == 4096
    orc = OracleIndex(w.points, pr)
    assert np.array_equal(as_u32(idx.hash(dev(w.points))), orc.keys)
    bf = oracle.brute_force(w.points, w.d, w.queries, w.r)
    assert_same_lists(csr_lists(*idx.query(dev(w.queries), w.r)), bf.ids)
    idx.close()


def test_many_matches_per_bin_across_the_lane_limit():
    """Groups of 1, 8, 31, 32, 33 and 64 equal points: their keys are equal in
    every table, so a query at one of them finds that many matches in one bin
    of each table.  Bins of up to 32 entries are verified by one lane (the
    matches kept in a 32-bit mask, one verified per round), larger ones go
    to the spill queue; both sides of that limit are hit.  Queries at the
    points and at distance 1 and 2 equal the linear scan."""
    rng = np.random.default_rng(47)
    d, r, seed = 64, 4, 47
    base = synth.uniform_points(4000, d, rng)
    sizes = [1, 8, 31, 32, 33, 64]
    reps = synth.uniform_points(len(sizes), d, rng)
    pts = np.concatenate([base] + [np.repeat(reps[i:i + 1], k, axis=0) for i, k in enumerate(sizes)])
    pts = pts[rng.permutation(len(pts))]
    idx = fc.Index(dev(pts), d, r, seed=seed)
    qs = np.concatenate([reps] + [np.stack([synth.flip_distinct(x, d, dist, rng) for x in reps]) for dist in (1, 2)])
    # the queried bins straddle the lane limit
    db = idx.info["dir_bits"]
    qk = as_u32(idx.hash(dev(reps)))
    dr = as_u32(idx.directory())
    sizes_seen = set()
    for T in range(qk.shape[0]):
        b = qk[T] >> np.uint32(31 - db)
        sizes_seen.update((dr[T, b + 1] - dr[T, b]).tolist())
    assert min(sizes_seen) <= 32 < max(sizes_seen), sorted(sizes_seen)[:5]
    want = oracle.brute_force(pts, d, qs, r).ids
    assert_same_lists(csr_lists(*idx.query(dev(qs), r)), want)
    assert_same_lists(csr_lists(*idx.query_plain(dev(qs[:6]), r)), want[:6])
    idx.close()


@pytest.mark.parametrize("d,r,times", [(128, 2, 4), (128, 3, 3), (100, 2, 3), (64, 5, 2)],
                         ids=["r2x4", "r3x3", "general", "r5x2"])
def test_replication(d, r, times):
    """Alg. 1's replication: the family is drawn for times copies of every
    point (times * d coordinates, radius times * r, one part; Fig. 3's
    settings give L = 511, 1023, 2047).  The GPU hashes the points
    themselves, each copy of a bit being one more gather entry; its keys and
    tables equal the oracle's on the replicated points, and the answers
    (dedupe over all copies of a differing bit) equal the linear scan on the
    points."""
    seed = 3100 + 10 * r + times
    w = synth.uniform_with_planted(3000, d, r, 30, 6, seed, f"rep{times}")
    _say(f"[replication] d={d} r={r} x{times}")
    idx = fc.Index(dev(w.points), d, r, seed=seed, replicate=times)
    pr = oracle.derive_params(times * d, times * r, seed, override_t=1)
    assert idx.info["L"] == pr.L and idx.info["t"] == 1
    p = idx.params()
    assert np.array_equal(p["col"], pr.col) and np.array_equal(p["b"], pr.b)
    orc = OracleIndex(oracle.replicate(w.points, d, times), pr, with_tables=False)
    assert np.array_equal(as_u32(idx.hash(dev(w.points))), orc.keys)
    assert np.array_equal(as_u32(idx.hash(dev(w.queries))), oracle.keys(oracle.replicate(w.queries, d, times), pr))
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(idx.info["dir_bits"])
    assert np.array_equal(as_u32(tk), wk) and np.array_equal(as_u32(ti), wi)
    for rq in sorted({0, max(0, r - 1), r}):
        want = oracle.brute_force(w.points, d, w.queries, rq).ids
        assert_same_lists(csr_lists(*idx.query(dev(w.queries), rq)), want)
    want = oracle.brute_force(w.points, d, w.queries[:4], r).ids
    assert_same_lists(csr_lists(*idx.query_plain(dev(w.queries[:4]), r)), want)
    idx.close()


@pytest.mark.parametrize("d,r,t", [(31, 4, 0), (64, 4, 0), (100, 6, 0), (128, 10, 0)],
                         ids=["specific-boundary", "general", "specific", "two-parts"])
def test_exclude_column0(d, r, t):
    """The Sec. 3.3 variant whose map avoids column 0: the parameters, keys
    and tables equal the oracle's for the same draw, and the answers equal
    the linear scan."""
    seed = 3300 + d + r
    w = synth.uniform_with_planted(3000, d, r, 30, 6, seed, f"x0-{d}")
    _say(f"[exclude column 0] d={d} r={r}")
    idx = fc.Index(dev(w.points), d, r, seed=seed, partitions=t, exclude_column0=True)
    pr = oracle.derive_params(d, r, seed, override_t=t, exclude_column0=True)
    p = idx.params()
    assert np.array_equal(p["col"], pr.col) and np.array_equal(p["b"], pr.b) and p["col"].min() >= 1
    orc = OracleIndex(w.points, pr, with_tables=False)
    assert np.array_equal(as_u32(idx.hash(dev(w.points))), orc.keys)
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(idx.info["dir_bits"])
    assert np.array_equal(as_u32(tk), wk) and np.array_equal(as_u32(ti), wi)
    for rq in sorted({0, r}):
        want = oracle.brute_force(w.points, d, w.queries, rq).ids
        assert_same_lists(csr_lists(*idx.query(dev(w.queries), rq)), want)
    idx.close()


def test_rebuild_is_deterministic():
    w = synth.small(0.1)
    idx = fc.Index(dev(w.points), w.d, w.r, seed=5)
    tk0, ti0 = (as_u32(t) for t in idx.tables())
    idx.rebuild()
    tk1, ti1 = (as_u32(t) for t in idx.tables())
    assert np.array_equal(tk0, tk1) and np.array_equal(ti0, ti1)
    idx.close()


def test_timed_rebuild_reports_every_kernel():
    """The timed rebuild gives the same tables and a positive duration for
    each of its five kernels."""
    w = synth.small(0.1)
    idx = fc.Index(dev(w.points), w.d, w.r, seed=5)
    tk0, ti0 = (as_u32(t) for t in idx.tables())
    ms = idx.rebuild_timed()
    assert list(ms) == list(fc.Index.REBUILD_PHASES)
    assert all(v > 0 for v in ms.values()), ms
    tk1, ti1 = (as_u32(t) for t in idx.tables())
    assert np.array_equal(tk0, tk1) and np.array_equal(ti0, ti1)
    idx.close()


def test_split_pass_8byte_entries():
    """Above 2^25 points ids no longer fit the 6-byte entries, so the passes
    hand on 8-byte ones through the split (4 bits here).  33.6 million
    points of 32 bits, r = 2 (7 tables): the oracle checks the keys of
    sampled points; two whole tables are checked against the library's
    keys of every point (themselves pinned by the samples): grouped by bin,
    ids ascending in a bin, a permutation, the directory, each point under
    its own key; then sampled answers against the linear scan."""
    rng = np.random.default_rng(47)
    n, d, r, seed = (1 << 25) + 4099, 32, 2, 97
    pts = synth.uniform_points(n, d, rng)
    _say(f"[split8] n={n}")
    pts_d = dev(pts)
    idx = fc.Index(pts_d, d, r, seed=seed)
    inf = idx.info
    assert inf["group_bits"] == 12 and idx.table_pointers()[4] == 2
    pr = oracle.derive_params(d, r, seed)
    which = np.sort(rng.choice(n, size=64, replace=False))
    want = oracle.keys(pts, pr, which=which)
    keys = idx.hash(pts_d)
    assert np.array_equal(as_u32(keys[:, torch.from_numpy(which).cuda()]), want)
    db = inf["dir_bits"]
    dr_all = as_u32(idx.directory())
    for T in (0, pr.L - 1):
        _say(f"[split8] table {T}")
        tk, ti = (as_u32(x)[0] for x in idx.tables(T, T + 1))
        kt = as_u32(keys[T])
        bins = tk >> np.uint32(31 - db)
        assert np.all(np.diff(bins.astype(np.int64)) >= 0)
        same = np.diff(bins.astype(np.int64)) == 0
        assert np.all(np.diff(ti.astype(np.int64))[same] > 0)
        assert np.array_equal(np.sort(ti), np.arange(n, dtype=np.uint32))
        assert np.array_equal(tk, kt[ti])
        assert np.array_equal(dr_all[T], np.searchsorted(bins, np.arange((1 << db) + 1)).astype(np.uint32))
    del keys
    qs = pts[rng.choice(n, size=4, replace=False)]
    assert_same_lists(csr_lists(*idx.query(dev(qs), r)), oracle.brute_force(pts, d, qs, r).ids)
    idx.close()


@pytest.mark.parametrize("n,dup,split", [(1_200_000, False, 1), (1_200_000, True, 1), (4_500_000, False, 3)],
                         ids=["uniform", "heavy", "three_bits"])
def test_split_pass_for_large_n(n, dup, split):
    """Above about a million points the table build splits each super-bin
    by more key bits before the last pass.  Only 7 tables (d=64, r=2) keep
    the oracle quick: every table entry and the directory are compared.
    With 400,000 copies of one point, the heavy bins take the stable
    fallback, which then reorders the ids in place.  4.5 million points
    split by 3 bits (8 sub-digits, the split's 4096-entry chunks)."""
    rng = np.random.default_rng(40 + int(dup) + n % 7)
    d, r, seed = 64, 2, 95
    pts = synth.uniform_points(n, d, rng)
    if dup:
        pts[::3] = pts[0]
    _say(f"[split] n={n} dup={dup}")
    idx = fc.Index(dev(pts), d, r, seed=seed)
    inf = idx.info
    assert inf["group_bits"] == 8 + split
    pr = oracle.derive_params(d, r, seed)
    orc = OracleIndex(pts, pr, with_tables=False)
    assert np.array_equal(as_u32(idx.hash(dev(pts))), orc.keys)
    tk, ti = idx.tables()
    wk, wi = orc.binned_tables(inf["dir_bits"])
    assert np.array_equal(as_u32(tk), wk)
    assert np.array_equal(as_u32(ti), wi)
    # a rebuild in the form the first build's counters chose gives the same
    # tables (uniform keys: the slot-all form)
    mode = idx.build_mode
    assert dup or mode == "slot_all"
    _say(f"[split] rebuild ({mode})")
    idx.rebuild()
    tk, ti = idx.tables()
    assert np.array_equal(as_u32(tk), wk), mode
    assert np.array_equal(as_u32(ti), wi), mode
    db = inf["dir_bits"]
    dr = as_u32(idx.directory())
    for T in range(pr.L):
        bins = np.sort(orc.keys[T] >> np.uint32(31 - db))
        assert np.array_equal(dr[T], np.searchsorted(bins, np.arange((1 << db) + 1)).astype(np.uint32)), f"table {T}"
    # the queries see the same tables: a few sampled answers against the scan
    qs = pts[rng.choice(n, size=6, replace=False)]
    want = oracle.brute_force(pts, d, qs, r).ids
    assert_same_lists(csr_lists(*idx.query(dev(qs), r)), want)
    idx.close()
