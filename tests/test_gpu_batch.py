"""GPU tests of the batched query machinery: per-query radii, the spill queue
for large buckets, the synchronisation-free path and its HIP-graph replays,
the autotuner, overflow reporting, and equality of every answer alone and in
a mixed batch.  Expected answers come from the CPU oracle's linear scan."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import assert_same_lists, csr_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return fc.to_device_words(a)


def brute_mixed(points, d, queries, radii):
    out = []
    for i in range(queries.shape[0]):
        out.append(oracle.brute_force(points, d, queries[i:i + 1], int(radii[i])).ids[0])
    return out


@pytest.fixture(scope="module")
def served():
    # shape of the served index A (r = 10, two parts), scaled down; per-query
    # radii with neighbours planted inside each query's own radius
    rng = np.random.default_rng(4)
    nq = 48
    radii = rng.integers(0, 11, size=nq).astype(np.int32)
    w = synth.uniform_with_planted(6000, 256, 10, nq, 5, 1205, "served_small", query_radius=radii)
    _say(f"[build] served_small n={w.n}")
    idx = fc.Index(dev(w.points), w.d, w.r, seed=3105)
    yield w, idx
    idx.close()


def test_mixed_radii(served):
    w, idx = served
    want = brute_mixed(w.points, w.d, w.queries, w.query_radius)
    got = csr_lists(*idx.query_radii(dev(w.queries), torch.from_numpy(w.query_radius)))
    assert_same_lists(got, want)


def test_alone_equals_in_mix(served):
    """Every query's answer is the same alone and inside a mixed batch."""
    w, idx = served
    rad = torch.from_numpy(w.query_radius)
    mix = csr_lists(*idx.query_radii(dev(w.queries), rad))
    for i in range(0, w.nq, 5):
        alone = csr_lists(*idx.query_radii(dev(w.queries[i:i + 1]), rad[i:i + 1]))[0]
        assert np.array_equal(alone, mix[i]), f"query {i}"
        plain = csr_lists(*idx.query_plain(dev(w.queries[i:i + 1]), int(w.query_radius[i])))[0]
        assert np.array_equal(plain, mix[i])


def test_spill_queue_for_large_buckets():
    # 1500 copies of one point: its bucket in every table holds >= 1500 entries;
    # with 64-entry tiles each such bucket is cut into ~23 spill chunks
    rng = np.random.default_rng(10)
    base = synth.uniform_points(1, 128, rng)
    pts = synth.uniform_points(4500, 128, rng)
    pts[::3] = base
    qs = np.vstack([base, synth.flip_distinct(base[0], 128, 2, rng)[None], pts[1:4]])
    idx = fc.Index(dev(pts), 128, 4, seed=91)
    want = oracle.brute_force(pts, 128, qs, 4).ids
    for tile, bpc in [(64, 1), (64, 8), (256, 4), (4096, 2)]:
        for schedule in ("static", "claim"):
            idx.set_tuning(tile, bpc)
            idx.set_schedule(schedule)
            assert idx.get_tuning() == {"tile": tile, "blocks_per_cu": bpc, "schedule": schedule}
            assert_same_lists(csr_lists(*idx.query(dev(qs), 4)), want)
    with pytest.raises(fc.FclshError):
        fc._check(fc.lib().fclsh_index_set_schedule(idx._h, 2))
    idx.close()


@pytest.mark.parametrize("schedule", ["static", "claim"])
def test_async_and_graph_replays(served, schedule):
    # the claim schedule's counters are cleared by the batch's first kernel,
    # so every replay starts from zero
    w, idx = served
    idx.set_schedule(schedule)
    nq = 16
    r = 8
    stream = torch.cuda.Stream()
    total_cap = 4096
    qbuf = torch.empty((nq, fc.words(w.d)), dtype=torch.int64, device="cuda")
    offsets = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.zeros(total_cap, dtype=torch.int32, device="cuda")
    result = torch.zeros(2, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream):
        idx.reserve(nq, pair_capacity=1 << 15, spill_capacity=1 << 12, stream=stream)
        # direct asynchronous call
        qbuf.copy_(dev(w.queries[:nq]))
        idx.query_async(qbuf, r, offsets, ids, result, stream=stream)
    stream.synchronize()
    want = oracle.brute_force(w.points, w.d, w.queries[:nq], r).ids
    assert int(result[1]) == 0 and int(result[0]) == sum(len(x) for x in want)
    assert_same_lists(csr_lists(offsets, ids[:int(result[0])]), want)
    # graph: capture once, replay on new query contents, with eager work and
    # synchronisations between the replays
    with torch.cuda.stream(stream):
        g = idx.query_graph(qbuf, r, offsets, ids, result, stream=stream)
    stream.synchronize()
    for rep, start in enumerate([0, 16, 32, 0]):
        batch = w.queries[start:start + nq]
        with torch.cuda.stream(stream):
            qbuf.copy_(dev(batch))
            ids.fill_(-1)
            g.launch(stream=stream)
        stream.synchronize()
        want = oracle.brute_force(w.points, w.d, batch, r).ids
        assert int(result[1]) == 0, f"replay {rep} status {int(result[1])}"
        assert_same_lists(csr_lists(offsets, ids[:int(result[0])]), want)
        _ = torch.randn(1000, device="cuda").sum().item()  # unrelated eager work between replays
    g.close()
    idx.set_schedule("static")


def test_async_reports_overflow(served):
    w, idx = served
    stream = torch.cuda.Stream()
    nq = 8
    q = dev(w.queries[:nq])
    offsets = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.zeros(1, dtype=torch.int32, device="cuda")
    result = torch.zeros(2, dtype=torch.int64, device="cuda")
    want = oracle.brute_force(w.points, w.d, w.queries[:nq], 10).ids
    total = sum(len(x) for x in want)
    assert total > 1
    with torch.cuda.stream(stream):
        idx.reserve(nq, pair_capacity=1 << 14, spill_capacity=1 << 12, stream=stream)
        idx.query_async(q, 10, offsets, ids, result, stream=stream)
    stream.synchronize()
    assert int(result[0]) == total and int(result[1]) & fc.QUERY_IDS_OVERFLOW
    assert int(offsets[-1]) == total
    # a pair buffer smaller than the answer is reported, not overrun (a fresh
    # stream has a fresh workspace: reserving only ever grows one)
    ids = torch.zeros(total, dtype=torch.int32, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        idx.reserve(nq, pair_capacity=1, spill_capacity=1 << 12, stream=stream)
        idx.query_async(q, 10, offsets, ids, result, stream=stream)
    stream.synchronize()
    assert int(result[1]) & fc.QUERY_PAIR_OVERFLOW
    # the synchronous path grows its buffers and answers
    assert_same_lists(csr_lists(*idx.query(q, 10, stream=stream)), want)


def test_autotune_keeps_answers(served):
    w, idx = served
    res = idx.autotune(dev(w.queries), 10)
    assert res["tile"] in (64, 128, 256, 512, 1024, 4096) and 1 <= res["blocks_per_cu"] <= 16
    assert res["ms"] > 0
    assert idx.get_tuning() == {"tile": res["tile"], "blocks_per_cu": res["blocks_per_cu"],
                                "schedule": res["schedule"]}
    want = oracle.brute_force(w.points, w.d, w.queries, 10).ids
    assert_same_lists(csr_lists(*idx.query(dev(w.queries), 10)), want)


def test_large_result_segment_sort():
    # one query whose answer (> 4096 ids) takes the long-segment sort
    rng = np.random.default_rng(12)
    base = synth.uniform_points(1, 64, rng)
    pts = synth.uniform_points(9000, 64, rng)
    pts[::2] = base
    idx = fc.Index(dev(pts), 64, 3, seed=93)
    want = oracle.brute_force(pts, 64, base, 3).ids
    assert len(want[0]) > 4096
    assert_same_lists(csr_lists(*idx.query(dev(base), 3)), want)
    idx.close()


def test_long_segments_over_several_bitmap_passes():
    # two queries with answers far over 4096 ids spread over ids above 2^21
    # (the long-segment sort marks 2^20 ids per pass), between queries with
    # short and empty answers, and the async path with the same buffers
    rng = np.random.default_rng(13)
    bases = synth.uniform_points(2, 64, rng)
    pts = synth.uniform_points(2_500_000, 64, rng)
    pts[5::97] = bases[0]
    pts[11::131] = bases[1]
    qs = np.concatenate([synth.uniform_points(1, 64, rng), bases[:1], pts[7:8], bases[1:2], pts[123:124]])
    idx = fc.Index(dev(pts), 64, 3, seed=94)
    want = oracle.brute_force(pts, 64, qs, 3).ids
    assert len(want[1]) > 20_000 and len(want[3]) > 15_000 and int(want[1][-1]) > 2 ** 21
    assert_same_lists(csr_lists(*idx.query(dev(qs), 3)), want)
    total = sum(len(x) for x in want)
    offs = torch.empty(len(qs) + 1, dtype=torch.int64, device="cuda")
    ids = torch.empty(total, dtype=torch.int32, device="cuda")
    res = torch.zeros(2, dtype=torch.int64, device="cuda")
    idx.reserve(len(qs), pair_capacity=2 * total)
    for _ in range(2):
        ids.zero_()
        idx.query_async(dev(qs), 3, offs, ids, res)
        torch.cuda.synchronize()
        assert res.cpu().tolist() == [total, 0]
        assert_same_lists(csr_lists(offs, ids), want)
    idx.close()


def _heavy_index():
    # 1500 copies of one point: every table holds a bucket of >= 1500 entries
    rng = np.random.default_rng(10)
    base = synth.uniform_points(1, 128, rng)
    pts = synth.uniform_points(4500, 128, rng)
    pts[::3] = base
    return base, pts, fc.Index(dev(pts), 128, 4, seed=91)


def test_sync_path_grows_overflowing_buffers():
    """100 copies of the heavy query: with 64-entry tiles the first run needs
    more spill chunks (~23 per bucket, 31 tables) and more pairs than the
    first sizing holds; the synchronous path grows both and answers exactly."""
    base, pts, idx = _heavy_index()
    rng = np.random.default_rng(13)
    qs = np.vstack([np.repeat(base, 100, axis=0), synth.uniform_points(4, 128, rng)])
    want = oracle.brute_force(pts, 128, qs, 4).ids
    assert sum(len(x) for x in want) > 1 << 17
    idx.set_tuning(64, 2)
    stream = torch.cuda.Stream()
    _say("[batch] heavy queries, 64-entry tiles, fresh workspace")
    with torch.cuda.stream(stream):
        got = csr_lists(*idx.query(dev(qs), 4, stream=stream))
    assert_same_lists(got, want)
    # the asynchronous path on a workspace reserved too small reports it
    stream2 = torch.cuda.Stream()
    nq = qs.shape[0]
    offsets = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.zeros(1 << 18, dtype=torch.int32, device="cuda")
    result = torch.zeros(2, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream2):
        idx.reserve(nq, pair_capacity=1 << 18, spill_capacity=64, stream=stream2)
        idx.query_async(dev(qs), 4, offsets, ids, result, stream=stream2)
    stream2.synchronize()
    assert int(result[1]) & fc.QUERY_SPILL_OVERFLOW
    idx.close()


def test_autotune_with_heavy_buckets():
    """Shapes whose spill queue overflows the first sizing are run complete
    (the workspace grows) before they are timed; the chosen shape answers
    exactly."""
    base, pts, idx = _heavy_index()
    rng = np.random.default_rng(14)
    qs = np.vstack([np.repeat(base, 40, axis=0), synth.flip_distinct(base[0], 128, 3, rng)[None],
                    synth.uniform_points(8, 128, rng)])
    want = oracle.brute_force(pts, 128, qs, 4).ids
    _say("[batch] autotune over heavy buckets")
    res = idx.autotune(dev(qs), 4)
    assert res["ms"] > 0 and idx.get_tuning() == {"tile": res["tile"], "blocks_per_cu": res["blocks_per_cu"],
                                                  "schedule": res["schedule"]}
    assert_same_lists(csr_lists(*idx.query(dev(qs), 4)), want)
    idx.close()


def test_graph_owns_its_workspace_and_keeps_the_index():
    """A captured graph keeps its own workspace: a larger batch on the same
    stream (which grows the stream's workspace) does not disturb its replays.
    Releasing the index while the graph lives leaves the graph working and
    makes later calls on the index fail; the graph's free releases it."""
    w = synth.small(0.3)
    r = w.r
    _say(f"[graph] n={w.n} d={w.d} r={r}")
    idx = fc.Index(dev(w.points), w.d, r, seed=5)
    nq = 8
    stream = torch.cuda.Stream()
    qbuf = torch.empty((nq, fc.words(w.d)), dtype=torch.int64, device="cuda")
    offsets = torch.zeros(nq + 1, dtype=torch.int64, device="cuda")
    ids = torch.zeros(4096, dtype=torch.int32, device="cuda")
    result = torch.zeros(2, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream):
        idx.reserve(nq, pair_capacity=1 << 12, spill_capacity=1 << 10, stream=stream)
        qbuf.copy_(dev(w.queries[:nq]))
        g = idx.query_graph(qbuf, r, offsets, ids, result, stream=stream)
    stream.synchronize()
    before = idx.memory()["workspace_bytes"]
    # a much larger batch on the same stream grows the stream's workspace
    big = np.concatenate([w.queries] * 8)
    with torch.cuda.stream(stream):
        idx.query(dev(big), r, stream=stream)
    stream.synchronize()
    assert idx.memory()["workspace_bytes"] > before
    want = oracle.brute_force(w.points, w.d, w.queries[:nq], r).ids
    for rep in range(2):
        with torch.cuda.stream(stream):
            ids.fill_(-1)
            g.launch(stream=stream)
        stream.synchronize()
        assert int(result[1]) == 0
        assert_same_lists(csr_lists(offsets, ids[:int(result[0])]), want)
    raw = fc.ctypes.c_void_p(idx._h.value)
    idx.close()  # the graph still holds the tables
    # the released handle refuses calls (it stays allocated while the graph lives)
    L = fc.ctypes.c_int32()
    st = fc.lib().fclsh_index_info(raw, None, None, None, None, None, fc.ctypes.byref(L), None, None)
    assert st == fc.FCLSH_EINVAL
    with torch.cuda.stream(stream):
        qbuf.copy_(dev(w.queries[nq:2 * nq]))
        ids.fill_(-1)
        g.launch(stream=stream)
    stream.synchronize()
    want = oracle.brute_force(w.points, w.d, w.queries[nq:2 * nq], r).ids
    assert_same_lists(csr_lists(offsets, ids[:int(result[0])]), want)
    g.close()


def test_index_memory_report():
    """Resident bytes of a served index: the point copy, the tables and the
    directory (plus a few KB of hash parameters); the build scratch is gone
    after the build unless it was asked to stay, and a rebuild keeps it."""
    w = synth.small(0.5)
    _say(f"[memory] n={w.n} d={w.d} r={w.r}")
    idx = fc.Index(dev(w.points), w.d, w.r, seed=6)
    inf = idx.info
    L, n = inf["L"], inf["n"]
    key_bytes = idx.table_pointers()[4]
    assert key_bytes == (2 if 31 - inf["dir_bits"] <= 16 else 4)
    tables = (4 + key_bytes) * L * n
    points = 8 * fc.words(w.d) * n
    directory = 4 * L * ((1 << inf["dir_bits"]) + 1)
    m = idx.memory()
    assert m["build_scratch_bytes"] == 0
    assert tables + points + directory <= m["index_bytes"] <= tables + points + directory + (1 << 20)
    idx.rebuild()
    assert idx.memory()["build_scratch_bytes"] >= 3 * 4 * L * n
    idx.close()
    kept = fc.Index(dev(w.points), w.d, w.r, seed=6, keep_build_scratch=True)
    assert kept.memory()["build_scratch_bytes"] >= 3 * 4 * L * n
    kept.close()
    # a large index stores the key bits below its bin, 16 of them
    big = synth.uniform_points(200_000, 64, np.random.default_rng(7))
    idx = fc.Index(dev(big), 64, 3, seed=8)
    inf = idx.info
    assert inf["dir_bits"] >= 15 and idx.table_pointers()[4] == 2
    L, n = inf["L"], inf["n"]
    directory = 4 * L * ((1 << inf["dir_bits"]) + 1)
    tables, points = 6 * L * n, 8 * n
    m = idx.memory()
    assert tables + points + directory <= m["index_bytes"] <= tables + points + directory + (1 << 20)
    idx.close()
