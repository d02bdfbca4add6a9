"""GPU parity of the sparse path (points and queries given as rows of nonzero
coordinates): the parameters, every key of the O(nnz + L log L) hash kernel,
every table entry and every query answer against the CPU oracle
(oracle.keys_sparse, oracle.brute_force_sparse), the sparse keys against the
dense kernel's on the same points, and the edge cases (empty rows, an empty
batch, ragged sizes, every Hadamard order family, malformed rows, calls of
the wrong point format).  Full-size bag-of-words and user-rating shapes are
checked on sampled keys and on every answer of their 100 queries."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import as_u32, assert_same_lists, csr_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rows(ptr, cols):
    return fc.to_device_rows(ptr, cols)


def small_sparse(n, d, r, nq, mean, seed):
    return synth.sparse_planted(n, d, r, nq, mean, 1.0, 1.0, min(nq, 6), 4, seed=seed, name=f"sparse{d}")


CASES = {
    # name: (workload, index seed, partitions); D = 2^(floor(r/t)+1)
    "d8": (lambda: small_sparse(900, 3000, 2, 9, 20.0, 1201), 4001, 0),         # D = 8
    "d64": (lambda: small_sparse(1300, 20_000, 5, 11, 40.0, 1202), 4002, 0),    # D = 64
    "d1024": (lambda: small_sparse(800, 28_102, 9, 8, 60.0, 1203), 4003, 0),    # D = 1024
    "t2_d128": (lambda: small_sparse(2100, 140_214, 13, 12, 30.0, 1204), 4004, 0),  # 2 parts, D = 128
    "t3_d1024": (lambda: small_sparse(600, 28_102, 29, 8, 80.0, 1205), 4005, 3),   # 3 parts, D = 1024
    "d4096": (lambda: small_sparse(300, 9000, 11, 5, 25.0, 1206), 4006, 1),    # D = 4096, one part
}


@pytest.fixture(scope="module", params=sorted(CASES))
def case(request):
    make, seed, t = CASES[request.param]
    w = make()
    _say(f"[sparse build] {request.param} n={w.n} d={w.d} r={w.r} nnz={w.cols.size} seed={seed} t={t}")
    idx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, w.r, seed=seed, partitions=t)
    pr = oracle.derive_params(w.d, w.r, seed, override_t=t)
    yield request.param, w, idx, pr
    idx.close()


def test_params_agree(case):
    name, w, idx, pr = case
    inf = idx.info
    assert (inf["t"], inf["r_part"], inf["n"], inf["L"]) == (pr.t, pr.rpart, w.n, pr.L)
    p = idx.params()
    assert np.array_equal(p["part"], pr.part) and np.array_equal(p["col"], pr.col)
    assert np.array_equal(p["b"], pr.b)


def test_keys_and_tables_match_oracle(case):
    name, w, idx, pr = case
    _say(f"[sparse keys] {name}")
    want = oracle.keys_sparse(w.ptr, w.cols, pr)
    got = as_u32(idx.hash(*rows(w.ptr, w.cols)))
    assert np.array_equal(got, want), f"{name}: keys differ"
    # the index's tables hold the same keys: per table, bins of the top
    # dir_bits key bits in order, ids ascending inside a bin
    db = idx.info["dir_bits"]
    tk, ti = idx.tables()
    tk, ti = as_u32(tk), as_u32(ti)
    ids = np.arange(w.n, dtype=np.uint32)
    for T in range(0, pr.L, max(1, pr.L // 64)):
        order = np.lexsort((ids, want[T] >> np.uint32(31 - db)))
        assert np.array_equal(ti[T], ids[order]) and np.array_equal(tk[T], want[T][order]), f"{name}: table {T}"


def test_queries_match_linear_scan(case):
    name, w, idx, pr = case
    for rq in sorted({0, w.r // 2, w.r}):
        _say(f"[sparse query] {name} rq={rq}")
        got = csr_lists(*idx.query(*rows(w.qptr, w.qcols), rq))
        want = oracle.brute_force_sparse(w.ptr, w.cols, w.qptr, w.qcols, w.d, rq).ids
        assert_same_lists(got, want, what=f"{name} rq={rq}")
    # the planted neighbours were found
    got = csr_lists(*idx.query(*rows(w.qptr, w.qcols), w.r))
    for j, slots in enumerate(w.meta["planted"]):
        assert set(int(s) for s in slots) <= set(got[j].tolist())


def test_sparse_keys_equal_dense_kernel():
    # the same points as bit vectors through the dense kernel, same family
    w = small_sparse(1500, 2000, 9, 6, 30.0, 1207)
    sidx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, w.r, seed=4007)
    p, inf = sidx.params(), sidx.info
    didx = fc.Index.with_params(fc.to_device_words(w.dense_points()), w.d, w.r, inf["t"], inf["r_part"],
                                p["part"], p["col"], p["b"])
    assert np.array_equal(as_u32(sidx.hash(*rows(w.ptr, w.cols))),
                          as_u32(didx.hash(fc.to_device_words(w.dense_points()))))
    a = csr_lists(*sidx.query(*rows(w.qptr, w.qcols), w.r))
    b = csr_lists(*didx.query(fc.to_device_words(w.dense_queries()), w.r))
    assert_same_lists(a, b, what="sparse vs dense index")
    sidx.close()
    didx.close()


def test_empty_rows_and_empty_batch():
    d, r = 5000, 6
    rng = np.random.default_rng(1208)
    ptr, cols = synth.sparse_rows(700, d, 10.0, 1.0, 1.0, rng)
    # rows 0, 5 and the last are empty
    lists = [cols[ptr[i]:ptr[i + 1]] for i in range(700)]
    lists[0] = lists[5] = lists[-1] = np.zeros(0, np.int32)
    ptr = np.zeros(701, np.int64)
    ptr[1:] = np.cumsum([len(x) for x in lists])
    cols = np.concatenate(lists).astype(np.int32)
    idx = fc.SparseIndex(*rows(ptr, cols), d, r, seed=4008)
    pr = oracle.derive_params(d, r, 4008)
    keys = as_u32(idx.hash(*rows(ptr, cols)))
    assert np.array_equal(keys, oracle.keys_sparse(ptr, cols, pr))
    assert not keys[:, 0].any() and not keys[:, 5].any()
    # an empty query finds the empty rows and every row of at most r ones
    qp = np.array([0, 0], np.int64)
    got = csr_lists(*idx.query(*rows(qp, np.zeros(0, np.int32)), r))
    want = oracle.brute_force_sparse(ptr, cols, qp, np.zeros(0, np.int32), d, r).ids
    assert_same_lists(got, want, what="empty query")
    assert {0, 5, 699} <= set(got[0].tolist())
    offs, ids = idx.query(*rows(np.zeros(1, np.int64), np.zeros(0, np.int32)), r)
    assert offs.cpu().tolist() == [0] and ids.numel() == 0
    idx.close()


def _bad_rows():
    good_p = np.array([0, 2, 3], np.int64)
    return {
        "unsorted": (good_p, np.array([7, 3, 1], np.int32)),
        "repeat": (good_p, np.array([3, 3, 1], np.int32)),
        "col_out_of_range": (good_p, np.array([3, 9000, 1], np.int32)),
        "negative_col": (good_p, np.array([-1, 3, 1], np.int32)),
        "ptr_decreasing": (np.array([0, 3, 2], np.int64), np.array([1, 2, 3], np.int32)),
        "ptr_past_nnz": (np.array([0, 2, 5], np.int64), np.array([1, 2, 3], np.int32)),
    }


@pytest.mark.parametrize("kind", sorted(_bad_rows()))
def test_malformed_rows_rejected(kind):
    # rows are checked on the device before any kernel reads them as points;
    # query rows are checked within the batch and the kernels clamp them
    ptr, cols = _bad_rows()[kind]
    with pytest.raises(fc.FclshError) as e:
        fc.SparseIndex(*rows(ptr, cols), 8000, 4, seed=1)
    assert e.value.status == fc.FCLSH_EINVAL
    w = small_sparse(400, 8000, 4, 4, 12.0, 1209)
    idx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, w.r, seed=4009)
    with pytest.raises(fc.FclshError) as e:
        idx.query(*rows(ptr, cols), 4)
    assert e.value.status == fc.FCLSH_EINVAL
    # the index still answers well-formed batches afterwards
    got = csr_lists(*idx.query(*rows(w.qptr, w.qcols), 4))
    assert_same_lists(got, oracle.brute_force_sparse(w.ptr, w.cols, w.qptr, w.qcols, w.d, 4).ids)
    idx.close()


def test_wrong_format_calls_rejected():
    w = small_sparse(300, 3000, 3, 3, 10.0, 1210)
    sidx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, w.r, seed=4010)
    dq = fc.to_device_words(w.dense_queries())
    for call in (lambda: fc.Index.hash(sidx, dq),
                 lambda: fc.Index.query(sidx, dq, 3),
                 lambda: fc.Index.collisions(sidx, dq)):
        with pytest.raises(fc.FclshError) as e:
            call()
        assert e.value.status == fc.FCLSH_EINVAL
    didx = fc.Index(fc.to_device_words(w.dense_points()), w.d, w.r, seed=4010)
    with pytest.raises(fc.FclshError) as e:
        fc.SparseIndex.query(didx, *rows(w.qptr, w.qcols), 3)
    assert e.value.status == fc.FCLSH_EINVAL
    with pytest.raises(fc.FclshError) as e:
        fc.SparseIndex(*rows(w.ptr, w.cols), 600_000, 3)
    assert e.value.status == fc.FCLSH_EUNSUPPORTED
    sidx.close()
    didx.close()


_FULL = {}


def _full(name):
    # one draw of each full-size shape per module (the generator takes seconds)
    if name not in _FULL:
        _FULL[name] = synth.SPARSE_WORKLOADS[name](1.0)
    return _FULL[name]


@pytest.mark.parametrize("name,seed,r,t", [("enron_like", 4101, 29, 3), ("movielens_like", 4102, 13, 2),
                                           ("movielens_like", 4103, 7, 1)],
                         ids=["enron_like_r29", "movielens_like_r13", "movielens_like_r7"])
def test_full_size_sampled(name, seed, r, t):
    # the full bag-of-words / user-rating shapes (planted within the shape's
    # own radius): keys of sampled points against the oracle, every answer of
    # the 100 queries against the oracle's linear scan
    w = _full(name)
    _say(f"[sparse full] {w.name} n={w.n} d={w.d} nnz={w.cols.size} r={r} t={t}")
    idx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, r, seed=seed, partitions=t)
    pr = oracle.derive_params(w.d, r, seed, override_t=t)
    assert idx.info["L"] == pr.L
    keys = idx.hash(*rows(w.ptr, w.cols))
    rng = np.random.default_rng(seed)
    pick = np.unique(np.concatenate([rng.choice(w.n, 150, replace=False), [0, w.n - 1]]))
    sub_ptr = np.zeros(pick.size + 1, np.int64)
    sub_ptr[1:] = np.cumsum(w.ptr[pick + 1] - w.ptr[pick])
    sub_cols = np.concatenate([w.cols[w.ptr[i]:w.ptr[i + 1]] for i in pick])
    want = oracle.keys_sparse(sub_ptr, sub_cols, pr)
    got = as_u32(keys[:, torch.from_numpy(pick).to(keys.device)])
    assert np.array_equal(got, want)
    del keys
    _say(f"[sparse full] {w.name} queries r={r}")
    got = csr_lists(*idx.query(*rows(w.qptr, w.qcols), r))
    want = oracle.brute_force_sparse(w.ptr, w.cols, w.qptr, w.qcols, w.d, r).ids
    assert_same_lists(got, want, what=w.name)
    if r >= w.r:
        for j, slots in enumerate(w.meta["planted"]):
            assert set(int(s) for s in slots) <= set(got[j].tolist())
    idx.close()


def test_bitmap_and_first_table_dedupe_agree():
    # a batch whose per-query point bitmaps would exceed 1 GiB (40,000
    # queries x 234,834 points) uses the first-shared-table rule; the same
    # queries in a batch of 100 use the bitmaps: both answer alike, and the
    # small batch equals the oracle
    w = _full("movielens_like")
    r = 7
    idx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, r, seed=4103, partitions=1)
    small = csr_lists(*idx.query(*rows(w.qptr, w.qcols), r))
    assert_same_lists(small, oracle.brute_force_sparse(w.ptr, w.cols, w.qptr, w.qcols, w.d, r).ids)
    reps = 400
    sizes = np.diff(w.qptr)
    bptr = np.concatenate([[0], np.cumsum(np.tile(sizes, reps))]).astype(np.int64)
    _say(f"[sparse dedupe] {reps * w.nq} queries")
    big = csr_lists(*idx.query(*rows(bptr, np.tile(w.qcols, reps)), r))
    assert len(big) == reps * w.nq
    for k in range(0, reps * w.nq, 997):
        assert np.array_equal(big[k], small[k % w.nq]), k
    idx.close()


def test_cost_counters_match_oracle():
    # Sec. 4.1's #Collisions and #Candidates of query rows against the
    # oracle's Strategy 2 on the same points as bit vectors
    w = small_sparse(700, 3000, 6, 9, 20.0, 1211)
    idx = fc.SparseIndex(*rows(w.ptr, w.cols), w.d, w.r, seed=4011)
    pr = oracle.derive_params(w.d, w.r, 4011)
    pts, qs = w.dense_points(), w.dense_queries()
    keys = oracle.keys(pts, pr)
    tk, ti = oracle.tables(keys)
    want = oracle.query_batch(pts, w.d, tk, ti, qs, oracle.keys(qs, pr), w.r)
    coll, cand = idx.cost(*rows(w.qptr, w.qcols))
    assert np.array_equal(coll.cpu().numpy(), want.collisions)
    assert np.array_equal(cand.cpu().numpy(), want.candidates)
    with pytest.raises(fc.FclshError) as e:
        idx.cost(*rows(np.array([0, 2], np.int64), np.array([5, 1], np.int32)))
    assert e.value.status == fc.FCLSH_EINVAL
    idx.close()
