"""CPU checks of the seeded input generators (they hold no method
arithmetic; these only confirm each recipe draws what its docstring says)."""
import numpy as np

import synth


def _popcount_rows(x):
    return np.array([sum(bin(int(v)).count("1") for v in row) for row in x])


def test_hamming_balls_distances():
    w = synth.hamming_balls(2000, 128, 20, seed=3)
    owner = w.meta["owner"]
    assert np.array_equal(owner, np.arange(2000) % 20)
    dist = _popcount_rows(w.points ^ w.queries[owner])
    assert np.array_equal(dist, w.meta["flips"])
    assert dist.min() >= 1 and dist.max() <= 128
    # spread over the whole range (uniform draws)
    assert np.histogram(dist, bins=4, range=(1, 129))[0].min() > 300


def test_hamming_balls_is_seeded_and_masks_pad_bits():
    a = synth.hamming_balls(300, 100, 7, seed=5)
    b = synth.hamming_balls(300, 100, 7, seed=5)
    assert np.array_equal(a.points, b.points) and np.array_equal(a.queries, b.queries)
    assert not (a.points[:, 1] >> np.uint64(36)).any()  # bits 100..127 stay clear


def test_uniform_with_planted_distances():
    w = synth.uniform_with_planted(3000, 256, 8, 30, 5, seed=7)
    planted = w.meta["planted"]
    for j in range(30):
        dist = _popcount_rows(w.points[planted[j]] ^ w.queries[j])
        assert dist.max() <= 8


def test_sparse_rows_valid_csr():
    rng = np.random.default_rng(5)
    ptr, cols = synth.sparse_rows(500, 3000, 40.0, 1.0, 1.0, rng)
    assert ptr[0] == 0 and ptr[-1] == cols.size and np.all(np.diff(ptr) >= 1)
    for i in range(500):
        row = cols[ptr[i]:ptr[i + 1]]
        assert np.all(np.diff(row) > 0) and row.min() >= 0 and row.max() < 3000
    assert 30 < np.diff(ptr).mean() < 50


def test_sparse_planted_neighbours_within_radius():
    w = synth.enron_like(0.02, r=9)
    assert w.nq >= 8 and w.d == 28_102
    for j, slots in enumerate(w.meta["planted"]):
        q = set(w.qcols[w.qptr[j]:w.qptr[j + 1]].tolist())
        for s in slots:
            x = set(w.cols[w.ptr[s]:w.ptr[s + 1]].tolist())
            assert len(q ^ x) <= 9
    dense = w.dense_points()
    assert dense.shape == (w.n, (w.d + 63) // 64)
    assert int(sum(bin(int(v)).count("1") for v in dense[3])) == w.ptr[4] - w.ptr[3]
