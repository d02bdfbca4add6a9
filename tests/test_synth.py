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
