"""GPU tests of the pieces the Sec. 4.3 study runs on: the library's linear
scan (the ground truth recall is measured against) equals the oracle's, and
on the paper's synthetic sets (points around each query at distances spread
over 1..128) fcLSH reports exactly the linear scan's neighbours (recall 1)
with #Collisions / #Candidates equal to the oracle's Strategy 2, without
pre-processing, with replication and with two parts."""
import sys

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import OracleIndex, assert_same_lists, csr_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("n,d,nq,r", [(5000, 128, 37, 0), (5000, 128, 37, 3), (4097, 200, 21, 20),
                                      (8193, 64, 9, 6), (1, 64, 3, 64), (300, 1024, 5, 480)])
def test_linear_scan_matches_oracle(n, d, nq, r):
    _say(f"[linear] n={n} d={d} nq={nq} r={r}")
    rng = np.random.default_rng(n + d + r)
    pts = synth.uniform_points(n, d, rng)
    qs = np.concatenate([synth.uniform_points(nq - min(nq, 2), d, rng), pts[:min(nq, 2)]])
    got = csr_lists(*fc.linear_scan(fc.to_device_words(pts), d, fc.to_device_words(qs), r))
    want = oracle.brute_force(pts, d, qs, r).ids
    assert_same_lists(got, want)


def test_linear_scan_empty_batch():
    pts = synth.uniform_points(100, 64, np.random.default_rng(1))
    offs, ids = fc.linear_scan(fc.to_device_words(pts), 64, torch.zeros((0, 1), dtype=torch.int64,
                                                                          device="cuda"), 3)
    assert offs.cpu().tolist() == [0] and ids.numel() == 0


@pytest.mark.parametrize("r,copies,parts", [(6, 0, 0), (2, 4, 0), (3, 2, 0), (10, 0, 2)])
def test_study_settings_exact_with_oracle_counters(r, copies, parts):
    w = synth.hamming_balls(3000, 128, 10, seed=77 + r)
    _say(f"[study] n={w.n} r={r} copies={copies} parts={parts}")
    pts, qs = fc.to_device_words(w.points), fc.to_device_words(w.queries)
    idx = fc.Index(pts, 128, r, seed=9, replicate=copies, partitions=parts)
    got = csr_lists(*idx.query(qs, r))
    truth = csr_lists(*fc.linear_scan(pts, 128, qs, r))
    assert_same_lists(got, truth)  # recall 1 and nothing outside the radius
    assert sum(len(t) for t in truth) > 0
    # Strategy 2's counters from the oracle on the same family
    # (with k copies: the family of the replicated points at radius k*r)
    k = max(1, copies)
    rep = (lambda x: oracle.replicate(x, 128, k)) if k > 1 else (lambda x: x)
    pr = oracle.derive_params(k * 128, k * r, 9, override_t=1 if k > 1 else parts)
    orc = OracleIndex(rep(w.points), pr)
    s2 = orc.strategy2(rep(w.queries), k * r)
    coll, cand = (x.cpu().numpy() for x in idx.cost(qs))
    assert np.array_equal(coll, s2.collisions)
    assert np.array_equal(cand, s2.candidates)
    idx.close()
