"""GPU test of the continuous-batching request loop: requests of mixed
index, radius and size arrive while earlier ones are on the GPU; every answer
must equal the oracle's linear scan and the answer of the same request sent
alone."""
import sys
import time

import numpy as np
import pytest

import oracle
import synth
from tests._helpers import assert_same_lists, csr_lists

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1602_02620_amd as fc  # noqa: E402
from paper_1602_02620_amd.serve import Server, poisson_trace  # noqa: E402


def test_served_requests_exact_alone_and_in_mix():
    print("[serve] building two indexes", flush=True)
    a = synth.uniform_with_planted(5000, 256, 10, 40, 5, 1305, "A")
    b = synth.uniform_with_planted(1500, 1024, 20, 20, 5, 1306, "B")
    ia = fc.Index(fc.to_device_words(a.points), 256, 10, seed=3205)
    ib = fc.Index(fc.to_device_words(b.points), 1024, 20, seed=3206)
    srv = Server({"A": ia, "B": ib}, max_batch=256, streams=3, mem_budget=1 << 30, ids_per_query=4)
    # admission counted what is really resident: both indexes and every
    # workspace the slots reserved (plus the slots' own small buffers)
    held = sum(ix.memory()["index_bytes"] + ix.memory()["workspace_bytes"] for ix in (ia, ib))
    assert held <= srv.resident_bytes <= held + (8 << 20)
    rng = np.random.default_rng(21)
    reqs = []
    arrivals = poisson_trace(2000.0, 0.03, rng)
    t0 = time.perf_counter()
    for k, ta in enumerate(arrivals):
        while time.perf_counter() - t0 < ta:
            pass
        w = a if rng.random() < 0.6 else b
        name = "A" if w is a else "B"
        m = int(rng.integers(1, 33))
        rows = rng.integers(0, w.nq, size=m)
        rad = int(rng.integers(0, w.r + 1))
        reqs.append((name, w, w.queries[rows], rad, srv.submit(name, w.queries[rows], rad)))
    print(f"[serve] {len(reqs)} requests submitted", flush=True)
    results = [f.result(timeout=120) for *_, f in reqs]
    srv.close()
    st = srv.stats()
    assert st["requests"] == len(reqs) and st["p99_ms"] is not None
    assert st["batches"] < len(reqs)  # requests were batched together
    for (name, w, q, rad, _), got in zip(reqs, results):
        want = oracle.brute_force(w.points, w.d, q, rad).ids
        assert_same_lists(got, want, what=f"request on {name} r={rad}")
        ix = ia if name == "A" else ib
        alone = csr_lists(*ix.query(fc.to_device_words(q), rad))
        assert_same_lists(got, alone, what="alone vs mix")
    print(f"[serve] ok {st}", flush=True)
    # a budget below the indexes' own bytes is refused
    with pytest.raises(ValueError):
        Server({"A": ia, "B": ib}, max_batch=256, streams=1, mem_budget=ia.memory()["index_bytes"])
    ia.close()
    ib.close()
