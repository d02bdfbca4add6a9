"""Benchmark of the Fast CoveringLSH hot path on one MI355X.

A step is one pass of the whole hot path over the mid workload (n = 1,000,000
uniform 256-bit points, r = 8, L = 511 tables; 1,000 queries with 10 planted
neighbours each): hash every point into its L keys (Alg. 2), bucket the keys
into the L tables, and answer the query batch exactly (Strategy 2).  Inputs
are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is points per second through the whole step;
the breakdown (hash-only rate, keys/s, bucketing, queries/s, batched vs plain
per-query latency) and the roofline of the dominant kernel ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
METRIC = "points hashed/s (xL keys), queries/s at 100% recall, p99 latency vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mid", choices=["mid", "small", "learned_code", "batched"])
    ap.add_argument("--seed", type=int, default=3002)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="rough CPU budget of the oracle leg")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--plain-queries", type=int, default=200)
    ap.add_argument("--kernel-only", choices=["hash", "build"], default=None,
                    help="profiling aid: launch only this part (plus a plain copy of known size "
                         "for counter calibration) --kernel-reps times")
    return ap.parse_args()


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q)) if len(a) else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    import torch

    import paper_1602_02620_amd as fc
    import synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda", 0)
    w = synth.WORKLOADS[args.workload]()
    n, d, r, nq = w.n, w.d, w.r, w.nq
    W = fc.words(d)
    pts = fc.to_device_words(w.points, dev)
    qs = fc.to_device_words(w.queries, dev)
    stream = torch.cuda.current_stream()

    idx = fc.Index(pts, d, r, seed=args.seed)
    info = idx.info
    L = info["L"]
    if args.kernel_only:
        kernel_only(args, idx, pts, n, L, dev, torch)
        idx.close()
        return

    def step():
        idx.rebuild()
        return idx.query(qs, r)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        offs, ids = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) * 1e3 / args.steps
    total_ids = int(offs[-1].item())

    # ---- per-phase timing with HIP events on the stream the kernels run on
    def ev_time(fn, reps):
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        st.record(stream)
        for _ in range(reps):
            fn()
        en.record(stream)
        en.synchronize()
        return st.elapsed_time(en) / reps

    keys = torch.empty((L, n), dtype=torch.int32, device=dev)
    ms_hash = ev_time(lambda: idx.hash(pts, out=keys), args.kernel_reps)
    ms_build = ev_time(lambda: idx.rebuild(), max(2, args.kernel_reps // 3))
    ms_query = ev_time(lambda: idx.query(qs, r), max(2, args.kernel_reps // 3))

    # per-query latency: batched (whole batch, each query waits for the batch)
    # vs plain (one launch sequence and sync per query)
    nplain = min(args.plain_queries, nq)
    lat_plain = []
    for i in range(nplain):
        torch.cuda.synchronize()
        a = time.perf_counter()
        idx.query_plain(qs[i:i + 1], r)
        lat_plain.append((time.perf_counter() - a) * 1e3)
    lat_batch = []
    for _ in range(max(3, args.kernel_reps // 3)):
        torch.cuda.synchronize()
        a = time.perf_counter()
        idx.query(qs, r)
        lat_batch.append((time.perf_counter() - a) * 1e3)

    hash_bytes = n * (W * 8 + 4 * L)  # algorithmic: read the point, write L uint32 keys
    achieved = hash_bytes / (ms_hash * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": n / (ms_step * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: n={n} d={d} r={r} L={L} t={info['t']} nq={nq}",
                   "n": n, "d": d, "r": r, "L": L, "queries": nq, "seed": args.seed},
        "breakdown": {
            "hash_ms": ms_hash, "hash_points_per_s": n / (ms_hash * 1e-3),
            "hash_keys_per_s": n * L / (ms_hash * 1e-3),
            "build_ms": ms_build, "build_points_per_s": n / (ms_build * 1e-3),
            "query_batch_ms": ms_query, "queries_per_s": nq / (ms_query * 1e-3),
            "reported_ids": total_ids,
            "plain_query_ms_p50": pct(lat_plain, 50), "plain_query_ms_p99": pct(lat_plain, 99),
            "plain_queries_per_s": 1e3 / float(np.mean(lat_plain)) if lat_plain else None,
            "batch_latency_ms_p50": pct(lat_batch, 50), "batch_latency_ms_p99": pct(lat_batch, 99),
        },
        "roofline": {"kernel": "fht_hash_kernel", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "bytes_per_launch": hash_bytes},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, idx, qs, keys, args, fc)
    idx.close()
    print(json.dumps(out), flush=True)


COPY_BYTES = 1 << 30  # calibration copy: 1 GiB read + 1 GiB written per launch


def kernel_only(args, idx, pts, n, L, dev, torch):
    """Launches only the requested part, then a 1 GiB device copy, each
    --kernel-reps times, so that hardware counters of the part can be scaled
    by what the same counters read for a copy of known size."""
    keys = torch.empty((L, n), dtype=torch.int32, device=dev)
    for _ in range(args.kernel_reps):
        if args.kernel_only == "hash":
            idx.hash(pts, out=keys)
        else:
            idx.rebuild()
    src = torch.empty(COPY_BYTES // 4, dtype=torch.int32, device=dev).fill_(1)
    dst = torch.empty_like(src)
    for _ in range(args.kernel_reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"kernel_only": args.kernel_only, "reps": args.kernel_reps, "n": n, "L": L,
                      "copy_bytes": COPY_BYTES}), flush=True)


def cpu_baseline(w, idx, qs, keys, args, fc):
    """The oracle (plain O(dL) bcLSH keys + linear scan) timed on a bounded
    sample of the same workload on this host's cores, and compared with the
    GPU's answers on that sample."""
    import oracle

    budget = args.cpu_seconds
    pr = oracle.derive_params(w.d, w.r, args.seed)
    mask = oracle.masks(pr)
    cores = oracle.num_threads()
    # keys: calibrate on a small sample, then size the timed sample to ~half the budget
    probe = np.arange(64)
    a = time.perf_counter()
    oracle.keys(w.points, pr, which=probe, mask=mask)
    per_pt = (time.perf_counter() - a) / len(probe)
    npick = int(max(64, min(w.n, 0.5 * budget / max(per_pt, 1e-9))))
    rng = np.random.default_rng(7)
    which = np.sort(rng.choice(w.n, size=npick, replace=False))
    a = time.perf_counter()
    ok = oracle.keys(w.points, pr, which=which, mask=mask)
    t_keys = time.perf_counter() - a
    gk = keys[:, which].cpu().numpy().view(np.uint32)
    keys_equal = bool(np.array_equal(gk, ok))
    # queries: brute force on a sample of the batch, compared with the GPU answers
    a = time.perf_counter()
    oracle.brute_force(w.points, w.d, w.queries[:2], w.r)
    per_q = (time.perf_counter() - a) / 2
    nqs = int(max(2, min(w.nq, 0.4 * budget / max(per_q, 1e-9))))
    a = time.perf_counter()
    bf = oracle.brute_force(w.points, w.d, w.queries[:nqs], w.r)
    t_bf = time.perf_counter() - a
    got = fc.split_csr(*idx.query(qs[:nqs], w.r))
    same = all(np.array_equal(g, x) for g, x in zip(got, bf.ids))
    nn = sum(len(x) for x in bf.ids)
    found = sum(len(np.intersect1d(g, x)) for g, x in zip(got, bf.ids))
    return {"value": npick / t_keys, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": f"bcLSH keys (all {pr.L} tables) of {npick} random points of the workload; "
                      f"linear scan of {nqs} queries",
            "keys_per_s": npick * pr.L / t_keys, "linear_scan_queries_per_s": nqs / t_bf,
            "gpu_keys_equal_on_sample": keys_equal, "gpu_answers_equal_on_sample": bool(same),
            "recall_on_sample": (found / nn) if nn else 1.0}


if __name__ == "__main__":
    main()
