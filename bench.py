"""Benchmark of the Fast CoveringLSH hot path on one MI355X.

A step is one pass of the whole hot path over the mid workload (n = 1,000,000
uniform 256-bit points, r = 8, L = 511 tables; 1,000 queries with 10 planted
neighbours each): hash every point into its L keys (Alg. 2), bucket the keys
into the L tables, and answer the query batch exactly (Strategy 2).  Inputs
are resident in HBM before the timed region starts.

Prints one JSON line.  `value` is points per second through the whole step.
Alongside: the breakdown (hash-only rate, keys/s, bucketing, queries/s,
Sec. 4.1's #Collisions and #Candidates per query), the roofline of the
dominant kernel and the hash / build / query rooflines at their algorithmic
bytes, the batched block (an autotuned 100,000-query batch against the plain
one-launch-sequence-per-query path) and the served block (continuous batching
of Poisson-arriving requests over the resident index, p50/p99 latency).
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
    ap.add_argument("--workload", default="mid", choices=["mid", "small", "learned_code", "batched", "fig3_replication"])
    ap.add_argument("--seed", type=int, default=3002)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="rough CPU budget of the oracle leg")
    ap.add_argument("--kernel-reps", type=int, default=10)
    ap.add_argument("--plain-queries", type=int, default=200)
    ap.add_argument("--batched", action="store_true",
                    help="refused: the autotuned 100k-query section on the 4M-point skewed index")
    ap.add_argument("--served", action="store_true",
                    help="refused: the request loop over the two full-size served indexes")
    ap.add_argument("--no-blocks", action="store_true",
                    help="skip the batched and served blocks on the default index")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rps", type=float, default=100.0, help="Poisson request rate of the served run")
    ap.add_argument("--serve-max", type=int, default=4096, help="largest request (queries) of the served block")
    ap.add_argument("--big-batch", type=int, default=100_000, help="queries in the batched block's batch")
    ap.add_argument("--study", choices=["fig2", "fig3"], default=None,
                    help="the precision/recall and #Collisions/#Candidates study of Sec. 4.3 at the shapes "
                         "of Fig. 2 (n = 10K..50K, r = 6) or Fig. 3 (n = 64K, replication and 2 parts); "
                         "prints one JSON line of rows instead of the benchmark")
    ap.add_argument("--study-queries", type=int, default=100)
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the sparse section (bag-of-words and user-rating shapes as rows of nonzeros)")
    ap.add_argument("--sparse-batch", type=int, default=4096, help="queries in the sparse section's large batch")
    ap.add_argument("--sparse-only", action="store_true", help="run the sparse section alone")
    ap.add_argument("--kernel-only", choices=["hash", "build"], default=None,
                    help="profiling aid: launch only this part (plus a plain copy of known size "
                         "for counter calibration) --kernel-reps times")
    return ap.parse_args()


def stage(msg):
    """Progress line on stderr, flushed, naming the step about to run."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q)) if len(a) else None


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)
    if args.batched or args.served:
        # an extended run of these two sections ended in an illegal memory
        # access whose cause has not been found; until it is, they do not run
        print(json.dumps({"error": "the --batched and --served sections are switched off: an extended run of them "
                                   "faulted the GPU and no cause has been shown; the full-size shapes run in the "
                                   "GPU tests at the default launch shape instead"}), flush=True)
        sys.exit(2)
    import torch

    import paper_1602_02620_amd as fc
    import synth

    torch.cuda.set_device(0)
    if args.study:
        print(json.dumps(study(args, fc, torch, synth)), flush=True)
        return
    if args.sparse_only:
        print(json.dumps({"sparse": sparse_section(args, fc, torch)}), flush=True)
        return
    dev = torch.device("cuda", 0)
    w = synth.WORKLOADS[args.workload]()
    n, d, r, nq = w.n, w.d, w.r, w.nq
    W = fc.words(d)
    pts = fc.to_device_words(w.points, dev)
    qs = fc.to_device_words(w.queries, dev)
    stream = torch.cuda.current_stream()

    rep = int(w.meta.get("replicate", 1))  # Alg. 1's replication (1 = none)
    stage(f"build index: {w.name} n={n} d={d} r={r} copies={rep}")
    idx = fc.Index(pts, d, r, seed=args.seed, replicate=rep, keep_build_scratch=True)
    info = idx.info
    L = info["L"]
    if args.kernel_only:
        stage(f"kernel-only {args.kernel_only}")
        kernel_only(args, idx, pts, n, L, dev, torch)
        idx.close()
        return

    # a step enqueues the rebuild and the query batch without host waits
    # (fclsh_index_rebuild_async, fclsh_query_batch_async) into buffers sized
    # from one synchronous batch; every step's status is checked after the
    # timed block
    # the verification launch shape for this index and batch, picked once by
    # the autotuner before anything is timed (the 4M-point skewed index keeps
    # the default shape, as its batched block stays off)
    if args.workload == "batched":
        step_tuning = dict(idx.get_tuning(), autotuned=False)
    else:
        stage("autotuning the query launch shape")
        step_tuning = dict(idx.autotune(qs, r), autotuned=True)
    stage("sizing the step's buffers from a synchronous batch")
    offs0, _ = idx.query(qs, r)
    total0 = int(offs0[-1].item())
    offs_buf = torch.empty(nq + 1, dtype=torch.int64, device=dev)
    ids_buf = torch.empty(max(total0, 1), dtype=torch.int32, device=dev)
    res_buf = torch.zeros((max(args.steps, args.warmup), 2), dtype=torch.int64, device=dev)
    idx.reserve(nq, pair_capacity=max(2 * total0, 1 << 16), spill_capacity=1 << 16)

    def step(k=0):
        idx.rebuild_async()
        idx.query_async(qs, r, offs_buf, ids_buf, res_buf[k])
        return offs_buf, ids_buf

    def check_steps(count):
        res = res_buf[:count].cpu().numpy()
        if (res[:, 1] != 0).any() or (res[:, 0] != total0).any():
            raise RuntimeError(f"a benchmark step overflowed or changed its answer: {res.tolist()}")

    stage(f"{args.warmup} warmup + {args.steps} timed steps")
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    check_steps(args.warmup)
    t0 = time.perf_counter()
    for k in range(args.steps):
        offs, ids = step(k)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    check_steps(args.steps)
    ms_step = (t1 - t0) * 1e3 / args.steps
    total_ids = int(offs[-1].item())

    # ---- per-kernel durations: HIP events recorded by the library between
    # the kernels, on the stream they are launched on
    stage("per-kernel timing of the rebuild")
    idx.rebuild_timed()
    runs = [idx.rebuild_timed() for _ in range(args.kernel_reps)]
    phase_ms = {k: float(np.mean([run[k] for run in runs])) for k in runs[0]}
    nblk = (n + 8191) // 8192
    entries = n * L
    # how pass 2 treats the groups (entries sharing the top group_bits key
    # bits): the group kernel takes every group of at most 4608 entries, by
    # slot ranks when no bin holds over 48 entries, else by stable ballot
    # ranks; larger groups go to the second kernel
    dir_bits, group_bits = info["dir_bits"], info["group_bits"]
    binsz = idx.directory().to(torch.int64).diff(dim=1).view(L, 1 << group_bits, -1)
    sb_count, sb_max = binsz.sum(-1), binsz.amax(-1)
    rest = sb_count > 4608
    rest_entries = int(sb_count[rest].sum().item())
    ballot_entries = int(sb_count[~rest & (sb_max > 48)].sum().item())
    dir_bytes = 4 * L * ((1 << dir_bits) + 1)
    # the tables store a key as its low 16 bits when the bin holds the rest;
    # with such keys, no merged pass-2 groups (group_bits >= 8) and ids below
    # 2^25, the passes hand on 6-byte entries instead of 8-byte ones
    kb = idx.table_pointers()[4]
    mid_bytes = 6 if (kb == 2 and group_bits >= 8 and n <= 1 << 25) else 8
    # bytes each kernel moves itself (its reads and writes, for the counter
    # comparison) ...
    moved_bytes = {
        "fht_hash_kernel": n * (W * 8 + 4 * L),                    # read the point, write its L keys
        "p1_hist_kernel": 4 * entries + 4 * L * nblk * 256,          # read keys, write tile histograms
        "p1_scan_kernel": 8 * L * nblk * 256,                        # read + write the histograms
        "p1_scatter_kernel": (4 + mid_bytes) * entries,              # read key, write the entry
        # split of the super-bins (large n only): read the key words twice and
        # the id words once, write both
        "p1b_split_kernel": ((4 + 2 * mid_bytes) * entries + 4 * L * ((256 << (group_bits - 8)) + 1))
        if group_bits > 8 else 0,
        # pass 2: read the entry, write the stored key (kb bytes) and id of
        # each entry it reorders, and its bins' directory entries
        "p2_fast_kernel": (mid_bytes + 4 + kb) * (entries - rest_entries) + dir_bytes * (1 - rest_entries / entries),
        "p2_rest_kernel": (mid_bytes + 4 + kb) * rest_entries + dir_bytes * (rest_entries / entries) + 4,
    }
    # ... and the algorithmic bytes the roofline is priced at: the hash step
    # reads a point and writes its L keys (d/8 + 4L per point); the table
    # build's minimum is 8 + kb B per table entry (read a key, write the
    # stored key and the id), which each build kernel is charged for the
    # entries it handles
    per_entry = 8 + kb
    alg_bytes = {k: per_entry * entries for k in moved_bytes}
    alg_bytes["fht_hash_kernel"] = moved_bytes["fht_hash_kernel"]
    alg_bytes["p1b_split_kernel"] = per_entry * entries if group_bits > 8 else 0
    alg_bytes["p2_fast_kernel"] = per_entry * (entries - rest_entries)
    alg_bytes["p2_rest_kernel"] = per_entry * rest_entries
    dominant = max(phase_ms, key=phase_ms.get)
    achieved = alg_bytes[dominant] / (phase_ms[dominant] * 1e-3) / 1e9
    ms_hash = phase_ms["fht_hash_kernel"]
    build_bytes = per_entry * entries  # the table build as a whole: read key, write stored key + id
    ms_build = sum(v for k, v in phase_ms.items() if k != "fht_hash_kernel")

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

    stage("query batch timing")
    ms_query = ev_time(lambda: idx.query(qs, r), max(2, args.kernel_reps // 3))

    # per-query latency: batched (whole batch, each query waits for the batch)
    # vs plain (one launch sequence and sync per query)
    stage(f"plain path, {min(args.plain_queries, nq)} queries")
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

    # Sec. 4.1's cost measures per query: #Collisions (summed bucket sizes
    # over the L tables) and #Candidates (distinct points among them)
    # (on the 4M-point skewed index over its first 2,000 queries, as its
    # full-size test does, the averages standing for the batch)
    ncost = min(nq, 2000) if args.workload == "batched" else nq
    coll_t, cand_t = idx.cost(qs[:ncost])
    coll_per_query = float(coll_t.to(torch.float64).mean().item())
    cand_per_query = float(cand_t.to(torch.float64).mean().item())
    # the query side's algorithmic bytes: per query its d/8 bits, a directory
    # pair per table, a stored key and an id per bucket entry (bins mix keys),
    # a point per distinct candidate (at least one 64-byte sector) and 4 bytes
    # per reported id
    q_bytes = (nq * (W * 8 + 8 * L) + (kb + 4) * coll_per_query * nq
               + cand_per_query * nq * max(W * 8, 64) + 4 * total_ids)
    extra = {}
    if args.workload == "batched" or args.no_blocks:
        # the autotuned large batch and the request loop stay off the
        # 4M-point skewed index: a memory fault seen there is not explained
        why = "off on the 4M-point skewed index" if args.workload == "batched" else "--no-blocks"
        extra["batched"] = {"skipped": why}
        extra["served"] = {"skipped": why}
    else:
        stage("batched block: autotuned large batch vs plain")
        extra["batched"] = batched_block(args, w, idx, qs, r, total0, lat_plain, torch, fc)
        stage("served block: request loop over the resident index")
        extra["served"] = served_block(args, w, idx, r, lat_plain, torch, fc)
    stage("keys of all points for the oracle comparison")
    keys = torch.empty((L, n), dtype=torch.int32, device=dev)
    idx.hash(pts, out=keys)
    torch.cuda.synchronize()
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
        "config": {"workload": f"{w.name}: n={n} d={d} r={r}" + (f" copies={rep}" if rep > 1 else "")
                               + f" L={L} t={info['t']} nq={nq}",
                   "n": n, "d": d, "r": r, "L": L, "queries": nq, "seed": args.seed, "copies": rep},
        "breakdown": {
            "hash_ms": ms_hash, "hash_points_per_s": n / (ms_hash * 1e-3),
            "hash_keys_per_s": n * L / (ms_hash * 1e-3),
            "hash_GBps": alg_bytes["fht_hash_kernel"] / (ms_hash * 1e-3) / 1e9,
            "build_ms": ms_build, "build_entries_per_s": entries / (ms_build * 1e-3),
            "build_GBps_at_min_bytes": build_bytes / (ms_build * 1e-3) / 1e9, "build_bytes_per_entry": per_entry,
            "kernel_ms": phase_ms,
            "pass2_ballot_share": ballot_entries / entries, "pass2_rest_share": rest_entries / entries,
            "pass2_form": idx.build_mode, "query_tuning": step_tuning,
            "query_batch_ms": ms_query, "queries_per_s": nq / (ms_query * 1e-3),
            "reported_ids": total_ids, "cost_sample_queries": ncost, "collisions_per_query": coll_per_query,
            "candidates_per_query": cand_per_query,
            "plain_query_ms_p50": pct(lat_plain, 50), "plain_query_ms_p99": pct(lat_plain, 99),
            "plain_queries_per_s": 1e3 / float(np.mean(lat_plain)) if lat_plain else None,
            "batch_latency_ms_p50": pct(lat_batch, 50), "batch_latency_ms_p99": pct(lat_batch, 99),
        },
        "roofline": {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dominant, n, d, r),
                     "bytes_per_launch": alg_bytes[dominant], "ms_per_launch": phase_ms[dominant],
                     "moved_bytes_per_launch": moved_bytes[dominant]},
        "rooflines": {
            "hash": roof(alg_bytes["fht_hash_kernel"], ms_hash, "fht_hash_kernel", n, d, r,
                         "d/8 + 4L bytes per point"),
            "build": roof(build_bytes, ms_build, None, n, d, r,
                          f"{per_entry} bytes per table entry (key read, {kb}-byte key and id written), all build kernels"),
            "query": roof(q_bytes, ms_query, None, n, d, r,
                          f"per query d/8 + 8L + {kb + 4} per collision + max(d/8, 64) per candidate + 4 per id"),
        },
    }
    out.update(extra)
    if not args.no_cpu_baseline:
        stage(f"oracle on the host, about {args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(w, idx, qs, keys, args, fc)
    idx.close()
    del keys
    torch.cuda.empty_cache()
    if not args.no_sparse:
        stage("sparse section")
        out["sparse"] = sparse_section(args, fc, torch)
    print(json.dumps(out), flush=True)


# Settings of the study (Sec. 4.3): Fig. 2 without pre-processing, Fig. 3
# with Alg. 1's replication (copies 4, 3, 2, 2 for r = 2..5) and with two
# parts (r = 10, 12, 14, 16).  (n, r, copies, parts)
STUDY = {
    "fig2": [(n, 6, 1, 1) for n in (10_000, 20_000, 30_000, 40_000, 50_000)],
    "fig3": [(65_536, r, k, 1) for r, k in ((2, 4), (3, 3), (4, 2), (5, 2))]
            + [(65_536, r, 1, 2) for r in (10, 12, 14, 16)],
}


def study(args, fc, torch, synth):
    """Precision / recall and Sec. 4.1's cost measures of fcLSH on the
    paper's synthetic sets (d = 128, points around each query at distances
    spread over 1..128), one index per setting.  Recall is measured against
    the library's linear scan; precision is reported ids over distinct
    candidates (what the paper notes equals the speedup over a linear scan
    when C_lookup is ignored).  The hash time per query is the key
    computation of a whole query batch divided by its size."""
    rows = []
    d, nq = 128, args.study_queries
    for n, r, copies, parts in STUDY[args.study]:
        stage(f"study {args.study}: n={n} r={r} copies={copies} parts={parts}")
        w = synth.hamming_balls(n, d, nq, seed=5000 + n + 100 * r)
        pts, qs = fc.to_device_words(w.points), fc.to_device_words(w.queries)
        idx = fc.Index(pts, d, r, seed=args.seed, replicate=copies if copies > 1 else 0,
                       partitions=parts if parts > 1 else 0)
        L = idx.info["L"]
        got = fc.split_csr(*idx.query(qs, r))
        truth = fc.split_csr(*fc.linear_scan(pts, d, qs, r))
        coll, cand = (x.cpu().numpy() for x in idx.cost(qs))
        found = sum(len(np.intersect1d(g, t)) for g, t in zip(got, truth))
        ntruth = sum(len(t) for t in truth)
        nrep = sum(len(g) for g in got)
        keys = torch.empty((L, nq), dtype=torch.int32, device="cuda")
        idx.hash(qs, out=keys)
        torch.cuda.synchronize()
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st.record()
        for _ in range(10):
            idx.hash(qs, out=keys)
        en.record()
        en.synchronize()
        per_q = [len(g) / c if c else 1.0 for g, c in zip(got, cand)]
        rows.append({"n": n, "d": d, "r": r, "copies": copies, "parts": parts, "L": L, "queries": nq,
                     "recall": found / ntruth if ntruth else 1.0, "exact": nrep == found == ntruth,
                     "precision": nrep / float(cand.sum()) if cand.sum() else 1.0,
                     "precision_mean_per_query": float(np.mean(per_q)),
                     "neighbours_per_query": ntruth / nq,
                     "collisions_per_query": float(coll.mean()), "candidates_per_query": float(cand.mean()),
                     "hash_us_per_query": st.elapsed_time(en) * 1e3 / 10 / nq})
        idx.close()
    return {"study": args.study, "data": "synthetic: d=128, points around each query at distances U{1..128}",
            "rows": rows}


def roof(nbytes, ms, kernel, n, d, r, basis):
    gbps = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBS,
            "bytes": nbytes, "ms": ms, "basis": basis,
            "traffic": measured_traffic(kernel, n, d, r) if kernel else None}


def batched_block(args, w, idx, qs, r, total0, lat_plain, torch, fc):
    """The batched path at scale on the default index: the autotuner picks
    the verification launch shape on a sample, then one synchronous batch of
    the workload's queries repeated to --big-batch queries, against the plain
    path (one launch sequence and synchronisation per query)."""
    tune = idx.autotune(qs, r)
    reps = -(-args.big_batch // qs.shape[0])
    big = qs.repeat(reps, 1)[:args.big_batch].contiguous()
    offs, ids = idx.query(big, r)  # sizes the workspace
    torch.cuda.synchronize()
    lat = []
    for _ in range(3):
        a = time.perf_counter()
        offs, ids = idx.query(big, r)
        lat.append((time.perf_counter() - a) * 1e3)
    # every repeat of the base batch answers as the base batch did
    cnt = (offs[1:] - offs[:-1]).view(-1)
    base = cnt[:qs.shape[0]]
    same = bool(torch.equal(cnt, base.repeat(reps)[:cnt.numel()]))
    ms = float(np.median(lat))
    qps = big.shape[0] / (ms * 1e-3)
    plain_qps = 1e3 / float(np.mean(lat_plain))
    return {"queries": int(big.shape[0]), "tuning": tune, "batch_ms": ms, "queries_per_s": qps,
            "batch_latency_ms_p50": pct(lat, 50), "batch_latency_ms_p99": pct(lat, 99),
            "plain_queries_per_s": plain_qps, "plain_query_ms_p50": pct(lat_plain, 50),
            "plain_query_ms_p99": pct(lat_plain, 99), "speedup_vs_plain": qps / plain_qps,
            "answers_equal_across_repeats": same, "reported_ids": int(offs[-1].item())}


def served_block(args, w, idx, r, lat_plain, torch, fc):
    """Continuous batching over the resident default index: Poisson request
    arrivals, request sizes U[1, --serve-max] queries drawn from the
    workload's queries, radius U{0..r} per request.  Latency is arrival to
    completion; the plain path's service time for the same request (its
    queries one launch sequence each) is reported beside it.  Sampled answers
    are compared with the same queries answered alone."""
    from paper_1602_02620_amd.serve import Server, poisson_trace

    srv = Server({"mid": idx}, max_batch=args.serve_max, streams=3)
    rng = np.random.default_rng(31)
    arrivals = poisson_trace(args.serve_rps, args.serve_seconds, rng)
    reqs = []
    t0 = time.perf_counter()
    for ta in arrivals:
        while time.perf_counter() - t0 < ta:
            time.sleep(50e-6)
        m = int(rng.integers(1, args.serve_max + 1))
        rows = rng.integers(0, w.nq, size=m)
        rad = int(rng.integers(0, r + 1))
        reqs.append((rows, rad, srv.submit("mid", w.queries[rows], rad)))
    results = [f.result(timeout=300) for *_, f in reqs]
    t_end = time.perf_counter()
    srv.close()
    st = srv.stats()
    per_q = float(np.mean(lat_plain))
    plain_req = [per_q * len(rows) for rows, _, _ in reqs]
    # alone vs in the mix, for a few sampled requests
    same = True
    for k in rng.choice(len(reqs), size=min(4, len(reqs)), replace=False):
        rows, rad, _ = reqs[k]
        alone = fc.split_csr(*idx.query_radii(fc.to_device_words(w.queries[rows]),
                                              torch.full((len(rows),), rad, dtype=torch.int32)))
        same &= all(np.array_equal(a, b) for a, b in zip(alone, results[k]))
    return {"requests": st["requests"], "queries": st["queries"], "batches": st["batches"],
            "offered_requests_per_s": args.serve_rps, "seconds": t_end - t0,
            "queries_per_s": st["queries"] / (t_end - t0),
            "latency_ms_p50": st["p50_ms"], "latency_ms_p99": st["p99_ms"],
            "plain_service_ms_p50": pct(plain_req, 50), "plain_service_ms_p99": pct(plain_req, 99),
            "alone_equals_mix": bool(same), "reruns": st["reruns"], "resident_bytes": st["resident_bytes"]}


# The sparse shapes (Table 2's Enron and MovieLens as synthetic rows), with
# the paper's partitions for them (Sec. 4.4): Enron up to r = 29 with 3
# parts, MovieLens r = 8..13 with 2 parts and r <= 7 with 1.
SPARSE_RUNS = [("enron_like", 29, 3, 4101), ("movielens_like", 13, 2, 4102), ("movielens_like", 7, 1, 4103)]


def sparse_section(args, fc, torch):
    """Per shape: the sparse index's build (hash kernel and table kernels
    timed by events between them), the hash kernel's roofline (algorithmic
    bytes: per point its row, 8 + 4 nnz bytes, and its L keys), the 100-query
    batch and a large batch of those queries repeated, every answer of the
    100 queries checked against the oracle's linear scan, and the oracle's
    own per-query time on a sample beside it."""
    import oracle
    import synth

    runs = []
    cache = {}
    for name, r, t, seed in SPARSE_RUNS:
        if name not in cache:
            cache[name] = synth.SPARSE_WORKLOADS[name](1.0)
        w = cache[name]
        stage(f"sparse {name}: n={w.n} d={w.d} nnz={w.cols.size} r={r} t={t}")
        ptr, cols = fc.to_device_rows(w.ptr, w.cols)
        qptr, qcols = fc.to_device_rows(w.qptr, w.qcols)
        torch.cuda.synchronize()
        a = time.perf_counter()
        idx = fc.SparseIndex(ptr, cols, w.d, r, seed=seed, partitions=t, keep_build_scratch=True)
        build_wall = (time.perf_counter() - a) * 1e3
        L = idx.info["L"]
        idx.rebuild_timed()
        phases = [idx.rebuild_timed() for _ in range(args.kernel_reps)]
        ph = {("fht_hash_sparse_kernel" if k == "fht_hash_kernel" else k): float(np.mean([p[k] for p in phases]))
              for k in phases[0]}
        ms_hash = ph["fht_hash_sparse_kernel"]
        ms_tables = sum(v for k, v in ph.items() if k != "fht_hash_sparse_kernel")
        hash_bytes = w.n * (8 + 4 * L) + 4 * w.cols.size
        offs, ids = idx.query(qptr, qcols, r)  # sizes the workspace
        got = fc.split_csr(offs, ids)
        coll, cand = (x.to(torch.float64) for x in idx.cost(qptr, qcols))
        st, en = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        st.record()
        for _ in range(5):
            idx.query(qptr, qcols, r)
        en.record()
        en.synchronize()
        ms_q100 = st.elapsed_time(en) / 5
        reps = -(-args.sparse_batch // w.nq)
        sizes = np.diff(w.qptr)
        bptr = np.concatenate([[0], np.cumsum(np.tile(sizes, reps))]).astype(np.int64)
        bptr_d, bcols_d = fc.to_device_rows(bptr, np.tile(w.qcols, reps))
        boffs, _ = idx.query(bptr_d, bcols_d, r)
        torch.cuda.synchronize()
        st.record()
        for _ in range(3):
            boffs, _ = idx.query(bptr_d, bcols_d, r)
        en.record()
        en.synchronize()
        ms_big = st.elapsed_time(en) / 3
        cnt = (boffs[1:] - boffs[:-1]).cpu().numpy()
        same_rep = bool(np.array_equal(cnt, np.tile(cnt[:w.nq], reps)))
        stage(f"sparse {name}: oracle linear scan of {w.nq} queries")
        a = time.perf_counter()
        want = oracle.brute_force_sparse(w.ptr, w.cols, w.qptr, w.qcols, w.d, r).ids
        t_bf = time.perf_counter() - a
        equal = len(got) == len(want) and all(np.array_equal(g, x) for g, x in zip(got, want))
        pr = oracle.derive_params(w.d, r, seed, override_t=t)
        pick = np.arange(0, w.n, max(1, w.n // 200))[:200]
        sp = np.concatenate([[0], np.cumsum(w.ptr[pick + 1] - w.ptr[pick])]).astype(np.int64)
        sc = np.concatenate([w.cols[w.ptr[i]:w.ptr[i + 1]] for i in pick])
        a = time.perf_counter()
        oracle.keys_sparse(sp, sc, pr)
        t_keys = time.perf_counter() - a
        runs.append({
            "workload": f"{name}: n={w.n} d={w.d} nnz={w.cols.size} r={r} t={t} L={L} nq={w.nq}",
            "build_ms_wall": build_wall, "hash_ms": ms_hash, "tables_ms": ms_tables, "kernel_ms": ph,
            "hash_points_per_s": w.n / (ms_hash * 1e-3),
            "hash_roofline": roof(hash_bytes, ms_hash, None, w.n, w.d, r,
                                  "per point 8 + 4 nnz bytes of its row and 4L bytes of keys"),
            "query_batch100_ms": ms_q100, "query_ms_per_query_batch100": ms_q100 / w.nq,
            "big_batch_queries": int(reps * w.nq), "big_batch_ms": ms_big,
            "big_batch_queries_per_s": reps * w.nq / (ms_big * 1e-3),
            "reported_ids_per_query": sum(len(g) for g in got) / w.nq,
            "collisions_per_query": float(coll.mean().item()), "candidates_per_query": float(cand.mean().item()),
            "answers_equal_oracle": bool(equal), "repeats_answer_alike": same_rep,
            "cpu_baseline": {"kind": "oracle", "cores": oracle.num_threads(),
                             "linear_scan_ms_per_query": t_bf * 1e3 / w.nq,
                             "keys_points_per_s": len(pick) / t_keys,
                             "sample": f"linear scan of the {w.nq} queries; O(nnz L) keys of {len(pick)} points"},
        })
        idx.close()
        del ptr, cols
        torch.cuda.empty_cache()
    return {"data": "synthetic sparse rows: log-normal row lengths, Zipf column popularity, planted neighbours",
            "runs": runs}


KERNEL_SOURCES = {"fht_hash_kernel": "hash.hip", "p1_hist_kernel": "tables.hip", "p1_scan_kernel": "tables.hip",
                  "p1_scatter_kernel": "tables.hip", "p2_fast_kernel": "tables.hip",
                  "p2_rest_kernel": "tables.hip", "p1b_split_kernel": "tables.hip"}


def measured_traffic(kernel, n, d, r):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by what it reads for a copy of
    known size), or None when there is none for this kernel and workload or
    the kernel's source has changed since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f).get(kernel)
    if not rec or (rec["n"], rec["d"], rec["r"]) != (n, d, r):
        return None
    src = os.path.join(ROOT, "paper_1602_02620_amd", "csrc", KERNEL_SOURCES[kernel])
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return rec["fetch_bytes"] + rec["write_bytes"]


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
    rep = int(w.meta.get("replicate", 1))
    if rep > 1:  # the family of the replicated points (Alg. 1): k*d coordinates, radius k*r, one part
        pr = oracle.derive_params(rep * w.d, rep * w.r, args.seed, override_t=1)
        kpts = oracle.replicate(w.points, w.d, rep)
    else:
        pr = oracle.derive_params(w.d, w.r, args.seed)
        kpts = w.points
    mask = oracle.masks(pr)
    cores = oracle.num_threads()
    # keys: calibrate on a sample that keeps every thread busy (the oracle
    # hands out points in chunks of 64), then size the timed sample to about
    # half the budget
    probe = np.arange(min(w.n, 64 * 4 * cores))
    a = time.perf_counter()
    oracle.keys(kpts, pr, which=probe, mask=mask)
    per_pt = (time.perf_counter() - a) / len(probe)
    npick = int(max(64, min(w.n, 0.5 * budget / max(per_pt, 1e-9))))
    rng = np.random.default_rng(7)
    which = np.sort(rng.choice(w.n, size=npick, replace=False))
    a = time.perf_counter()
    ok = oracle.keys(kpts, pr, which=which, mask=mask)
    t_keys = time.perf_counter() - a
    gk = keys[:, which].cpu().numpy().view(np.uint32)
    keys_equal = bool(np.array_equal(gk, ok))
    # queries: brute force on a sample of the batch, compared with the GPU answers
    nprobe = min(w.nq, 2 * cores)  # one query per thread at a time
    a = time.perf_counter()
    oracle.brute_force(w.points, w.d, w.queries[:nprobe], w.r)
    per_q = (time.perf_counter() - a) / nprobe
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
