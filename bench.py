#!/usr/bin/env python3
"""Benchmark of the MASK hot path on one MI355X.

Workload: 1,000,000 x 128 Gaussian mixture (1,000 components, log-uniform
sigma in [0.1, 3]), index levels 100 chunks x 1,000 -> 5,000 -> 100, 30
Lloyd iterations, 10,000 queries, k = 10, beam r (default: the smallest
r of the sweep that reaches recall@10 >= 0.95 against exhaustive FP64
search).  A step is one pass of the whole hot path: mask_build on the
device-resident data, then mask_query of the 10,000 queries.

Prints one JSON line.  ``value`` is the query throughput (queries/s) of the
plain FP32 form with the index resident; ``build_s`` is the index build
time; kernel times come from HIP events recorded on the launch stream.
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--r", type=int, default=128)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--iters", type=int, default=30)
    ap.add_argument("--recall-sample", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sweep", type=str, default="",
                    help="comma-separated r values: report recall and q/s for each")
    ap.add_argument("--n", type=int, default=None, help="override the number of points")
    return ap.parse_args()


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the index and its queries live on a single MI355X)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import datagen
    import paper_2208_02734_amd as pk

    pk.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t_gen = time.time()
    cfg = datagen.config_scale(n=args.n)
    X, Q = cfg.X, cfg.Q
    print(f"# data {X.shape} queries {Q.shape} generated in {time.time() - t_gen:.1f}s",
          file=sys.stderr, flush=True)
    Xd = torch.from_numpy(X).cuda()
    Qd = torch.from_numpy(Q).cuda()
    torch.cuda.synchronize()
    levels = cfg.levels
    n, d = X.shape
    nq = Q.shape[0]
    stream = torch.cuda.current_stream()

    def step(r):
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        ix = pk.mask_build(Xd, levels, iters=args.iters, seed=1)
        e1.record(stream)
        ids, dist = pk.mask_query(ix, Qd, args.k, r)
        e2.record(stream)
        torch.cuda.synchronize()
        return ix, ids, dist, e0.elapsed_time(e1), e1.elapsed_time(e2)

    for w in range(args.warmup):
        ix, _, _, b_ms, q_ms = step(args.r)
        ix.free()
        print(f"# warmup {w}: build {b_ms:.1f} ms, query {q_ms:.2f} ms", file=sys.stderr,
              flush=True)

    pk.mask_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    build_ms, query_ms = [], []
    last = None
    for s in range(args.steps):
        if last is not None:
            last[0].free()
        last = step(args.r)
        build_ms.append(last[3])
        query_ms.append(last[4])
        print(f"# step {s}: build {last[3]:.1f} ms, query {last[4]:.2f} ms", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kt = pk.mask_timing_report()
    pk.mask_timing_enable(False)
    ix, ids, dist = last[0], last[1], last[2]

    # ---- roofline of the dominant kernel (MFMA assignment) and of the descent
    flops_per_build = 0.0
    items = n
    for (C, k) in levels:
        flops_per_build += 2.0 * items * k * d  # every item against the k prototypes of its chunk
        items = C * k
    flops_per_build *= (args.iters + 1)
    a_cnt, a_ms = kt.get("assign_l2_mfma", (0, 0.0))
    assign_tflops = flops_per_build * args.steps / (a_ms * 1e-3) / 1e12 if a_ms else 0.0
    d_cnt, d_ms = kt.get("descent", (0, 0.0))
    rows = kt.get("descent_rows", (0, 0.0))[0]
    ld = (d + 3) // 4 * 4
    desc_bytes = rows * (ld * 4 + 4)
    desc_gbs = desc_bytes / (d_ms * 1e-3) / 1e9 if d_ms else 0.0
    counters = ("descent_rows", "refine_small_points", "refine_full_points")
    kernels = {name: {"launches": c, "total_ms": round(ms, 3),
                      "avg_ms": round(ms / c, 4) if c else None}
               for name, (c, ms) in kt.items() if name not in counters}
    refine_stats = {"small_per_build": kt.get("refine_small_points", (0, 0))[0] // args.steps,
                    "full_per_build": kt.get("refine_full_points", (0, 0))[0] // args.steps}

    # ---- recall against exhaustive FP64 search (the oracle), and the CPU baseline
    result_recall = None
    cpu = None
    sweep = {}
    if not args.no_cpu_baseline:
        from oracle import compare as oc
        from oracle import mask_oracle as mo
        g = np.random.default_rng(0)
        sample = np.sort(g.choice(nq, min(args.recall_sample, nq), replace=False))
        t = time.time()
        tids, tdist = mo.exact_knn(X, Q[sample], args.k)
        print(f"# exact kNN of {sample.size} queries on the host: {time.time() - t:.1f}s",
              file=sys.stderr, flush=True)

        def recall_of(ids_np):
            got = ids_np[sample].astype(np.int64)
            got_true = oc.true_distances(X, Q[sample], got)
            return oc.recall_at_k(got, tids, tdist, got_true, args.k)

        result_recall = recall_of(ids.cpu().numpy())
        for r in [int(x) for x in args.sweep.split(",") if x]:
            e1, e2 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e1.record(stream)
            i2, _ = pk.mask_query(ix, Qd, args.k, r)
            e2.record(stream)
            torch.cuda.synchronize()
            sweep[r] = {"recall@10": round(recall_of(i2.cpu().numpy()), 4),
                        "queries_per_s": round(nq / (e1.elapsed_time(e2) * 1e-3), 1)}
            print(f"# sweep r={r}: {sweep[r]}", file=sys.stderr, flush=True)
        # the oracle's own descent on the same (exported) index, bounded sample
        protos, parents = [], []
        for lev in range(1, len(levels) + 1):
            P, par = ix.export_level(lev)
            protos.append(P)
            parents.append(par)
        oix = mo.index_from_arrays(X, protos, parents)
        oix.children(0)
        t = time.time()
        done = 0
        while done < nq and (time.time() - t < args.cpu_seconds or done < 20):
            mo.query_one(oix, Q[done], args.k, args.r)
            done += 1
        el = time.time() - t
        cpu = {"value": round(done / el, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
               "sample": f"FP64 numpy descent (r={args.r}, k={args.k}) of the first {done} "
                         f"queries on the GPU-built index, single thread, {el:.1f}s"}

    q_med = statistics.median(query_ms)
    b_med = statistics.median(build_ms)
    qs = sorted(query_ms)
    out = {
        "metric": "queries/s at recall@10>=0.95 vs FP64 oracle; p50/p99 latency; index build s",
        "value": round(nq / (q_med * 1e-3), 1),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mixture-1M-d128: 1,000,000 x 128 Gaussian mixture "
                               "(1,000 comps), levels 100x1000->5000->100, 30 Lloyd iters, "
                               "10,000 queries",
                   "k": args.k, "r": args.r, "form": "plain FP32"},
        "recall@10": None if result_recall is None else round(result_recall, 4),
        "build_s": round(b_med * 1e-3, 4),
        "query_batch_ms": {"p50": round(q_med, 3), "p99": round(qs[-1], 3)},
        "roofline": {"bound": "mfma", "kernel": "assign_l2_mfma",
                     "achieved": round(assign_tflops, 2), "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(assign_tflops / PEAK_FP32_TFLOPS, 4),
                     "traffic": None},
        "roofline_query": {"bound": "hbm", "kernel": "descent", "achieved": round(desc_gbs, 1),
                           "peak": PEAK_HBM_GBS, "unit": "GB/s",
                           "frac": round(desc_gbs / PEAK_HBM_GBS, 4), "traffic": None},
        "kernels": kernels,
        "refined_points": refine_stats,
        "cpu_baseline": cpu,
    }
    if sweep:
        out["sweep"] = sweep
    print(json.dumps(out), flush=True)
    ix.free()
    return 0


if __name__ == "__main__":
    sys.exit(main())
