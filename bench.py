#!/usr/bin/env python3
"""Benchmark of the batched B+-tree on one MI355X.

Workload: 2^24 distinct uniform u64 keys (seed 2), values hash64(key ^ 2),
bulk-loaded at fill 1.0 (fanout 16, 16 keys per leaf, height 6), resident in
HBM.  A timed step is one lookup batch of B = 1024 keys drawn uniformly from
the present keys, already in HBM; `value` is lookups per second over the K
timed steps (whole job, one GPU), `ms_per_step` the time per batch.

Also reported, measured in the same run outside the K timed steps:
  sweep          device time per lookup batch for B = 1, 8, 64, 256, 1024
                 (uniform and Zipf(0.99) queries)
  large_batch    one 2^20-key lookup batch (cold and warm)
  roofline       the lookup kernel at B = 2^20: algorithmic bytes per launch
                 over its average duration (HIP events on its own stream)
  cpu_baseline   the oracle's pointer B+-tree on the host cores, a bounded
                 sample of the same B = 1024 batches

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBS = 8000.0
N_LOG2 = 24
SEED = 2


def iqm(x):
    s = np.sort(np.asarray(x, dtype=np.float64))
    n = len(s) - len(s) % 4
    s = s[:n] if n else s
    q = len(s) // 4
    return float(s[q:len(s) - q].mean()) if len(s) >= 4 else float(s.mean())


def algorithmic_bytes(sorted_keys: np.ndarray, q: np.ndarray, height: int, hits: int, kb: int = 8) -> dict:
    """Bytes a lookup batch must move: every distinct node it visits once
    (inner node = key line + child line, leaf = key line), plus the value
    of each hit and the batch's input keys and outputs.  Exact for the
    bulk-loaded tree at fill 1.0 with 16 keys per leaf, where the leaf of
    the key of rank r is r // 16 and its level-l ancestor r // 16^(h-l)."""
    ranks = np.searchsorted(sorted_keys, q)
    ranks = np.minimum(ranks, len(sorted_keys) - 1).astype(np.int64)
    leaf = ranks // 16
    per_level = []
    node = leaf
    per_level.append(len(np.unique(node)))
    for _ in range(height - 1):
        node = node // 16
        per_level.append(len(np.unique(node)))
    per_level = per_level[::-1]  # root first
    inner_bytes = sum(per_level[:-1]) * (16 * kb + 64)
    leaf_bytes = per_level[-1] * 16 * kb
    io = len(q) * (kb + kb + 1) + hits * kb
    return {"distinct_nodes_per_level": per_level, "bytes": int(inner_bytes + leaf_bytes + io)}


def cpu_baseline(keys, vals, batches, budget_s=12.0):
    import oracle
    threads = len(os.sched_getaffinity(0))
    pt = oracle.PointerTree(16, 16, 64)
    pt.bulk_load(keys, vals)
    done = 0
    t0 = time.perf_counter()
    while True:
        for q in batches:
            pt.lookup(q, threads)
            done += len(q)
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt / 1e6, "unit": "Mops/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} lookups in batches of {len(batches[0])} on the oracle's pointer B+-tree "
                      f"(2^{N_LOG2} keys), batch split evenly over {threads} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--log2n", type=int, default=N_LOG2)
    ap.add_argument("--profile", action="store_true",
                    help="counter-collection mode: a 1 GiB device copy (calibration) and 2^20-key lookup "
                         "batches, three each, then exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the tree runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2604_21117_amd as g

    dev = "cuda"
    n = 1 << args.log2n
    keys = synth.uniform_keys(n, SEED, 64)
    vals = synth.values_for(keys, SEED, 64)
    skeys = np.sort(keys)

    tree = g.Tree(keys, vals, 8, leaf_slack=1 << 18, max_batch=1 << 20)
    st = tree.stats()
    stream = torch.cuda.Stream()

    if args.profile:
        # calibration: a plain copy of exactly 1 GiB (reads 1 GiB, writes 1 GiB)
        src = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
        src.fill_(3)
        BL = 1 << 20
        qld = tree.dev(synth.present_queries(keys, BL, SEED, purpose=5000))
        vl = torch.empty(BL, dtype=torch.int64, device=dev)
        fl = torch.empty(BL, dtype=torch.uint8, device=dev)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        for _ in range(3):
            g.tree_lookup_batch(tree.h, qld, vl, fl)
        torch.cuda.synchronize()
        print(json.dumps({"profile": "done", "copy_bytes": 1 << 30, "lookup_batch": BL}), flush=True)
        return

    B = 1024
    nbatch = 64
    qs = [synth.present_queries(keys, B, SEED, purpose=1000 + i) for i in range(nbatch)]
    qd = [tree.dev(q) for q in qs]
    vo = torch.empty(B, dtype=torch.int64, device=dev)
    fo = torch.empty(B, dtype=torch.uint8, device=dev)

    # correctness spot check of the timed path against the generator's closed
    # form (present keys return hash64(key ^ seed))
    with torch.cuda.stream(stream):
        g.tree_lookup_batch(tree.h, qd[0], vo, fo, stream)
    stream.synchronize()
    assert g.to_numpy(fo).all() and np.array_equal(g.to_numpy(vo, np.uint64), synth.values_for(qs[0], SEED, 64))

    # ---- timed steps: B = 1024 lookup batches, back to back on one stream
    with torch.cuda.stream(stream):
        for i in range(args.warmup):
            g.tree_lookup_batch(tree.h, qd[i % nbatch], vo, fo, stream)
    stream.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        for i in range(args.steps):
            g.tree_lookup_batch(tree.h, qd[i % nbatch], vo, fo, stream)
    stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed * 1e3 / args.steps
    value = args.steps * B / elapsed / 1e6

    # ---- per-batch device time sweep (events on the launch stream)
    zipf = synth.Zipf(n, 0.99, SEED)
    sweep = {}
    for dist in ("uniform", "zipf"):
        sweep[dist] = {}
        for b in (1, 8, 64, 256, 1024):
            if dist == "uniform":
                q = synth.present_queries(keys, b, SEED, purpose=3000 + b)
            else:
                q = keys[zipf.indices(b)]
            qdv = tree.dev(q)
            v2 = torch.empty(b, dtype=torch.int64, device=dev)
            f2 = torch.empty(b, dtype=torch.uint8, device=dev)
            ts = []
            for rep in range(110):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                with torch.cuda.stream(stream):
                    e0.record(stream)
                    g.tree_lookup_batch(tree.h, qdv, v2, f2, stream)
                    e1.record(stream)
                e1.synchronize()
                if rep >= 10:
                    ts.append(e0.elapsed_time(e1) * 1e3)
            us = iqm(ts)
            sweep[dist][str(b)] = {"us_per_batch": round(us, 3), "mops": round(b / us, 3)}

    # ---- large batch: roofline of the lookup kernel
    BL = 1 << 20
    ql = synth.present_queries(keys, BL, SEED, purpose=5000)
    qld = tree.dev(ql)
    vl = torch.empty(BL, dtype=torch.int64, device=dev)
    fl = torch.empty(BL, dtype=torch.uint8, device=dev)
    flush = torch.empty(2 << 30, dtype=torch.uint8, device=dev)
    cold, warm = [], []
    for rep in range(24):
        if rep % 2 == 0:
            with torch.cuda.stream(stream):
                flush.add_(1)  # stream 2 GiB through HBM to evict L2 and MALL
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(stream):
            e0.record(stream)
            g.tree_lookup_batch(tree.h, qld, vl, fl, stream)
            e1.record(stream)
        e1.synchronize()
        (cold if rep % 2 == 0 else warm).append(e0.elapsed_time(e1) * 1e3)
    del flush
    got = g.to_numpy(fl)
    assert got.all()
    ab = algorithmic_bytes(skeys, ql, st["height"], hits=int(got.sum()))
    cold_us, warm_us = iqm(cold[2:]), iqm(warm[2:])
    achieved = ab["bytes"] / (cold_us * 1e-6) / 1e9

    line = {
        "metric": "lookup Mops/s and us/batch at B=1..1024, 2^24 keys; learned vs plain tree",
        "value": round(value, 3),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 6),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"plain B+-tree lookups, 2^{args.log2n} uniform u64 keys, B=1024 uniform present "
                               f"queries", "keys": n, "batch": B, "fanout": 16, "leaf_cap": 16,
                   "height": st["height"], "path": "plain"},
        "sweep_us_per_batch": sweep,
        "large_batch": {"batch": BL, "cold_us": round(cold_us, 2), "warm_us": round(warm_us, 2),
                        "cold_glookups_per_s": round(BL / cold_us / 1e3, 3),
                        "warm_glookups_per_s": round(BL / warm_us / 1e3, 3),
                        "distinct_nodes_per_level": ab["distinct_nodes_per_level"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "k_lookup (B=2^20, cold)", "algorithmic_bytes": ab["bytes"]},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(keys, vals, qs[:16])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
