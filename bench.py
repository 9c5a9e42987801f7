"""Benchmark of the hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

One step = one pass of the hot path over the workload "balls64" (exact SDF
of a union of 8 seeded balls on a 64^3 grid, 128^3 refinement queries): the
dense float32 bound sweep with float64 tie resolution over all 262144 x
2097152 query-sample pairs.  Prints one JSON line.
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

FLOP_PER_PAIR = 13          # 3 sub, 1 mul, 2 fma (x2), sqrt, sub, add, max, min
FP32_VECTOR_PEAK = 157.3e12  # MI355X published float32 vector peak, FLOP/s


def cpu_baseline(w, sample_queries=1500):
    """The oracle's bound definition timed on a bounded sample of queries."""
    from oracle import bounds as OB
    q = w.queries[np.random.default_rng(0).choice(w.m, sample_queries, replace=False)]
    t0 = time.perf_counter()
    OB.cone_bounds(w.points, w.values, q, chunk=64)
    dt = time.perf_counter() - t0
    pairs = sample_queries * w.n
    return {"value": pairs / dt / 1e9, "unit": "G pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample_queries} random queries x all {w.n} samples, numpy float64, one thread"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the hot path runs on one "
              "MI355X; see DESIGN.md for how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_01919_amd import sdfi
    from sdfgen import configs

    w = configs.by_name("balls64")
    dev = torch.device("cuda:0")
    samples = torch.tensor(np.c_[w.points, w.values], device=dev)
    queries = torch.tensor(w.queries, device=dev)
    n, m = w.n, w.m

    for _ in range(args.warmup):
        sdfi.bounds(samples, queries, "fp32")
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        sdfi.bounds(samples, queries, "fp32")
    stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop) / args.steps
    pairs = n * m
    value = pairs / (ms * 1e-3) / 1e9
    achieved = FLOP_PER_PAIR * pairs / (ms * 1e-3)
    out = {
        "metric": "G query-sample bound evals/s", "value": round(value, 2), "unit": "G pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic", "config": {"workload": "balls64", "samples": n, "queries": m,
                                        "precision": "fp32 sweep, fp64 ties"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK, 4), "traffic": None},
        "wall_s": round(wall, 3),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
