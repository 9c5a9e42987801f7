"""Benchmark of the hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]

Timed step: the dense query x sample bound sweep (float32 sweep, float64 tie
resolution) over the workload "balls64": exact SDF of a union of 8 seeded
balls sampled on a 64^3 grid, against all 128^3 refinement queries
(262144 x 2097152 pairs).  Reported beside it, each timed on its own:
  - the greedy interpolation (order, witnesses, sequential assignment,
    certificate) of "sphere16" (16^3 samples, 32^3 queries), queries/s;
  - the batched greedy (one launch, one work-group per instance) against the
    same instances run one after another;
  - the oracle's bound definition on a bounded sample on the host CPU.
Prints one JSON line.
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

FLOP_PER_PAIR = 13           # 3 sub, 1 mul, 2 fma (x2), sqrt, sub, add, max, min
FP32_VECTOR_PEAK = 157.3e12  # MI355X published float32 vector peak, FLOP/s


def cpu_baseline(w, sample_queries=1500):
    """The oracle's bound definition timed on a bounded sample of queries."""
    from oracle import bounds as OB
    q = w.queries[np.random.default_rng(0).choice(w.m, sample_queries, replace=False)]
    t0 = time.perf_counter()
    OB.cone_bounds(w.points, w.values, q, chunk=64)
    dt = time.perf_counter() - t0
    pairs = sample_queries * w.n
    return {"value": round(pairs / dt / 1e9, 4), "unit": "G pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample_queries} random queries x all {w.n} samples of balls64, numpy float64, "
                      f"one thread, {dt:.1f} s"}


def timed(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(steps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / steps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-greedy", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the hot path runs on one "
              "MI355X; DESIGN.md section 9 describes how it would shard)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2605_01919_amd import sdfi
    from sdfgen import configs

    dev = torch.device("cuda:0")
    w = configs.by_name("balls64")
    samples = torch.tensor(np.c_[w.points, w.values], device=dev)
    queries = torch.tensor(w.queries, device=dev)
    n, m = w.n, w.m

    lib_ms = {}

    def step():
        sdfi.bounds(samples, queries, "fp32")

    sdfi.timing(True)
    t0 = time.perf_counter()
    ms = timed(step, args.steps, args.warmup)
    wall = time.perf_counter() - t0
    kt = sdfi.timing_read()
    sdfi.timing(False)
    sweep_ms = kt["sweep"][0] / max(kt["sweep"][1], 1)
    pairs = n * m
    achieved = FLOP_PER_PAIR * pairs / (sweep_ms * 1e-3)
    out = {
        "metric": "G query-sample bound evals/s + queries/s, batched vs plain, at 1e-5 abs",
        "value": round(pairs / (ms * 1e-3) / 1e9, 2), "unit": "G pair-evals/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 sweep + f64 decisions",
        "data": "synthetic",
        "config": {"workload": "balls64", "samples": n, "queries": m, "pairs": pairs,
                   "step": "sdfi_bounds: float32 sweep + float64 resolve"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK, 4), "traffic": None,
                     "kernel": "sweep_kernel", "kernel_ms": round(sweep_ms, 3),
                     "flop_per_launch": FLOP_PER_PAIR * pairs},
        "wall_s": round(wall, 3),
    }
    if not args.no_greedy:
        c1 = configs.by_name("sphere16")
        s1 = torch.tensor(np.c_[c1.points, c1.values], device=dev)
        q1 = torch.tensor(c1.queries, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g = sdfi.greedy(s1, q1, grid=c1.grid, certify=True)
        torch.cuda.synchronize()
        gt = time.perf_counter() - t0
        rep = g["report"]
        out["greedy"] = {"workload": "sphere16", "queries": c1.m, "samples": c1.n, "seconds": round(gt, 3),
                         "queries_per_s": round(c1.m / gt, 1),
                         "greedy_ms": round(rep["ms_phase"][2], 1), "order_ms": round(rep["ms_phase"][0], 1),
                         "witness_ms": round(rep["ms_phase"][1], 1), "certificate_ms": round(rep["ms_phase"][3], 1),
                         "pairs": rep["pairs_evaluated"],
                         "violations": rep["n_violations_pairwise"] + rep["n_violations_witness"],
                         "kinds": {"hi": rep["n_hi"], "lo": rep["n_lo"], "zero": rep["n_zero"],
                                   "rmin": rep["n_rmin"]}}
        inst = configs.batch(16, grids=(4, 5, 6))
        tens = [(torch.tensor(np.c_[x.points, x.values], device=dev), torch.tensor(x.queries, device=dev), x.grid)
                for x in inst]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sdfi.greedy_batched(tens)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        t0 = time.perf_counter()
        for s_, q_, g_ in tens:
            sdfi.greedy(s_, q_, grid=g_)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        mq = sum(x.m for x in inst)
        out["batched"] = {"workload": "16 sphere/box unions, grids {4,5,6}", "queries": mq,
                          "batched_s": round(tb, 3), "plain_s": round(tp, 3),
                          "batched_queries_per_s": round(mq / tb, 1), "plain_queries_per_s": round(mq / tp, 1),
                          "speedup": round(tp / tb, 2)}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
