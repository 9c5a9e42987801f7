"""Benchmark of the hot path on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-greedy] [--no-batched]
                [--no-repair] [--copy-bytes N]
python bench.py --csg N [--save OUT.npz]    (the repair workload on an N^3 grid only, timed in parts)

Timed step (the JSON line's `value`): the dense query x sample bound
reduction (Sec. 4.3 cone bounds with argmin/argmax, float32 sweep and float64
tie resolution) of the workload "balls64": the exact SDF of a union of 8
seeded balls sampled on a 64^3 grid, against all 128^3 refinement queries
(262144 x 2097152 pairs), inputs resident in device memory.  The float32
sweep evaluates only the pairs of the tiles and blocks it cannot rule out
from their box and value range (the results are those of the full sweep):
`value` is those evaluated pairs per second of whole step time,
`dense_equivalent_per_s_G` counts all n x m pairs per second, and
roofline.achieved counts the evaluated pairs at 13 FLOP each over the sweep
kernel's own duration.

Reported beside it, each timed on its own with the device synchronised
around it (wall clock):
  greedy    the whole greedy interpolation (refinement order, sample
            witnesses, sequential assignment with exact validity checks,
            Prop. 1 certificate) of "sphere16" (16^3 samples, 32^3 queries),
            float64 throughout, in queries/s;
  backward  the gradient of the sphere16 values w.r.t. the samples;
  batched   64 sphere/box union instances on uneven grids in one launch
            (one work-group per instance) against the same 64 instances
            run one after another through the single-instance entry;
  repair    the pseudo-SDF repair of a CSG field (witnesses of all samples,
            removal of the fully covered ones, minimum valid radius of the
            removed samples and of scattered extension queries);
  cpu_baseline  the oracle's bound definition on a bounded sample of
            balls64 queries on one host core.
Each leg prints a progress line on stderr when it ends.  Prints one JSON
line on stdout.

roofline.traffic is the sweep kernel's HBM bytes per launch from the
FETCH_SIZE and WRITE_SIZE counter runs recorded in
profiles/sweep_traffic_balls64.md, reported only while the sweep's source
is the one those counters were taken on (null otherwise).  --copy-bytes N
adds one plain device copy of N bytes after the timed steps: the
calibration kernel of those counter runs.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic cost of one query-sample pair in the float32 sweep: 3 sub, 1 mul,
# 2 fma (4 flops), sqrt, sub (s - d), add (s + d), max, min.
FLOP_PER_PAIR = 13
FP32_VECTOR_PEAK = 157.3e12  # MI355X published float32 vector peak, FLOP/s
BATCH_COUNT = 64
BATCH_GRIDS = (4, 5, 6)
REPAIR_GRID = 48
REPAIR_QUERIES = 50000


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "sweep_traffic_balls64.md")
SWEEP_SOURCE = os.path.join(ROOT, "paper_2605_01919_amd", "csrc", "bounds.hip")


# the greedy's named work counters (sdfi_counter_query), reported with --counters
GREEDY_COUNTERS = (
    "greedy_cover_ticks", "greedy_vnew_ticks", "greedy_threat_ticks", "greedy_reval_ticks", "greedy_threatened",
    "rmin_scan_ticks", "rmin_ray_ticks", "rmin_list_ticks", "rmin_search_ticks", "rmin_calls", "rmin_passes",
    "rmin_list_len", "rmin_local_len", "rmin_searches", "ln_early", "ln_first", "ln_loop", "ln_rounds",
    "ln_fallback", "ln_first_ticks", "ln_loop_ticks", "ln_fallback_ticks", "ln_early_ticks", "rmin_wide_passes",
    "rmin_open_passes", "rmin_pre_held", "rmin_pull_ticks", "exist_walks", "greedy_instance_max_ticks")


def recorded_traffic():
    """HBM bytes per sweep launch from the recorded counter runs, or None when
    the sweep's source changed since they were taken."""
    try:
        text = open(TRAFFIC_FILE).read()
        src = hashlib.sha256(open(SWEEP_SOURCE, "rb").read()).hexdigest()
    except OSError:
        return None
    sha = re.search(r"bounds\.hip sha256: ([0-9a-f]{64})", text)
    val = re.search(r"traffic_bytes_per_launch: ([0-9]+)", text)
    if not sha or not val or sha.group(1) != src:
        return None
    return int(val.group(1))


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(w, sample_queries=4500):
    """The oracle's bound definition timed on a bounded sample of queries."""
    from oracle import bounds as OB
    q = w.queries[np.random.default_rng(0).choice(w.m, sample_queries, replace=False)]
    t0 = time.perf_counter()
    OB.cone_bounds(w.points, w.values, q, chunk=64)
    dt = time.perf_counter() - t0
    pairs = sample_queries * w.n
    return {"value": round(pairs / dt / 1e9, 4), "unit": "G pair-evals/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample_queries} seeded random queries of balls64 x all {w.n} samples, numpy float64 "
                      f"on one thread, {dt:.1f} s"}


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


def wall(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def measure_csg(grid=96, save=None):
    """The pseudo-SDF repair workload (CSG samples on a grid^3 grid; at 96 the
    full recipe with 400 000 scattered extension queries, at smaller grids the
    query count scaled by (grid/96)^3), timed in parts so that no single GPU
    call runs for minutes: (1) sdfi_repair on the samples (witness of every sample, removal
    of the fully covered ones, minimum valid radius of the removed points);
    (2) the extension queries' minimum valid radius against the kept samples
    (the same values the repair gives them), in chunks of 50 000 through
    sdfi_min_valid_radius, whose own witness pass over the kept samples is
    timed apart and not counted.  Kernel times come from the library's HIP
    event timers on the launch stream.  Prints one JSON line."""
    import torch
    from paper_2605_01919_amd import sdfi
    from sdfgen import configs
    dev = torch.device("cuda:0")
    half = int(round(200000 * (grid / 96) ** 3))
    w = configs.csg(grid, uniform_queries=half, near_queries=half)
    samples = torch.tensor(np.c_[w.points, w.values], device=dev)
    progress(f"csg{grid}: {w.n} samples, {w.m} queries generated")
    sdfi.timing(True)
    (rv, removed, _, kind, rep), t_rep = wall(lambda: sdfi.repair(samples))
    kt = sdfi.timing_read()
    sdfi.timing(False)
    progress(f"repair of the samples: {t_rep:.1f} s, {int(rep['n_removed'])} removed; witness kernel "
             f"{kt['witness'][0]:.0f} ms, minimum radius of removed points {kt['rmin'][0]:.0f} ms")
    keep = removed == 0
    base = samples[keep].contiguous()
    q_ms = 0.0
    q_wall = 0.0
    qkinds = []
    qvals = []
    for c0 in range(0, w.m, 50000):
        q = torch.tensor(w.queries[c0:c0 + 50000], device=dev)
        sdfi.timing(True)
        (val, k, _), tq = wall(lambda: sdfi.min_valid_radius(base, q))
        kq = sdfi.timing_read()
        sdfi.timing(False)
        q_ms += kq["rmin"][0]
        q_wall += tq - kq["witness"][0] * 1e-3
        qkinds.append(k.cpu().numpy())
        qvals.append(val.cpu().numpy())
        progress(f"extension queries {c0 + len(q)}/{w.m}: radius kernel {kq['rmin'][0]:.0f} ms")
    qk = np.concatenate(qkinds)
    total_s = t_rep + q_wall
    out = {"workload": f"csg{grid}: CSG pseudo-SDF of 16 primitives, {grid}^3 samples + {w.m} scattered queries "
                       "(half uniform, half near the zero set)",
           "samples": w.n, "queries": w.m, "removed": int(rep["n_removed"]),
           "repair_samples_s": round(t_rep, 3), "witness_kernel_ms": round(kt["witness"][0], 1),
           "removed_radius_kernel_ms": round(kt["rmin"][0], 1), "query_radius_kernel_ms": round(q_ms, 1),
           "total_s": round(total_s, 3), "points_per_s": round((int(rep["n_removed"]) + w.m) / total_s, 1),
           "query_kinds": {int(a): int(b) for a, b in zip(*np.unique(qk, return_counts=True))},
           "unresolved": int((qk == 255).sum() + (kind.cpu().numpy() == 255).sum())}
    if save:
        rng = np.random.default_rng(3003)
        qi = np.sort(rng.choice(w.m, 256, replace=False))
        si = np.sort(rng.choice(w.n, 512, replace=False))
        np.savez(save, P=w.points, S=w.values, Q=w.queries[qi], qidx=qi, qvals=np.concatenate(qvals)[qi],
                 qkind=qk[qi], sidx=si, removed=removed.cpu().numpy(), repaired=rv.cpu().numpy())
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-greedy", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-repair", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0)
    ap.add_argument("--counters", action="store_true",
                    help="run the greedy leg with the library's timers on and report its work counters")
    ap.add_argument("--csg", type=int, default=0,
                    help="only time the pseudo-SDF repair workload on a CSG^3 grid in parts (96: the full recipe)")
    ap.add_argument("--save", default=None, help="with --csg: save a seeded sample of the outputs (npz)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the hot path runs on a "
              "single MI355X (how it would shard across GPUs is described in the design notes)",
              file=sys.stderr)
        sys.exit(2)

    if args.csg:
        measure_csg(args.csg, args.save)
        return

    import torch
    from paper_2605_01919_amd import sdfi
    from sdfgen import configs

    dev = torch.device("cuda:0")
    w = configs.by_name("balls64")
    samples = torch.tensor(np.c_[w.points, w.values], device=dev)
    queries = torch.tensor(w.queries, device=dev)
    n, m = w.n, w.m

    def step():
        sdfi.bounds(samples, queries, "fp32")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sdfi.timing(True)  # kernel timers (HIP events on the launch stream) over the timed steps only
    ms = timed(step, args.steps, 0)
    kt = sdfi.timing_read()
    skipped = sdfi.counter_read("sweep_pairs_skipped")
    sdfi.timing(False)
    launches = max(kt["sweep"][1], 1)
    sweep_ms = kt["sweep"][0] / launches
    resolve_ms = kt["resolve"][0] / max(kt["resolve"][1], 1)
    pairs = n * m
    # pairs the sweep evaluated per launch: the rest were ruled out a tile at a
    # time (box gap and value range) and count as avoided work, not as flops
    evaluated = pairs - skipped // launches
    achieved = FLOP_PER_PAIR * evaluated / (sweep_ms * 1e-3)
    progress(f"bounds balls64: {ms:.2f} ms/step, sweep kernel {sweep_ms:.2f} ms ({evaluated / pairs:.3f} of the "
             f"pairs evaluated), resolve {resolve_ms:.2f} ms")
    if args.copy_bytes > 0:
        src_buf = torch.ones(args.copy_bytes, dtype=torch.uint8, device=dev)
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        progress(f"plain copy of {args.copy_bytes} bytes done")
        del src_buf, dst_buf
    out = {
        "metric": "G query-sample bound evals/s + queries/s, batched vs plain, at 1e-5 abs",
        "value": round(evaluated / (ms * 1e-3) / 1e9, 2), "unit": "G pair-evals/s",
        "value_basis": "query-sample pairs the sweep evaluated per step / whole step time (extent, sorts, "
                       "packing, sweep with float64 resolve, overflow resolve); the other pairs it ruled out a "
                       "tile or block at a time, and the results equal those of the full sweep",
        "pairs_evaluated": evaluated, "evaluated_per_s_G": round(evaluated / (sweep_ms * 1e-3) / 1e9, 2),
        "evaluated_per_s_basis": "pairs evaluated / the sweep kernel's own duration",
        "dense_equivalent_per_s_G": round(pairs / (ms * 1e-3) / 1e9, 2),
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "fp32+fp64",
        "data": "synthetic",
        "config": {"workload": "balls64: 8-ball union SDF, 64^3 samples x 128^3 refinement queries",
                   "samples": n, "queries": m, "pairs": pairs,
                   "step": "sdfi_bounds: float32 sweep + float64 tie resolution"},
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 2), "peak": FP32_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_VECTOR_PEAK, 4), "traffic": recorded_traffic(),
                     "kernel": "sweep_sorted_kernel", "kernel_ms": round(sweep_ms, 3),
                     "flop_per_launch": FLOP_PER_PAIR * evaluated, "evaluated_pairs_per_launch": evaluated,
                     "dense_pairs_per_launch": pairs,
                     "frac_basis": "13 FLOP per evaluated pair over the sweep's duration; the pairs it rules out "
                                   "a tile or block at a time are avoided work and not counted"},
    }
    if not args.no_greedy:
        c1 = configs.by_name("sphere16")
        s1 = torch.tensor(np.c_[c1.points, c1.values], device=dev)
        q1 = torch.tensor(c1.queries, device=dev)
        if args.counters:
            sdfi.timing(True)
        g, gt = wall(lambda: sdfi.greedy(s1, q1, grid=c1.grid, certify=True))
        rep = g["report"]
        counters = None
        if args.counters:
            khz = sdfi.counter_read("wall_clock_khz") or 100000
            counters = {}
            for name in GREEDY_COUNTERS:
                v = sdfi.counter_read(name)
                counters[name] = round(v / khz, 1) if name.endswith("_ticks") else v
            sdfi.timing(False)
            progress("greedy counters: " + json.dumps(counters))
        bad = rep["n_violations_pairwise"] + rep["n_violations_witness"]
        progress(f"greedy sphere16: {gt:.1f} s, {c1.m / gt:.0f} queries/s, violations {bad}, "
                 f"capped searches {rep['n_search_capped']}")
        if rep["n_search_capped"]:
            progress("WARNING: some exact searches hit their cap; those queries are UNRESOLVED")
        # gradient of sum(values) w.r.t. the samples through the active parents (extension)
        ones = torch.ones(c1.m, dtype=torch.float64, device=dev)
        _, bt = wall(lambda: sdfi.greedy_backward(ones, s1, q1, g["values"], g["active"], g["kind"]))
        progress(f"backward sphere16: {bt * 1e3:.2f} ms")
        out["greedy"] = {
            "workload": "sphere16: sphere SDF, 16^3 samples, 32^3 refinement queries, float64",
            "queries": c1.m, "samples": c1.n, "seconds": round(gt, 3), "queries_per_s": round(c1.m / gt, 1),
            "ms": {"order": round(rep["ms_phase"][0], 1), "witnesses": round(rep["ms_phase"][1], 1),
                   "greedy": round(rep["ms_phase"][2], 1), "certificate": round(rep["ms_phase"][3], 1)},
            "device_ms": {"bounds": round(rep["ms_phase"][4], 1), "candidates": round(rep["ms_phase"][5], 1),
                          "rmin": round(rep["ms_phase"][6], 1), "record": round(rep["ms_phase"][7], 1)},
            "greedy_dense_pairs": rep["pairs_evaluated"], "violations": bad,
            "exact_searches": rep["n_exact_searches"], "searches_capped": rep["n_search_capped"],
            "unresolved": rep["n_unresolved"], "infeasible": rep["n_infeasible"],
            "kinds": {"hi": rep["n_hi"], "lo": rep["n_lo"], "zero": rep["n_zero"], "rmin": rep["n_rmin"],
                      "coincident": rep["n_coincident"]},
            "backward_ms": round(bt * 1e3, 3)}
        if counters is not None:
            out["greedy"]["counters"] = counters
            out["greedy"]["counters_basis"] = ("library work counters of the run (*_ticks: ms of the device clock, "
                                               "summed over wavefronts for ln_* and rmin_pull_ticks)")
    if not args.no_greedy and not args.no_batched:
        inst = configs.batch(BATCH_COUNT, grids=BATCH_GRIDS)
        tens = [(torch.tensor(np.c_[x.points, x.values], device=dev), torch.tensor(x.queries, device=dev), x.grid)
                for x in inst]
        bo, tb = wall(lambda: sdfi.greedy_batched(tens))
        progress(f"batched {BATCH_COUNT} instances: {tb:.1f} s")

        def plain():
            return [sdfi.greedy(s_, q_, grid=g_) for s_, q_, g_ in tens]
        po, tp = wall(plain)
        same = bool(torch.equal(torch.nan_to_num(bo["values"], nan=7.0),
                                torch.nan_to_num(torch.cat([p["values"] for p in po]), nan=7.0)))
        mq = sum(x.m for x in inst)
        progress(f"plain {BATCH_COUNT} instances: {tp:.1f} s (batched values identical: {same})")
        out["batched"] = {"workload": f"{BATCH_COUNT} sphere/box unions, grids drawn from {list(BATCH_GRIDS)}^3, "
                                      "2x refinement queries",
                          "queries": mq, "batched_s": round(tb, 3), "plain_s": round(tp, 3),
                          "batched_queries_per_s": round(mq / tb, 1), "plain_queries_per_s": round(mq / tp, 1),
                          "speedup": round(tp / tb, 2), "identical_values": same}
    if not args.no_greedy and not args.no_repair:
        c3 = configs.csg(grid=REPAIR_GRID, uniform_queries=REPAIR_QUERIES // 2, near_queries=REPAIR_QUERIES // 2)
        s3 = torch.tensor(np.c_[c3.points, c3.values], device=dev)
        q3 = torch.tensor(c3.queries, device=dev)
        r3, rt = wall(lambda: sdfi.repair(s3, q3))
        rr = r3[-1]
        progress(f"repair csg{REPAIR_GRID}: {rt:.2f} s, {int(rr['n_removed'])} samples removed")
        out["repair"] = {"workload": f"CSG pseudo-SDF of 16 primitives, {REPAIR_GRID}^3 samples + {c3.m} scattered "
                                     "queries (half uniform, half near the zero set)",
                         "samples": c3.n, "queries": c3.m, "seconds": round(rt, 3),
                         "points_per_s": round((c3.n + c3.m) / rt, 1), "removed": int(rr["n_removed"]),
                         "ms": {"witnesses": round(rr["ms_phase"][0], 1), "removal": round(rr["ms_phase"][1], 1),
                                "rmin": round(rr["ms_phase"][2], 1)}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
        progress(f"cpu baseline: {out['cpu_baseline']['value']} G pair-evals/s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
