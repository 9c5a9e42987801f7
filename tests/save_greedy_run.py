"""Runs one greedy interpolation on the GPU and saves what the oracle replay
needs (tests/replay_oracle.py), so that a long replay can run on any host.

    python tests/save_greedy_run.py sphere16 OUT.npz [steps]
    python tests/save_greedy_run.py balls64-subset OUT.npz [steps] [queries]

sphere16: the 16^3 sphere samples and all 32^3 refinement queries.
balls64-subset: the 64^3 eight-ball samples (seed 1002) with a seeded subset
(seed 2002) of the 128^3 refinement queries, as scattered queries in their
bucketed order.  `steps`: how many seeded steps (seed 2016) to mark for the
replay.  Prints the run's report.
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2605_01919_amd import sdfi  # noqa: E402
from sdfgen import configs  # noqa: E402


def main():
    which, out = sys.argv[1], sys.argv[2]
    nsteps = int(sys.argv[3]) if len(sys.argv) > 3 else 500
    dev = torch.device("cuda:0")
    if which == "sphere16":
        w = configs.sphere(16)
        P, S, Q = w.points, w.values, w.queries
        s, q = torch.tensor(np.c_[P, S], device=dev), torch.tensor(Q, device=dev)
        t0 = time.time()
        g = sdfi.greedy(s, q, grid=w.grid, certify=True, sample_witness=True)
    elif which == "balls64-subset":
        count = int(sys.argv[4]) if len(sys.argv) > 4 else 256
        w = configs.ball_union(64, 1002)
        idx = np.sort(np.random.default_rng(2002).choice(w.m, count, replace=False))
        P, S, Q = w.points, w.values, w.queries[idx]
        s, q = torch.tensor(np.c_[P, S], device=dev), torch.tensor(Q, device=dev)
        t0 = time.time()
        order = sdfi.refinement_order(s, w.grid, q)
        g = sdfi.greedy(s, q, order=order, certify=True, sample_witness=True)
    else:
        raise SystemExit(f"unknown run {which}")
    torch.cuda.synchronize()
    print(which, "seconds", round(time.time() - t0, 2), g["report"], flush=True)
    steps = np.sort(np.random.default_rng(2016).choice(len(Q), min(nsteps, len(Q)), replace=False))
    np.savez(out, P=P, S=S, Q=Q, order=g["order"].cpu().numpy(), values=g["values"].cpu().numpy(),
             kind=g["kind"].cpu().numpy(), active=g["active"].cpu().numpy(), SW=g["sample_witness"].cpu().numpy(),
             QW=g["witness"].cpu().numpy(), steps=steps)


if __name__ == "__main__":
    main()
