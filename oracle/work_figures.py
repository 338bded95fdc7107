"""Algorithmic work per cell of the method, measured by the oracle (test
infrastructure: run by hand, its output is quoted in the design notes and in
bench.py's roofline constants).

The algorithmic work of a cell is the work of the method with a list just
long enough: the box is clipped by the nearest neighbours in (d^2, index)
order until the security radius certifies it.  Counted per cell, with the
weights of the hot-path scope's measurement plan: vertex-vs-plane evaluations
(7 flops each: n.v - c and the sign), vertices created (40 flops each: the
solve of a vertex from three planes) and R^2 updates (5 flops per vertex
norm evaluated after a cut).  Work the GPU spends on lists that fail, on
retries or on its stream phase is overhead, not algorithmic work.

    python -m oracle.work_figures cluster-16m-f32 20000
"""
from __future__ import annotations

import json
import sys
import time

import numpy as np

import oracle
from paper_2412_04514_amd import gen

FLOPS_PER_EVAL = 7
FLOPS_PER_CREATED = 40
FLOPS_PER_R2 = 5


def figures(name: str, sample: int, seed: int = 0, kcap: int = 16384) -> dict:
    P = gen.make(name, seed=seed).astype(np.float64)
    rng = np.random.default_rng(1234)
    cells = np.sort(rng.choice(len(P), size=min(sample, len(P)), replace=False))
    t = time.time()
    k = oracle.kneeded(P, cells=cells, kcap=kcap, kwork=kcap)
    dt = time.time() - t
    flops = FLOPS_PER_EVAL * k["evals"] + FLOPS_PER_CREATED * k["created"] + FLOPS_PER_R2 * k["r2upd"]
    kn = k["kneeded"]
    return dict(workload=name, n=len(P), sample=len(cells), seconds=dt,
                flops_per_cell=float(flops.mean()), evals_per_cell=float(k["evals"].mean()),
                created_per_cell=float(k["created"].mean()), r2upd_per_cell=float(k["r2upd"].mean()),
                planes_tested_per_cell=float(k["tested"].mean()),
                weights=dict(eval=FLOPS_PER_EVAL, created=FLOPS_PER_CREATED, r2=FLOPS_PER_R2),
                kneeded_median=float(np.median(kn)), kneeded_p99=float(np.percentile(kn, 99)),
                kneeded_max=int(kn.max()),
                frac_le={str(b): float((kn <= b).mean()) for b in (8, 12, 16, 24, 32, 48, 64, 128, 256)})


if __name__ == "__main__":
    name = sys.argv[1] if len(sys.argv) > 1 else "cluster-16m-f32"
    sample = int(sys.argv[2]) if len(sys.argv) > 2 else 20000
    print(json.dumps(figures(name, sample), indent=1))
