"""Writes tests/golden/batch32_gd_trajectory.json: the FP64 oracle's gradient
descent on the 32 uneven reconstructions of the batched workload
(ptycho_synth.batch_specs(4): objects of 256-1024 px, 1-8 slices, 64- or
128-windows, Poisson doses 1e4-1e6).

For every reconstruction: the step length (the oracle's reading of it), the
loss of each of 20 full-batch iterations t <- t - alpha dF/dt (Section II-B),
and a 4 x 4 block of the first iteration's gradient on every slice at the
centre of the scanned area.  Inputs are the seeded generators' arrays with
the object and probe rounded to complex64 (what the GPU receives) and
measurements = Poisson counts of the oracle's intensities at the truth.

Calls only oracle/ and the input generators.  Run from the repository root:
    python tests/golden/make_batch32_trajectory.py --workers 8
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
TESTS = os.path.join(ROOT, "tests")
for p in (ROOT, TESTS):
    if p not in sys.path:
        sys.path.insert(0, p)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch32_gd_trajectory.json")
ITERATIONS = 20
BLOCK = 4


def block_origin(pos, M):
    """Top-left of the 4 x 4 gradient block: the centre of the scanned area."""
    y = (int(pos[:, 0].min()) + int(pos[:, 0].max()) + M) // 2 - BLOCK // 2
    x = (int(pos[:, 1].min()) + int(pos[:, 1].max()) + M) // 2 - BLOCK // 2
    return y, x


def trajectory(spec):
    from threadpoolctl import threadpool_limits

    import oracle
    from oracle_pool import batch_problem  # the inputs the GPU test builds, from the same function
    with threadpool_limits(1):
        p = batch_problem(spec)
        t = p["obj"]
        losses = []
        by, bx = block_origin(p["pos"], spec.M)
        blk = None
        for k in range(ITERATIONS):
            L, _, G = oracle.loss_and_gradient(t, p["probe"], p["pos"], p["meas"], p["H"])
            losses.append(float(L))
            if k == 0:
                blk = G[:, by:by + BLOCK, bx:bx + BLOCK]
            t = oracle.gd_step(t, G, p["alpha"])
    return {"name": spec.name, "M": spec.M, "S": spec.S, "W": spec.W, "n": spec.n, "alpha": p["alpha"],
            "loss": losses, "block_origin": [by, bx],
            "grad_block_re": blk.real.tolist(), "grad_block_im": blk.imag.tolist()}


def main():
    import multiprocessing as mp

    import ptycho_synth as ps
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=8)
    args = ap.parse_args()
    specs = ps.batch_specs(4)
    order = sorted(range(len(specs)), key=lambda r: -specs[r].n * (4 * specs[r].S - 2) * specs[r].M ** 2)
    t0 = time.time()
    with mp.get_context("spawn").Pool(args.workers) as pool:
        res = pool.map(trajectory, [specs[r] for r in order], chunksize=1)
    by_name = {r["name"]: r for r in res}
    out = {
        "what": "FP64 oracle gradient descent on ptycho_synth.batch_specs(4): loss per iteration, step length, "
                "and a 4 x 4 block of the first iteration's gradient on every slice",
        "iterations": ITERATIONS, "block": BLOCK,
        "recons": [by_name[sp.name] for sp in specs],
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s")


if __name__ == "__main__":
    main()
