"""Launch-shape autotuners: batched reconstructions and the tile walk of one reconstruction.

For every window-size class of a batch the persistent launch can use a
different number of workgroups (the register and LDS budget allows one
128-window workgroup per CU, and up to four 64-window workgroups).  The two
classes run side by side on two streams, so the tuner times one full
loss/gradient pass of the batch for every pair of candidates with HIP events
on the batch stream, keeps the fastest, and caches the choice in a JSON file
keyed by the device and the batch's shape signature, so later runs of the same
shape skip the search.  A class with no reconstruction keeps grid 0 (the
default).
"""
from __future__ import annotations

import hashlib
import json
import os
from typing import Dict, Optional

from .batch import Batch

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ptycho_mi355x", "autotune.json")


def signature(batch: Batch, device_name: str) -> str:
    """Device + per-reconstruction (M, S, H, W, n) list, hashed."""
    shapes = [(r.probe.shape[0], r.obj.shape[0], r.obj.shape[1], r.obj.shape[2], r.pos.shape[0])
              for r in batch.recons]
    h = hashlib.sha1(json.dumps([device_name, shapes]).encode()).hexdigest()[:16]
    return f"{device_name}:{h}"


def _time_pass(batch: Batch, reps: int) -> float:
    import torch
    stream = torch.cuda.ExternalStream(batch.stream_ptr)
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    batch.loss_grad()  # warm
    start.record(stream)
    for _ in range(reps):
        batch.loss_grad()
    stop.record(stream)
    stop.synchronize()
    return start.elapsed_time(stop) / reps


def tune(batch: Batch, reps: int = 3, cache_path: Optional[str] = DEFAULT_CACHE, use_cache: bool = True,
         rounds: int = 3) -> Dict:
    """Pick the workgroup count of each window-size class; returns {M: grid, "ms": best pass time}.

    Every candidate pair is timed once per round, the rounds interleaving the pairs, and the pair with
    the lowest median wins: neighbouring candidates differ by a few percent, about the spread of a
    single timing."""
    import torch
    dev = torch.cuda.get_device_properties(0)
    cus = dev.multi_processor_count
    key = signature(batch, dev.name)
    cache = {}
    if cache_path and use_cache and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        choice = cache[key]
        for M in (64, 128):
            batch.set_grid(M, int(choice[str(M)]))
        return {64: int(choice["64"]), 128: int(choice["128"]), "ms": choice["ms"], "cached": True}
    # the two window sizes run side by side, so their workgroup counts are tuned jointly
    cand = {64: [cus, 2 * cus, 3 * cus, 4 * cus], 128: [cus // 2, cus]}
    present = {M: any(r.probe.shape[0] == M for r in batch.recons) for M in (64, 128)}
    for M in (64, 128):
        cand[M] = sorted({max(1, min(g, 2 * cus * (2 if M == 64 else 1))) for g in cand[M]}) if present[M] else [0]
    pairs = [(g64, g128) for g64 in cand[64] for g128 in cand[128]]
    times = {p: [] for p in pairs}
    for _ in range(max(1, int(rounds))):
        for g64, g128 in pairs:
            batch.set_grid(64, g64)
            batch.set_grid(128, g128)
            times[(g64, g128)].append(_time_pass(batch, reps))
    g64, g128 = min(pairs, key=lambda p: (sorted(times[p])[len(times[p]) // 2], p))
    best = {64: g64, 128: g128}
    for M in (64, 128):
        batch.set_grid(M, best[M])
    t_best = _time_pass(batch, reps)
    result = {"64": best[64], "128": best[128], "ms": t_best}
    if cache_path:
        cache[key] = result
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {64: best[64], 128: best[128], "ms": t_best, "cached": False}


# ---------------------------------------------------------------------------
# tile walk of one large reconstruction: walk shape and wave checkpoint interval
# ---------------------------------------------------------------------------
def walk_signature(ctx, plan, device_name: str) -> str:
    """Device + window size, slices, object, tile grid, halo and the per-tile position counts, hashed."""
    shape = [ctx.M, ctx.S, plan.H, plan.W, list(plan.tiles), plan.halo, [p.hi - p.lo for p in plan.plans]]
    h = hashlib.sha1(json.dumps([device_name, shape]).encode()).hexdigest()[:16]
    return f"{device_name}:walk:{h}"


def _make_walk(ctx, plan, kind: str, lanes: int):
    from .tilewalk import AllTilesWalk, ResidentTileWalk
    if kind == "all":
        return AllTilesWalk(ctx, plan)
    return ResidentTileWalk(ctx, plan, lanes=lanes)


def tune_walk(ctx, plan, obj, probe, meas_sorted, grad, reps: int = 3, rounds: int = 2,
              checkpoints=(1, 2, 4), lanes=(1, 2, 3), cache_path: Optional[str] = DEFAULT_CACHE,
              use_cache: bool = True) -> Dict:
    """Pick the tile walk of a decomposed gradient step: every tile in one launch ("all") or one launch
    per tile on 1-3 alternating lanes ("lanes"), and the interval k at which the fused kernel keeps
    incident waves (the others are recomputed in the adjoint sweep).  Each candidate's step is timed
    with HIP events over `reps` steps, once per round (rounds interleave the candidates); the lowest
    median wins and is applied to ctx (ptycho_set_checkpoint).  Returns {"walk", "lanes",
    "checkpoint", "ms", "timings", "cached"}; the choice is cached per device and shape."""
    import torch
    dev = torch.cuda.get_device_properties(0)
    key = walk_signature(ctx, plan, dev.name)
    cache = {}
    if cache_path and use_cache and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        c = cache[key]
        ctx.set_checkpoint(int(c["checkpoint"]))
        return {**c, "cached": True}
    cands = [("all", 1, k) for k in checkpoints] + [("lanes", n, k) for n in lanes for k in checkpoints]
    times = {c: [] for c in cands}
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(max(1, int(rounds))):
        for kind, n, k in cands:
            ctx.set_checkpoint(k)
            walk = _make_walk(ctx, plan, kind, n)
            walk.step(obj, probe, meas_sorted, grad)  # warm (and the lanes' contexts take k)
            torch.cuda.synchronize()
            start.record()
            for _ in range(reps):
                walk.step(obj, probe, meas_sorted, grad)
            stop.record()
            stop.synchronize()
            times[(kind, n, k)].append(start.elapsed_time(stop) / reps)
            del walk
    best = min(cands, key=lambda c: (sorted(times[c])[len(times[c]) // 2], c))
    kind, n, k = best
    ctx.set_checkpoint(k)
    result = {"walk": kind, "lanes": n, "checkpoint": k, "ms": sorted(times[best])[len(times[best]) // 2],
              "timings": {f"{c[0]}/{c[1]}/k{c[2]}": round(sorted(v)[len(v) // 2], 3) for c, v in times.items()}}
    if cache_path:
        cache[key] = result
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(tmp, cache_path)
    return {**result, "cached": False}
