#!/usr/bin/env python3
"""Throughput of the fused forward + amplitude loss + adjoint gradient path.

One step = the whole hot path over one synthetic scan: for every tile of the
4x4 decomposition, the fused per-position kernel (multislice forward, loss,
adjoint sweep, scatter-add into the tile's extended box) followed by the
stitch of the tile gradient into the global gradient.  Inputs are resident in
HBM when the timed region starts.

Prints one JSON line with probe-positions/s, the roofline of the fused kernel
(timed with HIP events around each of its launches), the unfused torch-eager
("plain") path on the same GPU, the FP64 oracle on the host cores, and the
decomposition checks.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "probe-positions/s, forward+adjoint gradient, fused vs plain; % of HBM roofline"
HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, published
FP32_PEAK_TFLOPS = 157.3          # MI355X FP32 vector, published (packed FMA)
# 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz: the FP32 rate without packed instructions, which the
# kernels are compiled without
FP32_NONPACKED_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
HBM_TARGET_FRAC = 0.5             # planning target of the 16-slice workload


def kernel_source_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("ptycho_kernels.hip", "fft_lds.hpp", "ptycho_kernels.h"):
        with open(os.path.join(ROOT, "paper_2205_06327_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str):
    """HBM bytes per fused launch from the committed counter summary, or None when the kernel changed since."""
    path = os.path.join(ROOT, "profiles", f"fused_kernel_{workload}_hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("source_sha256") != kernel_source_sha256():
        return None
    return rec


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_bytes(M: int, S: int) -> int:
    """Per position: one pattern read (4 B/px), the S object windows read and the S gradient windows written."""
    return M * M * (4 + 16 * S)


def algorithmic_flops(M: int, S: int) -> float:
    """Per position: (4S-2) 2D DFTs at 5 N log2 N plus the pointwise work."""
    N = M * M
    return (4 * S - 2) * 5.0 * N * math.log2(N) + (30 * S + 10) * N


# ---------------------------------------------------------------------------
# unfused comparator: torch eager ops (rocFFT, elementwise, index_add)
# ---------------------------------------------------------------------------
def plain_loss_grad(torch, obj, probe, pos, meas, Hprop, grad, batch):
    """The same forward/loss/adjoint with one torch op per step, batched over positions."""
    S, Hh, Ww = obj.shape
    M = probe.shape[0]
    ar = torch.arange(M, device=obj.device)
    total = torch.zeros((), dtype=torch.float64, device=obj.device)
    flat = [obj[s].reshape(-1) for s in range(S)]
    gflat = [torch.view_as_real(grad[s]).reshape(-1) for s in range(S)]
    Hc = Hprop.conj()
    for b0 in range(0, pos.shape[0], batch):
        p = pos[b0:b0 + batch].long()
        lin = ((p[:, 0, None] + ar)[:, :, None] * Ww + (p[:, 1, None] + ar)[:, None, :]).reshape(-1)
        B = p.shape[0]
        psi = probe.expand(B, M, M)
        psis = []
        phi = None
        for s in range(S):
            psis.append(psi)
            phi = psi * flat[s][lin].view(B, M, M)
            if s + 1 < S:
                psi = torch.fft.ifft2(Hprop * torch.fft.fft2(phi))
        far = torch.fft.fft2(phi)
        mod = far.abs()
        amp = meas[b0:b0 + B].sqrt()
        total += ((mod - amp) ** 2).sum(dtype=torch.float64)
        scale = torch.where(mod > 0, 2.0 * (mod - amp) / torch.where(mod > 0, mod, torch.ones_like(mod)),
                            torch.zeros_like(mod))
        chi = torch.fft.ifft2(scale * far) * float(M * M)
        idx = torch.stack([2 * lin, 2 * lin + 1], dim=1).reshape(-1)
        for s in range(S - 1, -1, -1):
            g = chi * psis[s].conj()
            gflat[s].index_add_(0, idx, torch.view_as_real(g).reshape(-1))
            if s > 0:
                t = flat[s][lin].view(B, M, M)
                chi = torch.fft.ifft2(Hc * torch.fft.fft2(chi * t.conj()))
    return total


# ---------------------------------------------------------------------------
# CPU baseline: the FP64 oracle on a sample of positions, over a process pool
# ---------------------------------------------------------------------------
_CPU = {}


def _cpu_job(i):
    import oracle
    d = _CPU
    y0, x0 = (int(v) for v in d["pos"][i])
    return oracle.position_loss_and_patch_gradients(d["obj"], d["probe"], y0, x0, d["meas"][i], d["H"])[0]


def _cpu_fwd(i):
    import oracle
    d = _CPU
    y0, x0 = (int(v) for v in d["pos"][i])
    far = oracle.exit_waves(d["obj_true"], d["probe"], y0, x0, d["H"])[1]
    return far.real ** 2 + far.imag ** 2


def cpu_baseline(spec, inputs, sample_count, cores):
    import multiprocessing as mp

    import numpy as np

    import oracle
    import ptycho_synth as ps
    from threadpoolctl import threadpool_limits

    pos = inputs["pos"]
    M = spec.M
    idx = np.linspace(0, len(pos) - 1, sample_count).round().astype(int)
    H = oracle.fresnel_propagator(M, spec.wavelength_A, spec.dz_A, spec.pixel_A)
    # workers are forked after this, so they share the objects instead of copying them
    _CPU.update(obj=inputs["obj_eval"], obj_true=inputs["obj_true"], probe=inputs["probe"], H=H,
                pos=np.ascontiguousarray(pos[idx]))
    ctx = mp.get_context("fork")
    chunk = max(1, len(idx) // (4 * cores))
    with threadpool_limits(1):
        with ctx.Pool(cores) as pool:  # untimed: noise-free patterns of the sample's true windows
            I = np.stack(pool.map(_cpu_fwd, range(len(idx)), chunksize=chunk))
    _CPU["meas"] = ps.poisson_counts(I, np.random.SeedSequence(12345))
    with threadpool_limits(1):
        with ctx.Pool(cores) as pool:
            pool.map(_cpu_job, range(min(cores, len(idx))))  # start the workers
            t0 = time.perf_counter()
            pool.map(_cpu_job, range(len(idx)), chunksize=chunk)
            dt = time.perf_counter() - t0
        # one core: the same oracle in this process, single-threaded, on the first positions of the sample
        n1 = min(len(idx), 48)
        _cpu_job(0)
        t1 = time.perf_counter()
        for i in range(n1):
            _cpu_job(i)
        dt1 = time.perf_counter() - t1
    return {"value": len(idx) / dt, "unit": "positions/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(idx)} positions spread evenly over the {len(pos)}-position scan, FP64 numpy oracle "
                      f"(forward + loss + adjoint per position), one single-threaded process per core, "
                      f"{dt:.2f} s wall, {dt * cores:.0f} core-seconds",
            "per_core_value": round(n1 / dt1, 2),
            "per_core_sample": f"{n1} positions in one single-threaded process, {dt1:.2f} s",
            "host_cpu_count": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def run_batch(args, cores):
    """The uneven batch: 32 independent reconstructions, one graph-captured GD iteration per step."""
    import numpy as np
    import torch

    import ptycho_synth as ps
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.autotune import tune
    from paper_2205_06327_amd.batch import Batch, Recon

    dev = torch.device("cuda:0")
    specs = ps.batch_specs(4)
    log(f"generating {len(specs)} reconstructions")
    t0 = time.time()
    recons, total_pos, alg_bytes, alg_flops = [], 0, 0, 0.0
    for sp in specs:
        d = ps.build_inputs(sp, workers=cores)
        probe = torch.tensor(d["probe"], dtype=torch.complex64, device=dev)
        pos = torch.tensor(d["pos"], dtype=torch.int32, device=dev)
        ctx = pt.Context(sp.M, sp.S, sp.wavelength_A, sp.dz_A, sp.pixel_A, max(sp.n, 1))
        I = pt.ptycho_forward(ctx, torch.tensor(d["obj_true"], dtype=torch.complex64, device=dev), probe, pos)
        g = torch.Generator(device=dev)
        g.manual_seed(sp.seed)
        meas = torch.poisson(I, generator=g)
        alpha = pt.gd_step_size(d["probe"], d["pos"], sp.W, sp.W, sp.S)
        recons.append(Recon(torch.tensor(d["obj_eval"], dtype=torch.complex64, device=dev), probe, pos, meas,
                            sp.wavelength_A, sp.dz_A, sp.pixel_A, alpha))
        total_pos += sp.n
        alg_bytes += sp.n * algorithmic_bytes(sp.M, sp.S)
        alg_flops += sp.n * algorithmic_flops(sp.M, sp.S)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s: {total_pos} positions")
    iters = max(args.steps, 1)
    b = Batch(recons, history_rows=iters + args.warmup + 8)
    tuned = tune(b, reps=10, cache_path=None)
    log(f"autotuner: {tuned}")
    start = [r.obj.clone() for r in recons]
    torch.cuda.synchronize()
    b.reset_history()
    b.capture()
    for _ in range(args.warmup):
        b.replay()
    b.sync()
    for r, o in zip(recons, start):  # the timed iterations start from the evaluation point
        r.obj.copy_(o)
    torch.cuda.synchronize()
    b.reset_history()
    b.sync()
    t0 = time.perf_counter()
    for _ in range(iters):
        b.replay()
    b.sync()
    dt = time.perf_counter() - t0
    hist = b.history()
    total = hist.sum(axis=1)
    ms = dt * 1e3 / iters
    value = total_pos / (ms / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1, "steps": iters,
        "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch32-uneven", "reconstructions": len(specs), "positions": total_pos,
                   "windows": sorted({sp.M for sp in specs}), "slices": sorted({sp.S for sp in specs}),
                   "step": "one hipGraph-captured gradient-descent iteration over all reconstructions"},
        "autotuner": {"grid_m64": tuned[64], "grid_m128": tuned[128]},
        "algorithmic_TFLOPs": round(alg_flops / (ms / 1e3) / 1e12, 3),
        "algorithmic_GBs": round(alg_bytes / (ms / 1e3) / 1e9, 1),
        "loss_first": float(total[0]), "loss_last": float(total[-1]),
        "loss_monotone": bool(np.all(np.diff(total) < 0)),
    }
    print(json.dumps(out), flush=True)


def run_alg1(args, cores):
    """Alg. 1 over 2 x 2 tiles of the 8-slice 1024^2 scan with delayed accumulation: the loss per
    iteration when the passes run after every batch of positions, twice per iteration and once per
    iteration (the three communication frequencies the paper compares), and the rate of the iteration."""
    import numpy as np
    import torch

    import ptycho_synth as ps
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import Alg1Walk, TileWalk

    dev = torch.device("cuda:0")
    spec = ps.with_overrides(ps.workload("ms8-1024-m128"), tiles=(2, 2), halo=64)
    M, S, W = spec.M, spec.S, spec.W
    log(f"generating {spec.name}: {S} x {W}^2, {spec.n} positions, 2 x 2 tiles")
    inputs = ps.build_inputs(spec, workers=cores)
    plan = TileWalk(inputs["pos"], W, W, M, spec.tiles, spec.halo)
    ctx = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, max_positions=spec.n)
    probe = torch.tensor(inputs["probe"], dtype=torch.complex64, device=dev)
    pos_sorted = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=dev)
    I = pt.ptycho_forward(ctx, torch.tensor(inputs["obj_true"], dtype=torch.complex64, device=dev), probe, pos_sorted)
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed)
    meas = torch.poisson(I, generator=gen)
    del I
    obj0 = torch.tensor(inputs["obj_eval"], dtype=torch.complex64, device=dev)
    alpha = 0.5 * pt.gd_step_size(inputs["probe"], inputs["pos"], W, W, S)
    batch = 64  # positions per tile per update: 16 updates per tile per iteration
    iters = max(args.steps, 1)
    counts = [p.hi - p.lo for p in plan.plans]
    steps = max((c + batch - 1) // batch for c in counts)
    curves, ms = {}, {}
    for label, T in (("every batch", 1), ("twice per iteration", (steps + 1) // 2), ("once per iteration", steps)):
        walk = Alg1Walk(ctx, plan, obj0, probe, meas, alpha, batch, T, device=dev)
        for _ in range(args.warmup):  # warm-up on a copy of the start, then restart
            walk.iteration()
        walk = Alg1Walk(ctx, plan, obj0, probe, meas, alpha, batch, T, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        losses = [walk.iteration() for _ in range(iters)]
        torch.cuda.synchronize()
        ms[label] = (time.perf_counter() - t0) * 1e3 / iters
        assert walk.check() == 0
        curves[label] = [float(v.item()) for v in losses]
        log(f"T = {T} ({label}): {ms[label]:.2f} ms/iteration, loss {curves[label][0]:.4g} -> {curves[label][-1]:.4g}")
    once = "once per iteration"
    value = spec.n / (ms[once] / 1e3)
    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1, "steps": iters,
        "warmup": args.warmup, "ms_per_step": round(ms[once], 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "alg1-ms8-1024-m128-tiles2x2", "positions": spec.n, "slices": S,
                   "object": [W, W], "window": M, "tiles": [2, 2], "halo": spec.halo, "batch_per_tile": batch,
                   "updates_per_tile_per_iteration": steps,
                   "step": "one Alg. 1 iteration: every tile's positions in batches, tile updates, passes"},
        "convergence": {label: {"T_batches": T, "loss_per_iteration": curves[label],
                                "ms_per_iteration": round(ms[label], 3)}
                        for label, T in (("every batch", 1), ("twice per iteration", (steps + 1) // 2),
                                         ("once per iteration", steps))},
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="ms16-2048-m128-tiles4x4")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-checks", action="store_true", help="skip the undecomposed and streaming comparisons")
    ap.add_argument("--plain-positions", type=int, default=1024)
    ap.add_argument("--cpu-sample", type=int, default=3072)
    ap.add_argument("--lanes", type=int, default=2, help="streams the resident tile walk alternates between")
    ap.add_argument("--walk", choices=("all", "lanes"), default="all",
                    help="all: every tile's gradient in one launch; lanes: one launch per tile on alternating streams")
    ap.add_argument("--checkpoint", type=int, default=1,
                    help="keep every k-th incident wave, recompute the others in the adjoint sweep")
    ap.add_argument("--no-walk-tune", action="store_true", help="skip the walk-shape autotuner report")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy three times (HBM counter calibration) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        msg = ("this benchmark runs on one GPU only: the decomposed tile walk is measured on a single MI355X; "
               "multi-GPU tile exchange is not implemented")
        print(msg, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read_per_copy": src.numel() * 4,
                          "bytes_written_per_copy": dst.numel() * 4, "copies": 3}))
        return

    import paper_2205_06327_amd as pt
    import ptycho_synth as ps
    from paper_2205_06327_amd.tilewalk import (AllTilesWalk, DecomposedTileWalk, ResidentTileWalk,
                                               StreamingTileWalk, TileWalk)

    dev = torch.device("cuda:0")
    cores_avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(16, cores_avail))
    if args.workload == "batch32-uneven":
        return run_batch(args, cores)
    if args.workload == "alg1-convergence":
        return run_alg1(args, cores)
    spec = ps.workload(args.workload)
    M, S, W = spec.M, spec.S, spec.W
    log(f"generating {spec.name}: {S} x {W}^2 object, {spec.n} positions, M={M} ({cores} workers)")
    t0 = time.time()
    inputs = ps.build_inputs(spec, workers=cores)
    log(f"inputs ready in {time.time() - t0:.1f} s")
    cpu = None
    if not args.no_cpu_baseline:
        # before the GPU is initialised, so the worker processes fork a GPU-free parent
        log(f"cpu baseline: oracle on {args.cpu_sample} positions over {cores} processes")
        cpu = cpu_baseline(spec, inputs, args.cpu_sample, cores)
        log(f"cpu baseline {cpu['value']:.1f} positions/s")

    plan = TileWalk(inputs["pos"], W, W, M, spec.tiles, spec.halo)
    ctx = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, max_positions=spec.n)
    if args.checkpoint != 1:
        ctx.set_checkpoint(args.checkpoint)
    probe = torch.tensor(inputs["probe"], dtype=torch.complex64, device=dev)
    pos_sorted = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=dev)
    obj_true = torch.tensor(inputs["obj_true"], dtype=torch.complex64, device=dev)
    # measurements: Poisson counts of the noise-free intensities at the truth
    I_true = pt.ptycho_forward(ctx, obj_true, probe, pos_sorted)
    gen = torch.Generator(device=dev)
    gen.manual_seed(spec.seed)
    meas = torch.poisson(I_true, generator=gen)
    del I_true, obj_true
    obj = torch.tensor(inputs["obj_eval"], dtype=torch.complex64, device=dev)
    grad = torch.empty((S, W, W), dtype=torch.complex64, device=dev)
    if args.walk == "all":
        walk = AllTilesWalk(ctx, plan, device=dev)
    else:
        walk = ResidentTileWalk(ctx, plan, device=dev, lanes=args.lanes)
    walk.check()
    torch.cuda.synchronize()

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        walk.step(obj, probe, meas, grad)
    torch.cuda.synchronize()
    walk.profile(True)
    walk.profile_read()
    log(f"timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        loss_tiles = walk.step(obj, probe, meas, grad)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    k_ms, k_launches, k_pos = walk.profile_read()
    walk.profile(False)
    walk.check()
    loss_total = float(loss_tiles.sum().item())
    ms_per_step = dt * 1e3 / args.steps
    value = spec.n / (ms_per_step / 1e3)
    log(f"{ms_per_step:.3f} ms/step, {value:.4g} positions/s; fused kernel {k_ms / max(k_launches, 1):.3f} ms/launch")

    Bpos = algorithmic_bytes(M, S)
    Fpos = algorithmic_flops(M, S)
    k_s = k_ms / 1e3
    per_launch = k_pos / max(k_launches, 1)
    gbs = k_pos * Bpos / k_s / 1e9
    tflops = k_pos * Fpos / k_s / 1e12
    roofline = {
        "bound": "hbm",
        "achieved": round(gbs, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(gbs / HBM_PEAK_GBS, 4),
        "traffic": None,
        "kernel": f"fused_kernel<{M}, 2> (loss + gradient)",
        "avg_launch_ms": round(k_ms / max(k_launches, 1), 4),
        "launches": k_launches,
        "positions_per_launch": round(per_launch, 1),
        "algorithmic_bytes_per_position": Bpos,
        "algorithmic_flops_per_position": Fpos,
        "hbm_target_frac": HBM_TARGET_FRAC,
        "hbm_target_met": bool(gbs / HBM_PEAK_GBS >= HBM_TARGET_FRAC),
        # the same launches against the FP32 vector peaks: the published (packed FMA) one and the rate
        # without packed instructions
        "fp32_tflops": round(tflops, 3),
        "frac_vs_fp32_peak": round(tflops / FP32_PEAK_TFLOPS, 4),
        "frac_vs_fp32_nonpacked_peak": round(tflops / FP32_NONPACKED_PEAK_TFLOPS, 4),
        # hardware float atomics of the gradient scatter (2 S M^2 per position)
        "gradient_atomics_per_s": round(k_pos * 2 * S * M * M / k_s, 1),
    }
    # the same algorithmic work over the wall time of the whole step (zeroing and stitches included)
    roofline["step_GBs"] = round(spec.n * Bpos / (ms_per_step / 1e3) / 1e9, 1)
    roofline["step_frac"] = round(roofline["step_GBs"] / HBM_PEAK_GBS, 4)
    hbm_roofline_pos = HBM_PEAK_GBS * 1e9 / Bpos
    tr = measured_traffic(spec.name)
    if tr is not None:
        traffic = tr["traffic_bytes_per_dispatch"]
        roofline["traffic"] = round(traffic)
        roofline["traffic_bytes_per_position"] = round(traffic / per_launch)
        roofline["traffic_over_algorithmic"] = round(traffic / (per_launch * Bpos), 3)

    out = {
        "metric": METRIC, "value": round(value, 1), "unit": "positions/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": spec.name, "positions": spec.n, "slices": S, "object": [W, W], "window": M,
                   "tiles": list(spec.tiles), "halo": spec.halo, "step_px": spec.step, "dose": spec.dose,
                   "wave_checkpoint_interval": args.checkpoint,
                   "walk": "all tiles in one launch" if args.walk == "all" else f"{args.lanes} lanes"},
        "hbm_roofline_positions_per_s": round(hbm_roofline_pos, 1),
        "hbm_roofline_frac_of_step": round(value / hbm_roofline_pos, 4),
        "roofline": roofline,
        "loss": loss_total,
        # context only: the paper's time-to-solution on its own workload and machine
        "paper_context": {
            "reported": "2.2 min for 100 iterations over 16632 positions on 4158 V100 GPUs (Summit)",
            "position_iterations_per_s": round(16632 * 100 / 132.0, 1),
            "their_workload": "1024^2 windows, 100 slices, 3072^2 object",
            "transform_work_per_position_vs_this_workload": round(
                (4 * 100 - 2) * (1024 ** 2) * 20 / ((4 * S - 2) * (M * M) * math.log2(M * M)), 1),
        },
    }

    if not args.no_checks:
        log("undecomposed gradient for the decomposition check")
        gfull = torch.empty_like(grad)
        loss_full, _ = pt.ptycho_loss_grad(ctx, obj, probe, pos_sorted, meas, grad=gfull)
        torch.cuda.synchronize()
        diff = float(torch.linalg.vector_norm(gfull - grad) / torch.linalg.vector_norm(gfull))
        out["decomposition"] = {
            "rel_l2_decomposed_vs_undecomposed": diff,
            "loss_rel_diff": abs(float(loss_full.item()) - loss_total) / abs(loss_total),
            "undecomposed_gradient_bytes": gfull.numel() * 8,
            "tile_gradient_bytes": int(max(p.box[2] * p.box[3] for p in plan.plans) * S * 8),
            "walk": args.walk,
            "walk_tile_buffers_bytes": int(sum(b.numel() * 8 for b in (walk.bufs if args.walk == "all"
                                                                       else walk.tile_bufs))),
        }
        # per-tile accumulated-gradient buffers and the directional passes between them
        log("per-tile buffers and directional passes")
        dwalk = DecomposedTileWalk(ctx, plan, device=dev, lanes=args.lanes)
        dwalk.step(obj, probe, meas)
        dwalk.check()
        worst = 0.0
        for k, p in enumerate(plan.plans):
            ey0, ex0, eh, ew = p.box
            ref = gfull[:, ey0:ey0 + eh, ex0:ex0 + ew]
            worst = max(worst, float(torch.linalg.vector_norm(dwalk.bufs[k] - ref) / torch.linalg.vector_norm(ref)))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 5
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dwalk.passes()
        e1.record()
        e1.synchronize()
        pass_ms = e0.elapsed_time(e1) / reps
        ty_n, tx_n = plan.tiles
        out["passes"] = {
            "what": "vertical forward add, vertical backward replace, horizontal forward add, horizontal backward "
                    "replace between separately held tile buffers",
            "exchanges": 2 * (ty_n - 1) * tx_n + 2 * ty_n * (tx_n - 1),
            "ms": round(pass_ms, 4),
            "bytes": dwalk.pass_bytes(),
            "GBs": round(dwalk.pass_bytes() / (pass_ms / 1e3) / 1e9, 1),
            "max_rel_l2_tile_buffer_vs_undecomposed": worst,
            "all_tile_buffers_bytes": dwalk.device_bytes(),
        }
        # Section III's direct exchange with the eight neighbours (exact here: tiles >= 2 halo)
        dwalk.tile_gradients(obj, probe, meas)
        acc = dwalk.neighbour_add()
        dwalk.check()
        worst_n = 0.0
        for k, p in enumerate(plan.plans):
            ey0, ex0, eh, ew = p.box
            ref = gfull[:, ey0:ey0 + eh, ex0:ex0 + ew]
            worst_n = max(worst_n, float(torch.linalg.vector_norm(acc[k] - ref) / torch.linalg.vector_norm(ref)))
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            dwalk.neighbour_add()
        e1.record()
        e1.synchronize()
        nb = sum(1 for ty in range(ty_n) for tx in range(tx_n) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                 if 0 <= ty + dy < ty_n and 0 <= tx + dx < tx_n)
        out["passes"]["neighbour_add"] = {
            "what": "every tile buffer plus its eight direct neighbours' original gradients on the overlaps",
            "exchanges": nb, "ms": round(e0.elapsed_time(e1) / reps, 4),
            "max_rel_l2_vs_undecomposed": worst_n,
        }
        del dwalk, acc, gfull
        # Peak device footprint, the library's workspaces included: the undecomposed gradient (every input
        # resident, one context) against the streaming tile walk (inputs and the global gradient in pinned
        # host memory, the device holding per lane one tile's boxes, patterns and a context).  Each walk is
        # measured as the drop of free device memory (hipMemGetInfo) from before its contexts and buffers
        # exist to after a step.
        log("streaming tile walk (host-resident inputs) and device footprints")
        obj_h = obj.cpu().pin_memory()
        meas_h = meas.cpu().pin_memory()
        grad_h = torch.empty((S, W, W), dtype=torch.complex64).pin_memory()
        del walk
        undec = {"object": obj.numel() * 8, "patterns": meas.numel() * 4, "gradient": grad.numel() * 8,
                 "positions": spec.n * 8, "context_workspace": int(ctx.workspace_bytes())}
        undec["total"] = sum(undec.values())
        footprint = {"undecomposed_resident": undec, "streaming": []}
        for lanes, ck in ((2, 1), (1, 4)):
            # torch's tensors: the peak of torch's allocations over the walk; the library's own device
            # memory (contexts: tables, wave store, partial sums): the drop of free device memory that
            # torch's reserved memory does not account for
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
            alloc0, reserved0 = torch.cuda.memory_allocated(), torch.cuda.memory_reserved()
            torch.cuda.reset_peak_memory_stats()
            free0 = torch.cuda.mem_get_info()[0]
            c0 = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, max_positions=plan.max_count)
            c0.set_checkpoint(ck)
            sw = StreamingTileWalk(plan, c0, device=dev, lanes=lanes)
            sw.step(obj_h, probe, meas_h, grad_h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sw.step(obj_h, probe, meas_h, grad_h)
            torch.cuda.synchronize()
            st_ms = (time.perf_counter() - t0) * 1e3
            torch_peak = torch.cuda.max_memory_allocated() - alloc0
            lib_bytes = (free0 - torch.cuda.mem_get_info()[0]) - (torch.cuda.memory_reserved() - reserved0)
            peak = torch_peak + lib_bytes
            sw.check()
            sdiff = float(torch.linalg.vector_norm(grad_h.to(dev) - grad) / torch.linalg.vector_norm(grad))
            footprint["streaming"].append({
                "lanes": lanes, "wave_checkpoint_interval": ck,
                "ms_per_step_including_pcie": round(st_ms, 2),
                "positions_per_s_including_pcie": round(spec.n / (st_ms / 1e3), 1),
                "device_bytes_accounted": int(sw.device_bytes()),
                "context_workspaces_bytes": int(sum(c.workspace_bytes() for c in sw.ctxs)),
                "device_peak_bytes_measured": int(peak),
                "measured_torch_peak_bytes": int(torch_peak),
                "measured_library_bytes": int(lib_bytes),
                "peak_vs_undecomposed": round(peak / undec["total"], 4),
                "rel_l2_vs_resident": sdiff,
            })
            log(f"streaming, {lanes} lane(s), k = {ck}: {st_ms:.1f} ms, device peak {peak / 1e6:.0f} MB "
                f"(undecomposed {undec['total'] / 1e6:.0f} MB)")
            del sw, c0
        out["footprint"] = footprint
        del obj_h, meas_h, grad_h
        torch.cuda.empty_cache()

    if not args.no_walk_tune:
        # the walk-shape autotuner on this workload (its own context; the timed run above used the defaults)
        from paper_2205_06327_amd.autotune import tune_walk
        log("walk-shape autotuner")
        ctx_t = pt.Context(M, S, spec.wavelength_A, spec.dz_A, spec.pixel_A, max_positions=spec.n)
        out["walk_autotuner"] = tune_walk(ctx_t, plan, obj, probe, meas, grad, reps=3, rounds=2, cache_path=None)
        log(f"walk autotuner: {out['walk_autotuner']['walk']} / {out['walk_autotuner']['lanes']} lane(s) / "
            f"k = {out['walk_autotuner']['checkpoint']}, {out['walk_autotuner']['ms']:.2f} ms per step")
        del ctx_t
        torch.cuda.empty_cache()

    if not args.no_plain:
        npl = min(args.plain_positions, spec.n)
        log(f"plain torch-eager path on {npl} positions")
        Hprop = torch.tensor(np.fft.fftfreq(M, d=spec.pixel_A), dtype=torch.float64)
        Hprop = torch.exp(-1j * math.pi * spec.wavelength_A * spec.dz_A * (Hprop[:, None] ** 2 + Hprop[None, :] ** 2))
        Hprop = Hprop.to(torch.complex64).to(dev)
        sub_pos = pos_sorted[:npl].contiguous()
        sub_meas = meas[:npl].contiguous()
        gplain = torch.zeros_like(grad)
        plain_loss_grad(torch, obj, probe, sub_pos, sub_meas, Hprop, gplain, 128)  # warm-up
        gplain.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lp = plain_loss_grad(torch, obj, probe, sub_pos, sub_meas, Hprop, gplain, 128)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        gf = torch.empty_like(grad)
        lf, _ = pt.ptycho_loss_grad(ctx, obj, probe, sub_pos, sub_meas, grad=gf)
        ctx.profile(True)
        ctx.profile_read()
        pt.ptycho_loss_grad(ctx, obj, probe, sub_pos, sub_meas, grad=gf)
        f_ms, _, _ = ctx.profile_read()
        ctx.profile(False)
        torch.cuda.synchronize()
        out["plain"] = {
            "value": round(npl / tp, 1), "unit": "positions/s", "positions": npl,
            "what": "torch eager: rocFFT fft2/ifft2, elementwise ops and index_add_, batched 128 positions",
            "fused_kernel_positions_per_s_same_subset": round(npl / (f_ms / 1e3), 1),
            "fused_step_over_plain": round(value / (npl / tp), 2),
            "rel_l2_plain_vs_fused_gradient": float(torch.linalg.vector_norm(gplain - gf) /
                                                    torch.linalg.vector_norm(gf)),
            "loss_rel_diff": abs(float(lp.item()) - float(lf.item())) / abs(float(lf.item())),
        }
        del gplain, gf

    if cpu is not None:
        out["cpu_baseline"] = cpu

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
