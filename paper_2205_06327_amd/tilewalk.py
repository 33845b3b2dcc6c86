"""Tile-by-tile gradient decomposition on one GPU (Section III of the paper).

The object gradient and the probe locations are divided into tiles; every
position belongs to exactly one tile (the one holding its window centre, with
no extra positions per tile), each tile accumulates the gradients of its own
positions on its halo-extended box, and the global gradient is the sum of the
tile gradients embedded at their boxes -- the one-device form of the
neighbour-tile gradient addition and of the final stitch of Alg. 1.

Two ways to run a step:

* ``ResidentTileWalk.step``: object, measurements and the global gradient
  live in HBM; each tile reads its box as a strided view, writes its gradient
  into a tile-sized buffer that is then added into the global gradient.
  Consecutive tiles alternate between two lanes (a library context, a stream
  and a tile buffer each), so the next tile's launch fills the CUs that the
  previous tile's last workgroups leave idle; the stitches still run one after
  another, in tile order, because neighbouring boxes overlap.
* ``StreamingTileWalk.step``: object, measurements and the global gradient
  stay in pinned host memory; per tile only the extended box of the object,
  the tile's measurements and positions, its gradient and the global
  gradient's box are on the device (one set, reused tile after tile on one
  stream), so the device footprint is bounded by one tile.

All arithmetic runs in libptycho.so; this module only plans and enqueues.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import List, Tuple

import numpy as np

from . import _binding as B


@dataclass
class TilePlan:
    index: int                       # row-major tile index
    tile: Tuple[int, int, int, int]  # ty0, ty1, tx0, tx1
    box: Tuple[int, int, int, int]   # ey0, ex0, eh, ew
    lo: int                          # first position (in tile order)
    hi: int                          # one past the last position


class TileWalk:
    """Plan of a tile walk: positions reordered by tile and the tile geometry."""

    def __init__(self, pos: np.ndarray, H: int, W: int, M: int, tiles: Tuple[int, int], halo: int):
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.int32).reshape(-1, 2))
        self.H, self.W, self.M, self.halo = int(H), int(W), int(M), int(halo)
        self.tiles = (int(tiles[0]), int(tiles[1]))
        owner = B.bin_positions(pos, H, W, M, *self.tiles)
        self.order = np.argsort(owner, kind="stable").astype(np.int64)
        self.pos_sorted = pos[self.order]
        counts = np.bincount(owner, minlength=self.tiles[0] * self.tiles[1])
        starts = np.concatenate([[0], np.cumsum(counts)])
        self.plans: List[TilePlan] = []
        for ty in range(self.tiles[0]):
            for tx in range(self.tiles[1]):
                k = ty * self.tiles[1] + tx
                tile, (ey0, ey1, ex0, ex1) = B.tile_box(H, W, self.tiles[0], self.tiles[1], ty, tx, halo)
                self.plans.append(TilePlan(k, tile, (ey0, ex0, ey1 - ey0, ex1 - ex0), int(starts[k]),
                                           int(starts[k + 1])))
        self.max_box = (max(p.box[2] for p in self.plans), max(p.box[3] for p in self.plans))
        self.max_count = int(counts.max()) if len(counts) else 0

    @property
    def n(self) -> int:
        return len(self.pos_sorted)


class ResidentTileWalk:
    """Decomposed gradient of a whole scan with every input resident in HBM.

    ``lanes`` contexts/streams/tile buffers are used round-robin over the
    tiles (the first context is the caller's; the others are created with the
    same physics).  Each tile's gradient kernel waits for nothing but the
    previous use of its own lane; each stitch waits for the previous tile's
    stitch.
    """

    def __init__(self, ctx: B.Context, plan: TileWalk, device="cuda:0", lanes: int = 2):
        import torch
        self.ctx, self.plan = ctx, plan
        S = ctx.S
        eh, ew = plan.max_box
        lanes = max(1, int(lanes))
        self.ctxs = [ctx] + [B.Context(ctx.M, ctx.S, *ctx.physics, max_positions=max(plan.max_count, 1))
                             for _ in range(lanes - 1)]
        for c in self.ctxs:
            c.reserve(max(plan.max_count, 1))
        self.streams = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.pos = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=device)
        self.tile_bufs = [torch.empty((S, eh, ew), dtype=torch.complex64, device=device) for _ in range(lanes)]
        self.tile_loss = torch.zeros(len(plan.plans), dtype=torch.float64, device=device)

    @property
    def lanes(self) -> int:
        return len(self.ctxs)

    def device_bytes(self) -> int:
        """Tile buffers plus the contexts' workspaces (the walk's own device memory)."""
        return sum(t.numel() * t.element_size() for t in self.tile_bufs) + sum(c.workspace_bytes()
                                                                               for c in self.ctxs)

    def tile_views(self, k: int):
        """(tile gradient view in tile k's lane buffer, positions, plan) of tile k."""
        p = self.plan.plans[k]
        ey0, ex0, eh, ew = p.box
        buf = self.tile_bufs[k % self.lanes]
        return buf.view(-1)[: self.ctx.S * eh * ew].view(self.ctx.S, eh, ew), self.pos[p.lo:p.hi], p

    def profile(self, enable: bool = True) -> None:
        for c in self.ctxs:
            c.profile(enable)

    def profile_read(self):
        """(fused-kernel ms summed, launches, positions) over all lanes since the last read."""
        tot = [0.0, 0, 0]
        for c in self.ctxs:
            for i, v in enumerate(c.profile_read()):
                tot[i] += v
        return tuple(tot)

    def check(self) -> int:
        """OR of the status words of all lanes (raises on a HIP error)."""
        st = 0
        for c in self.ctxs:
            st |= c.check()
        return st

    def step(self, obj, probe, meas_sorted, grad):
        """grad <- sum over tiles of the embedded tile gradients; returns the per-tile loss tensor.

        obj: complex64 [S, H, W] (device); meas_sorted: float32 [n, M, M] in tile order.
        Enqueued on the lanes' streams; the caller's current stream waits for all of them.
        """
        import torch
        cur = torch.cuda.current_stream()
        B.ptycho_zero_gradient(self.ctx, grad)
        start = torch.cuda.Event()
        start.record(cur)
        for s in self.streams:
            s.wait_event(start)
        last_stitch = None
        for k, p in enumerate(self.plan.plans):
            if p.hi == p.lo:
                continue
            lane = k % self.lanes
            ey0, ex0, eh, ew = p.box
            tg, pos_k, _ = self.tile_views(k)
            s = self.streams[lane]
            with torch.cuda.stream(s):
                B.ptycho_tile_grad(self.ctxs[lane], obj[:, ey0:ey0 + eh, ex0:ex0 + ew], p.box, p.tile,
                                   self.plan.halo, self.plan.H, self.plan.W, probe, pos_k, meas_sorted[p.lo:p.hi],
                                   tile_grad=tg, loss=self.tile_loss[k:k + 1])
                if last_stitch is not None:
                    s.wait_event(last_stitch)
                B.ptycho_tile_accumulate(self.ctxs[lane], tg, p.box, grad)
                last_stitch = torch.cuda.Event()
                last_stitch.record(s)
        for s in self.streams:
            cur.wait_stream(s)
        return self.tile_loss


class StreamingTileWalk:
    """Decomposed gradient with object, measurements and the global gradient in pinned host memory.

    The device holds one extended object box, one tile of measurements and
    positions, one tile gradient and one gradient box at a time.  For every
    tile the global gradient's box is brought to the device, the tile gradient
    is added to it by the library's stitch kernel and the box is written back,
    so every addition happens on the GPU and the host only moves data.
    """

    def __init__(self, plan: TileWalk, ctx: B.Context, device="cuda:0"):
        import torch
        self.plan, self.ctx = plan, ctx
        S, M = ctx.S, ctx.M
        eh, ew = plan.max_box
        ctx.reserve(max(plan.max_count, 1))
        self.dev = {
            "obj": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
            "meas": torch.empty((max(plan.max_count, 1), M, M), dtype=torch.float32, device=device),
            "pos": torch.empty((max(plan.max_count, 1), 2), dtype=torch.int32, device=device),
            "tile": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
            "gbox": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
            "loss": torch.zeros(len(plan.plans), dtype=torch.float64, device=device),
        }
        self.pos_host = torch.tensor(plan.pos_sorted, dtype=torch.int32).pin_memory()

    def device_bytes(self) -> int:
        return sum(t.numel() * t.element_size() for t in self.dev.values())

    def step(self, obj_host, probe, meas_host_sorted, grad_host):
        """grad_host <- decomposed gradient (obj_host [S,H,W] complex64, meas_host [n,M,M] float32, pinned)."""
        S = self.ctx.S
        d = self.dev
        grad_host.zero_()
        for k, p in enumerate(self.plan.plans):
            if p.hi == p.lo:
                continue
            ey0, ex0, eh, ew = p.box
            n_k = p.hi - p.lo
            ob = d["obj"].view(-1)[: S * eh * ew].view(S, eh, ew)
            tg = d["tile"].view(-1)[: S * eh * ew].view(S, eh, ew)
            gb = d["gbox"].view(-1)[: S * eh * ew].view(S, eh, ew)
            ob.copy_(obj_host[:, ey0:ey0 + eh, ex0:ex0 + ew], non_blocking=True)
            d["meas"][:n_k].copy_(meas_host_sorted[p.lo:p.hi], non_blocking=True)
            d["pos"][:n_k].copy_(self.pos_host[p.lo:p.hi], non_blocking=True)
            B.ptycho_tile_grad(self.ctx, ob, p.box, p.tile, self.plan.halo, self.plan.H, self.plan.W, probe,
                               d["pos"][:n_k], d["meas"][:n_k], tile_grad=tg, loss=d["loss"][k:k + 1])
            gb.copy_(grad_host[:, ey0:ey0 + eh, ex0:ex0 + ew], non_blocking=True)
            B.ptycho_tile_accumulate(self.ctx, tg, (0, 0, eh, ew), gb)
            grad_host[:, ey0:ey0 + eh, ex0:ex0 + ew].copy_(gb)
        return d["loss"]
