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
            if c.checkpoint != ctx.checkpoint:
                c.set_checkpoint(ctx.checkpoint)
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


class AllTilesWalk:
    """Every tile's gradient in one persistent launch (ptycho_tiles_grad), then the stitch.

    The same decomposition as ResidentTileWalk -- each position adds into the
    gradient buffer of the tile that owns it, on that tile's extended box --
    but the tiles' launches become one, as a mesh of devices would run them
    side by side: no tail per tile and one launch to time.  It holds every
    tile's buffer (the sum of the extended boxes).
    """

    def __init__(self, ctx: B.Context, plan: TileWalk, device="cuda:0"):
        import torch
        self.ctx, self.plan = ctx, plan
        S = ctx.S
        ctx.reserve(max(plan.n, 1))
        self.pos = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=device)
        owner = np.empty(plan.n, dtype=np.int32)
        for p in plan.plans:
            owner[p.lo:p.hi] = p.index
        self.tile_of_pos = torch.tensor(owner, dtype=torch.int32, device=device)
        self.bufs = [torch.empty((S, p.box[2], p.box[3]), dtype=torch.complex64, device=device) for p in plan.plans]
        self.tiles = [(p.tile, p.box, self.bufs[k]) for k, p in enumerate(plan.plans)]
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)

    @property
    def lanes(self) -> int:
        return 1

    def device_bytes(self) -> int:
        """Tile buffers, positions and tile indices plus the context's workspace."""
        return sum(b.numel() * b.element_size() for b in self.bufs) + self.pos.numel() * 4 + \
            self.tile_of_pos.numel() * 4 + self.ctx.workspace_bytes()

    def profile(self, enable: bool = True) -> None:
        self.ctx.profile(enable)

    def profile_read(self):
        return self.ctx.profile_read()

    def check(self) -> int:
        return self.ctx.check()

    def step(self, obj, probe, meas_sorted, grad, loss_per_pos=None):
        """grad <- sum of the embedded tile gradients; returns the total loss (float64 [1]).
        loss_per_pos: optional float64 [n] device tensor receiving f_i in tile order."""
        B.ptycho_zero_gradient(self.ctx, grad)
        B.ptycho_tiles_grad(self.ctx, obj, self.tiles, self.plan.halo, self.tile_of_pos, probe, self.pos,
                            meas_sorted, loss=self.loss, loss_per_pos=loss_per_pos)
        for k, p in enumerate(self.plan.plans):
            B.ptycho_tile_accumulate(self.ctx, self.bufs[k], p.box, grad)
        return self.loss


class StreamingTileWalk:
    """Decomposed gradient with object, measurements and the global gradient in pinned host memory.

    The device holds, per lane, one extended object box, one tile of
    measurements and positions, one tile gradient and one gradient box.  For
    every tile the extended object box and the tile's measurements are copied
    in (pitched copies, ptycho_copy_box), the tile gradient is computed, the
    global gradient's box is assembled on the device (zero, plus its overlaps
    with the boxes already written back, the only parts of the global
    gradient that are not zero yet), the tile gradient is added by the
    library's stitch kernel and the box is written back, so every addition
    happens on the GPU and the host only moves data.  Tiles alternate between
    two lanes (context + stream + buffers), so one tile's transfers overlap the
    other lane's kernel; the gradient boxes of consecutive tiles overlap in the
    halos, so each tile's read of the global gradient waits for the previous
    tile's write-back.
    """

    def __init__(self, plan: TileWalk, ctx: B.Context, device="cuda:0", lanes: int = 2):
        import torch
        self.plan, self.ctx = plan, ctx
        S, M = ctx.S, ctx.M
        eh, ew = plan.max_box
        lanes = max(1, int(lanes))
        cap = max(plan.max_count, 1)
        self.ctxs = [ctx] + [B.Context(ctx.M, ctx.S, *ctx.physics, max_positions=cap) for _ in range(lanes - 1)]
        for c in self.ctxs:
            c.reserve(cap)
            if c.checkpoint != ctx.checkpoint:
                c.set_checkpoint(ctx.checkpoint)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.dev = []
        for _ in range(lanes):
            self.dev.append({
                "obj": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
                "meas": torch.empty((cap, M, M), dtype=torch.float32, device=device),
                "pos": torch.empty((cap, 2), dtype=torch.int32, device=device),
                "tile": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
                "gbox": torch.empty((S, eh, ew), dtype=torch.complex64, device=device),
            })
        self.loss = torch.zeros(len(plan.plans), dtype=torch.float64, device=device)
        self.pos_host = torch.tensor(plan.pos_sorted, dtype=torch.int32).pin_memory()

    def device_bytes(self) -> int:
        """The lanes' buffers plus every lane context's workspace (the walk's whole device memory)."""
        return sum(t.numel() * t.element_size() for d in self.dev for t in d.values()) + \
            self.loss.numel() * self.loss.element_size() + sum(c.workspace_bytes() for c in self.ctxs)

    def check(self) -> int:
        st = 0
        for c in self.ctxs:
            st |= c.check()
        return st

    def step(self, obj_host, probe, meas_host_sorted, grad_host):
        """grad_host <- decomposed gradient (obj_host [S,H,W] complex64, meas_host [n,M,M] float32, pinned)."""
        import torch
        S = self.ctx.S
        for s in self.streams:  # the previous step's write-backs into grad_host have landed
            s.synchronize()
        cur = torch.cuda.current_stream()
        start = torch.cuda.Event()
        start.record(cur)
        for s in self.streams:
            s.wait_event(start)
        written = None  # event after the previous tile's write-back of the global gradient
        for k, p in enumerate(self.plan.plans):
            lane = k % len(self.ctxs)
            c, d, s = self.ctxs[lane], self.dev[lane], self.streams[lane]
            ey0, ex0, eh, ew = p.box
            n_k = p.hi - p.lo
            ob = d["obj"].view(-1)[: S * eh * ew].view(S, eh, ew)
            tg = d["tile"].view(-1)[: S * eh * ew].view(S, eh, ew)
            gb = d["gbox"].view(-1)[: S * eh * ew].view(S, eh, ew)
            with torch.cuda.stream(s):
                if n_k > 0:
                    B.ptycho_copy_box(c, obj_host[:, ey0:ey0 + eh, ex0:ex0 + ew], ob)
                    d["meas"][:n_k].copy_(meas_host_sorted[p.lo:p.hi], non_blocking=True)
                    d["pos"][:n_k].copy_(self.pos_host[p.lo:p.hi], non_blocking=True)
                    B.ptycho_tile_grad(c, ob, p.box, p.tile, self.plan.halo, self.plan.H, self.plan.W, probe,
                                       d["pos"][:n_k], d["meas"][:n_k], tile_grad=tg, loss=self.loss[k:k + 1])
                else:
                    self.loss[k:k + 1].zero_()
                if written is not None:
                    s.wait_event(written)
                # Only the boxes written back so far hold this step's global gradient (the boxes cover
                # the object and every tile writes its box back, so nothing else is ever read): the
                # box is cleared on the device and only its overlaps with those boxes come in.
                B.ptycho_zero_gradient(c, gb)
                for j in range(k):
                    q = self.plan.plans[j]
                    y0, x0 = max(ey0, q.box[0]), max(ex0, q.box[1])
                    y1, x1 = min(ey0 + eh, q.box[0] + q.box[2]), min(ex0 + ew, q.box[1] + q.box[3])
                    if y0 < y1 and x0 < x1:
                        B.ptycho_copy_box(c, grad_host[:, y0:y1, x0:x1], gb[:, y0 - ey0:y1 - ey0, x0 - ex0:x1 - ex0])
                if n_k > 0:
                    B.ptycho_tile_accumulate(c, tg, (0, 0, eh, ew), gb)
                B.ptycho_copy_box(c, gb, grad_host[:, ey0:ey0 + eh, ex0:ex0 + ew])
                written = torch.cuda.Event()
                written.record(s)
        for s in self.streams:
            cur.wait_stream(s)
        return self.loss


def directional_passes(ctx: B.Context, plan: TileWalk, bufs) -> None:
    """Section IV's passes between per-tile buffers (bufs[k] holds tile k's extended box), enqueued
    on the caller's current stream: down every tile column add, up every column replace, along
    every tile row add, back along every row replace."""
    ty_n, tx_n = plan.tiles

    def exchange(src: int, dst: int, replace: bool) -> None:
        a, b = plan.plans[src].box, plan.plans[dst].box
        B.ptycho_box_exchange(ctx, bufs[src], (a[0], a[1]), bufs[dst], (b[0], b[1]), replace)

    for tx in range(tx_n):
        for ty in range(ty_n - 1):
            exchange(ty * tx_n + tx, (ty + 1) * tx_n + tx, replace=False)
    for tx in range(tx_n):
        for ty in range(ty_n - 1, 0, -1):
            exchange(ty * tx_n + tx, (ty - 1) * tx_n + tx, replace=True)
    for ty in range(ty_n):
        for tx in range(tx_n - 1):
            exchange(ty * tx_n + tx, ty * tx_n + tx + 1, replace=False)
    for ty in range(ty_n):
        for tx in range(tx_n - 1, 0, -1):
            exchange(ty * tx_n + tx, ty * tx_n + tx - 1, replace=True)


def neighbour_add(ctx: B.Context, plan: TileWalk, src, dst) -> None:
    """Section III's single exchange: dst[k] = src[k] plus, on the overlaps, the original gradients
    src[j] of tile k's (up to) eight direct neighbours; src and dst are separate per-tile buffers on
    the extended boxes.  It sums every contribution to tile k's box only when tiles two apart do
    not overlap (tile >= 2 halo); the directional passes cover the general case."""
    ty_n, tx_n = plan.tiles
    for k, p in enumerate(plan.plans):
        ty, tx = divmod(k, tx_n)
        origin = (p.box[0], p.box[1])
        B.ptycho_box_exchange(ctx, src[k], origin, dst[k], origin, replace=True)
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                if (dy, dx) == (0, 0) or not (0 <= ty + dy < ty_n and 0 <= tx + dx < tx_n):
                    continue
                q = plan.plans[(ty + dy) * tx_n + tx + dx]
                B.ptycho_box_exchange(ctx, src[q.index], (q.box[0], q.box[1]), dst[k], origin, replace=False)


def stitch_interiors(ctx: B.Context, plan: TileWalk, bufs, out) -> None:
    """out[:, tile] = interior of bufs[k] for every tile k (Alg. 1's final stitch)."""
    for k, p in enumerate(plan.plans):
        ty0, ty1, tx0, tx1 = p.tile
        ey0, ex0, _, _ = p.box
        inner = bufs[k][:, ty0 - ey0:ty1 - ey0, tx0 - ex0:tx1 - ex0]
        B.ptycho_box_exchange(ctx, inner, (ty0, tx0), out, (0, 0), replace=True)


class DecomposedTileWalk:
    """The decomposition's per-device data flow on one GPU (Section IV, Alg. 1).

    Every tile keeps its own accumulated-gradient buffer on its extended box,
    as each device of the paper's mesh does.  ``step`` computes every tile's
    gradient into its buffer (tile launches alternate between two lanes, as in
    the resident walk), then ``passes`` runs the four directional passes as
    exchanges between the buffers (``ptycho_box_exchange``): down each tile
    column add, up each column replace, along each tile row add, back along
    each row replace.  Afterwards every buffer holds the summed gradient of all
    tiles on its box -- what each device needs for its own update -- also
    where tiles two apart overlap (tile < 2 halo), which a single exchange with
    the direct neighbours does not cover.  ``stitch`` copies the tiles'
    interiors into one array (the final stitch of Alg. 1).  The buffers take
    the sum of all extended boxes, the memory of the whole device mesh.
    """

    def __init__(self, ctx: B.Context, plan: TileWalk, device="cuda:0", lanes: int = 2):
        import torch
        self.ctx, self.plan = ctx, plan
        S = ctx.S
        lanes = max(1, int(lanes))
        self.ctxs = [ctx] + [B.Context(ctx.M, ctx.S, *ctx.physics, max_positions=max(plan.max_count, 1))
                             for _ in range(lanes - 1)]
        for c in self.ctxs:
            c.reserve(max(plan.max_count, 1))
            if c.checkpoint != ctx.checkpoint:
                c.set_checkpoint(ctx.checkpoint)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.pos = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=device)
        self.bufs = [torch.empty((S, p.box[2], p.box[3]), dtype=torch.complex64, device=device)
                     for p in plan.plans]
        self.tile_loss = torch.zeros(len(plan.plans), dtype=torch.float64, device=device)

    def device_bytes(self) -> int:
        """The per-tile buffers plus every lane context's workspace."""
        return sum(b.numel() * b.element_size() for b in self.bufs) + sum(c.workspace_bytes() for c in self.ctxs)

    def check(self) -> int:
        st = 0
        for c in self.ctxs:
            st |= c.check()
        return st

    def tile_gradients(self, obj, probe, meas_sorted):
        """Every tile's own gradient into its buffer (no exchange yet); returns the per-tile losses."""
        import torch
        cur = torch.cuda.current_stream()
        start = torch.cuda.Event()
        start.record(cur)
        for s in self.streams:
            s.wait_event(start)
        for k, p in enumerate(self.plan.plans):
            lane = k % len(self.ctxs)
            ey0, ex0, eh, ew = p.box
            with torch.cuda.stream(self.streams[lane]):
                B.ptycho_tile_grad(self.ctxs[lane], obj[:, ey0:ey0 + eh, ex0:ex0 + ew], p.box, p.tile,
                                   self.plan.halo, self.plan.H, self.plan.W, probe, self.pos[p.lo:p.hi],
                                   meas_sorted[p.lo:p.hi], tile_grad=self.bufs[k], loss=self.tile_loss[k:k + 1])
        for s in self.streams:
            cur.wait_stream(s)
        return self.tile_loss

    def passes(self) -> None:
        """Vertical forward (add) and backward (replace), then horizontal forward and backward."""
        directional_passes(self.ctx, self.plan, self.bufs)

    def neighbour_add(self):
        """Section III's direct exchange of the tile gradients in ``bufs`` into a second set of
        buffers (allocated on first use), which it returns; ``bufs`` keep the tiles' own gradients."""
        import torch
        if getattr(self, "acc", None) is None:
            self.acc = [torch.empty_like(b) for b in self.bufs]
        neighbour_add(self.ctx, self.plan, self.bufs, self.acc)
        return self.acc

    def pass_bytes(self) -> int:
        """HBM bytes the passes move: overlap x S x 8 B, read twice and written once per add, read and
        written once per replace."""
        ty_n, tx_n = self.plan.tiles
        S = self.ctx.S
        total = 0

        def ov(i, j):
            a, b = self.plan.plans[i].box, self.plan.plans[j].box
            h = min(a[0] + a[2], b[0] + b[2]) - max(a[0], b[0])
            w = min(a[1] + a[3], b[1] + b[3]) - max(a[1], b[1])
            return max(h, 0) * max(w, 0)
        for tx in range(tx_n):
            for ty in range(ty_n - 1):
                total += 3 * ov(ty * tx_n + tx, (ty + 1) * tx_n + tx) + 2 * ov((ty + 1) * tx_n + tx, ty * tx_n + tx)
        for ty in range(ty_n):
            for tx in range(tx_n - 1):
                total += 3 * ov(ty * tx_n + tx, ty * tx_n + tx + 1) + 2 * ov(ty * tx_n + tx + 1, ty * tx_n + tx)
        return total * S * 8

    def step(self, obj, probe, meas_sorted):
        """Tile gradients, then the passes; returns the per-tile losses."""
        loss = self.tile_gradients(obj, probe, meas_sorted)
        self.passes()
        return loss

    def stitch(self, out) -> None:
        """out[:, tile] = buffer interior, for every tile (out: complex64 [S, H, W])."""
        stitch_interiors(self.ctx, self.plan, self.bufs, out)


class Alg1Walk:
    """Alg. 1 on one device: one tile per (virtual) device, mini-batch reading.

    Every tile keeps its own extended copy V_k of the object and an
    accumulation buffer AccBuf_k.  An iteration walks every tile's positions
    in scan order, ``batch`` at a time: the batch's gradient at V_k
    (ptycho_tile_grad) is added to AccBuf_k and V_k takes
    V_k -= step * gradient (ptycho_box_axpy).  After every ``T`` batches and
    after an iteration's last batch, the directional passes run on the
    buffers, every tile takes V_k -= step * AccBuf_k, and the buffers are
    cleared.  With batch = 1 this is the per-probe loop of Alg. 1; a batch of a
    few hundred positions per tile keeps the GPU busy.  Tiles' launches
    alternate between two lanes (contexts and streams); the passes and the
    accumulated update run on the caller's stream after both lanes.
    """

    def __init__(self, ctx: B.Context, plan: TileWalk, obj, probe, meas_sorted, step: float, batch: int, T: int,
                 device="cuda:0", lanes: int = 2):
        import torch
        self.ctx, self.plan = ctx, plan
        self.probe, self.meas = probe, meas_sorted
        self.step_size, self.batch, self.T = float(step), max(1, int(batch)), max(1, int(T))
        S = ctx.S
        lanes = max(1, int(lanes))
        self.ctxs = [ctx] + [B.Context(ctx.M, ctx.S, *ctx.physics, max_positions=self.batch)
                             for _ in range(lanes - 1)]
        for c in self.ctxs:
            c.reserve(self.batch)
            if c.checkpoint != ctx.checkpoint:
                c.set_checkpoint(ctx.checkpoint)
        self.streams = [torch.cuda.Stream(device=device) for _ in range(lanes)]
        self.pos = torch.tensor(plan.pos_sorted, dtype=torch.int32, device=device)
        self.V = []
        for p in plan.plans:
            ey0, ex0, eh, ew = p.box
            self.V.append(obj[:, ey0:ey0 + eh, ex0:ex0 + ew].contiguous())
        self.acc = [torch.zeros_like(v) for v in self.V]
        eh, ew = plan.max_box
        self.gbuf = [torch.empty((S, eh, ew), dtype=torch.complex64, device=device) for _ in range(lanes)]
        counts = [p.hi - p.lo for p in plan.plans]
        self.steps = max((c + self.batch - 1) // self.batch for c in counts) if counts else 0
        self.losses = torch.zeros((max(self.steps, 1), len(plan.plans)), dtype=torch.float64, device=device)

    def check(self) -> int:
        st = 0
        for c in self.ctxs:
            st |= c.check()
        return st

    def _flush(self) -> None:
        directional_passes(self.ctx, self.plan, self.acc)
        for k, p in enumerate(self.plan.plans):
            o = (p.box[0], p.box[1])
            B.ptycho_box_axpy(self.ctx, -self.step_size, self.acc[k], o, self.V[k], o)
            B.ptycho_zero_gradient(self.ctx, self.acc[k])

    def iteration(self):
        """One pass over every tile's positions; returns the iteration's loss (device float64 [1])."""
        import torch
        cur = torch.cuda.current_stream()
        self.losses.zero_()
        n_lanes = len(self.ctxs)
        for j in range(self.steps):
            ev = torch.cuda.Event()
            ev.record(cur)
            for s in self.streams:
                s.wait_event(ev)
            slot = 0
            for k, p in enumerate(self.plan.plans):
                lo = p.lo + j * self.batch
                hi = min(p.hi, lo + self.batch)
                if hi <= lo:
                    continue
                lane = slot % n_lanes
                slot += 1
                ey0, ex0, eh, ew = p.box
                g = self.gbuf[lane].view(-1)[: self.ctx.S * eh * ew].view(self.ctx.S, eh, ew)
                with torch.cuda.stream(self.streams[lane]):
                    B.ptycho_tile_grad(self.ctxs[lane], self.V[k], p.box, p.tile, self.plan.halo, self.plan.H,
                                       self.plan.W, self.probe, self.pos[lo:hi], self.meas[lo:hi], tile_grad=g,
                                       loss=self.losses[j, k:k + 1])
                    B.ptycho_box_axpy(self.ctxs[lane], 1.0, g, (ey0, ex0), self.acc[k], (ey0, ex0))
                    B.ptycho_box_axpy(self.ctxs[lane], -self.step_size, g, (ey0, ex0), self.V[k], (ey0, ex0))
            for s in self.streams:
                cur.wait_stream(s)
            if (j + 1) % self.T == 0 or j == self.steps - 1:
                self._flush()
        return self.losses.sum().reshape(1)

    def stitch(self, out) -> None:
        """out[:, tile] = interior of V_k for every tile: the reconstruction."""
        stitch_interiors(self.ctx, self.plan, self.V, out)
