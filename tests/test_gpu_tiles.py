"""GPU tile decomposition (Section III): per-tile gradients against the oracle,
the stitched sum against the undecomposed GPU gradient, and the device-side
halo / assignment checks."""
import numpy as np
import pytest

import oracle
import ptycho_synth as ps
from gpu_helpers import context, problem, rel_l2, say, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def tiled_spec():
    # 4 slices of 384^2, 2x2 tiles with a 64 px halo (= M/2), 18x18 raster with step 14
    return ps.with_overrides(ps.workload("ms16-2048-m128-tiles4x4"), W=384, S=4, ny=18, nx=18, tiles=(2, 2), halo=64)


def test_tile_gradients_match_oracle_and_sum_to_global(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import ResidentTileWalk, TileWalk
    spec = tiled_spec()
    say("tile walk 2x2 on 4 x 384^2, 324 positions")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    walk = ResidentTileWalk(ctx, plan)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    grad = torch.empty_like(t["obj"])
    losses = walk.step(t["obj"], t["probe"], meas_sorted, grad)
    assert walk.lanes == 2
    walk.check()
    gfull = torch.empty_like(grad)
    lfull, _ = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], grad=gfull)
    ctx.check()
    torch.cuda.synchronize()
    dec = rel_l2(grad.cpu().numpy(), gfull.cpu().numpy())
    say(f"  decomposed vs undecomposed rel L2 = {dec:.3e}")
    assert dec <= 1e-6
    assert abs(float(losses.sum()) - float(lfull.item())) <= 1e-9 * float(lfull.item())
    G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
    assert rel_l2(grad.cpu().numpy(), G_ref) <= 1e-4
    # every tile gradient against the oracle's tile gradient
    for k, p in enumerate(plan.plans):
        ty, tx = divmod(k, spec.tiles[1])
        ref = oracle.tile_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"], spec.tiles, spec.halo,
                                   ty, tx)
        ey0, ex0, eh, ew = p.box
        assert ref["box"] == (ey0, ey0 + eh, ex0, ex0 + ew)
        tg = torch.empty((spec.S, eh, ew), dtype=torch.complex64, device="cuda:0")
        loss_k, _ = pt.ptycho_tile_grad(ctx, t["obj"][:, ey0:ey0 + eh, ex0:ex0 + ew], p.box, p.tile, spec.halo,
                                        spec.W, spec.W, t["probe"], walk.pos[p.lo:p.hi], meas_sorted[p.lo:p.hi],
                                        tile_grad=tg)
        ctx.check()
        assert rel_l2(tg.cpu().numpy(), ref["grad"]) <= 1e-4
        assert abs(float(loss_k.item()) - ref["loss"]) <= 1e-5 * ref["loss"]


def test_tile_halo_and_assignment_checks(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    spec = tiled_spec()
    say("device-side halo and assignment checks of the tile gradient")
    d = problem(spec)
    t = to_dev(d)
    ctx = context(spec, spec.n)
    owner = pt.bin_positions(d["pos"], spec.W, spec.W, spec.M, 2, 2)
    # tile (1,1) with its own positions but a halo of 32 < M/2: some windows leave the box
    (ty0, ty1, tx0, tx1), (ey0, ey1, ex0, ex1) = pt.tile_box(spec.W, spec.W, 2, 2, 1, 1, 32)
    mine = np.nonzero(owner == 3)[0]
    pos_k = torch.tensor(d["pos"][mine], dtype=torch.int32, device="cuda:0")
    meas_k = t["meas"][torch.tensor(mine, device="cuda:0")].contiguous()
    box = (ey0, ex0, ey1 - ey0, ex1 - ex0)
    pt.ptycho_tile_grad(ctx, t["obj"][:, ey0:ey1, ex0:ex1], box, (ty0, ty1, tx0, tx1), 32, spec.W, spec.W,
                        t["probe"], pos_k, meas_k)
    with pytest.raises(pt.PtychoError) as e:
        ctx.check()
    assert e.value.name == "PTYCHO_E_HALO"
    # positions of tile 0 handed to tile 3 with a full halo: centres outside the tile
    (ty0, ty1, tx0, tx1), (ey0, ey1, ex0, ex1) = pt.tile_box(spec.W, spec.W, 2, 2, 1, 1, 192)
    other = np.nonzero(owner == 0)[0][-4:]
    pos_o = torch.tensor(d["pos"][other], dtype=torch.int32, device="cuda:0")
    meas_o = t["meas"][torch.tensor(other, device="cuda:0")].contiguous()
    box = (ey0, ex0, ey1 - ey0, ex1 - ex0)
    pt.ptycho_tile_grad(ctx, t["obj"][:, ey0:ey1, ex0:ex1], box, (ty0, ty1, tx0, tx1), 192, spec.W, spec.W,
                        t["probe"], pos_o, meas_o)
    with pytest.raises(pt.PtychoError) as e:
        ctx.check()
    assert e.value.name == "PTYCHO_E_ASSIGN"
    # a box that is not the tile grown by the halo is rejected on the host
    with pytest.raises(pt.PtychoError) as e:
        pt.ptycho_tile_grad(ctx, t["obj"][:, 0:200, 0:200], (0, 0, 200, 200), (0, 192, 0, 192), 64, spec.W,
                            spec.W, t["probe"], pos_o, meas_o)
    assert e.value.name == "PTYCHO_E_SHAPE"


def test_streaming_walk_matches_resident(torch_cuda):
    import torch
    from paper_2205_06327_amd.tilewalk import ResidentTileWalk, StreamingTileWalk, TileWalk
    spec = tiled_spec()
    say("streaming tile walk (pinned host inputs) vs resident walk")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    order = torch.tensor(plan.order, device="cuda:0")
    meas_sorted = t["meas"][order].contiguous()
    grad = torch.empty_like(t["obj"])
    ResidentTileWalk(ctx, plan).step(t["obj"], t["probe"], meas_sorted, grad)
    sw = StreamingTileWalk(plan, ctx)
    gh = torch.empty(tuple(grad.shape), dtype=torch.complex64).pin_memory()
    sw.step(t["obj"].cpu().pin_memory(), t["probe"], meas_sorted.cpu().pin_memory(), gh)
    torch.cuda.synchronize()
    ctx.check()
    assert rel_l2(gh.numpy(), grad.cpu().numpy()) <= 1e-6
    # a tile without positions: its box still gets written (zero plus its neighbours' overlaps), so a
    # host gradient full of garbage from before comes out right
    keep = np.array([plan.plans[0].hi <= i for i in range(spec.n)])  # drop tile 0's positions
    plan2 = TileWalk(plan.pos_sorted[keep], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    assert plan2.plans[0].hi == plan2.plans[0].lo
    meas2 = meas_sorted[torch.tensor(np.nonzero(keep)[0], device="cuda:0")][torch.tensor(plan2.order, device="cuda:0")]
    grad2 = torch.empty_like(t["obj"])
    ResidentTileWalk(ctx, plan2).step(t["obj"], t["probe"], meas2.contiguous(), grad2)
    gh.fill_(float("nan"))
    StreamingTileWalk(plan2, ctx).step(t["obj"].cpu().pin_memory(), t["probe"], meas2.cpu().pin_memory(), gh)
    torch.cuda.synchronize()
    assert ctx.check() == 0
    assert not torch.isnan(gh).any()
    assert rel_l2(gh.numpy(), grad2.cpu().numpy()) <= 1e-6


def test_lane_count_does_not_change_the_walk(torch_cuda):
    import torch
    from paper_2205_06327_amd.tilewalk import ResidentTileWalk, TileWalk
    spec = tiled_spec()
    say("resident walk with 1, 2 and 3 lanes (overlapping tile launches)")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    order = torch.tensor(plan.order, device="cuda:0")
    meas_sorted = t["meas"][order].contiguous()
    out = []
    for lanes in (1, 2, 3):
        walk = ResidentTileWalk(ctx, plan, lanes=lanes)
        grad = torch.empty_like(t["obj"])
        for _ in range(2):  # the second step reuses every lane's buffers
            loss = walk.step(t["obj"], t["probe"], meas_sorted, grad)
        assert walk.check() == 0
        torch.cuda.synchronize()
        out.append((grad.cpu().numpy(), float(loss.sum())))
    for g, l in out[1:]:
        assert rel_l2(g, out[0][0]) <= 1e-6
        assert abs(l - out[0][1]) <= 1e-9 * abs(out[0][1])


def test_decomposed_walk_directional_passes(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import DecomposedTileWalk, TileWalk
    spec = ps.with_overrides(tiled_spec(), tiles=(4, 4))  # 96 px tiles, 64 px halo: tiles two apart overlap
    say("per-tile buffers + directional passes, 4x4 tiles of 96 px with a 64 px halo")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    walk = DecomposedTileWalk(ctx, plan)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    gfull = torch.empty_like(t["obj"])
    lfull, _ = pt.ptycho_loss_grad(ctx, t["obj"], t["probe"], t["pos"], t["meas"], grad=gfull)
    G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
    g_h = gfull.cpu().numpy()
    # tile gradients alone: some box misses other tiles' contributions
    walk.tile_gradients(t["obj"], t["probe"], meas_sorted)
    assert walk.check() == 0
    torch.cuda.synchronize()
    before = [rel_l2(walk.bufs[k].cpu().numpy(), g_h[:, p.box[0]:p.box[0] + p.box[2], p.box[1]:p.box[1] + p.box[3]])
              for k, p in enumerate(plan.plans)]
    assert max(before) > 1e-2
    losses = walk.step(t["obj"], t["probe"], meas_sorted)
    assert walk.check() == 0
    torch.cuda.synchronize()
    assert abs(float(losses.sum()) - float(lfull.item())) <= 1e-9 * float(lfull.item())
    for k, p in enumerate(plan.plans):
        ey0, ex0, eh, ew = p.box
        buf = walk.bufs[k].cpu().numpy()
        assert rel_l2(buf, g_h[:, ey0:ey0 + eh, ex0:ex0 + ew]) <= 1e-6, k
        assert rel_l2(buf, G_ref[:, ey0:ey0 + eh, ex0:ex0 + ew]) <= 1e-4, k
    stitched = torch.zeros_like(gfull)
    walk.stitch(stitched)
    torch.cuda.synchronize()
    assert rel_l2(stitched.cpu().numpy(), g_h) <= 1e-6


@pytest.mark.parametrize("tiles", [(2, 2), (4, 4)])
def test_direct_neighbour_add(torch_cuda, tiles):
    """Section III's single exchange on the GPU against the oracle's: with 2x2 tiles of 192 px
    (>= 2 halo) every box then holds the undecomposed gradient; with 4x4 tiles of 96 px it misses
    the tiles two apart, exactly as the oracle's exchange does."""
    import torch
    from paper_2205_06327_amd.tilewalk import DecomposedTileWalk, TileWalk
    spec = ps.with_overrides(tiled_spec(), tiles=tiles)
    say(f"direct neighbour add, {tiles[0]}x{tiles[1]} tiles, halo {spec.halo}")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    walk = DecomposedTileWalk(ctx, plan)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    walk.tile_gradients(t["obj"], t["probe"], meas_sorted)
    acc = walk.neighbour_add()
    assert walk.check() == 0
    torch.cuda.synchronize()
    ref_tiles = [oracle.tile_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"], spec.tiles,
                                      spec.halo, *divmod(k, spec.tiles[1])) for k in range(len(plan.plans))]
    ref = oracle.neighbour_add(ref_tiles, spec.tiles)
    G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
    exact = min(p.tile[1] - p.tile[0] for p in plan.plans) >= 2 * spec.halo
    for k, p in enumerate(plan.plans):
        ey0, ex0, eh, ew = p.box
        buf = acc[k].cpu().numpy()
        assert rel_l2(buf, ref[k]["grad"]) <= 1e-4, k
        assert rel_l2(walk.bufs[k].cpu().numpy(), ref_tiles[k]["grad"]) <= 1e-4, k  # sources untouched
        if exact:
            assert rel_l2(buf, G_ref[:, ey0:ey0 + eh, ex0:ex0 + ew]) <= 1e-4, k
    if not exact:
        worst = max(rel_l2(acc[k].cpu().numpy(), G_ref[:, p.box[0]:p.box[0] + p.box[2], p.box[1]:p.box[1] + p.box[3]])
                    for k, p in enumerate(plan.plans))
        assert worst > 1e-2


@pytest.mark.parametrize("batch,T", [(4, 1), (4, 3)])
def test_alg1_walk_matches_oracle(torch_cuda, batch, T):
    import torch
    from paper_2205_06327_amd.tilewalk import Alg1Walk, TileWalk
    spec = ps.with_overrides(ps.workload("2d-256-m64"), W=192, S=2, ny=17, nx=17, step=8, tiles=(4, 4), halo=32)
    say(f"Alg. 1 walk, 4x4 tiles of 48 px, halo 32, batch {batch}, T {T}, 2 iterations")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    alpha = 0.5 * oracle.gd_step_size(d["probe"], d["pos"], spec.W, spec.W, spec.S)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    walk = Alg1Walk(ctx, plan, t["obj"], t["probe"], meas_sorted, alpha, batch, T)
    losses = [float(walk.iteration().item()) for _ in range(2)]
    assert walk.check() == 0
    V = torch.empty_like(t["obj"])
    walk.stitch(V)
    torch.cuda.synchronize()
    ref_l, ref_V = oracle.alg1_tiles(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"], spec.tiles, spec.halo,
                                     alpha, batch, T, 2)
    np.testing.assert_allclose(losses, ref_l, rtol=1e-4)
    assert losses[1] < losses[0]
    # the update V - V0 is small next to V (|t| ~ 1): every FP32 write of V_k rounds by up to
    # 2^-24 |V|, so the update's relative error is bounded by 1e-4 plus the number of writes per
    # pixel (a step per batch and per flush, two iterations) times 2^-24 ||V0|| / ||V - V0||
    V0 = d["obj_eval"].astype(np.complex128)
    dV = ref_V - V0
    writes = 2 * (walk.steps + -(-walk.steps // T))
    tol = 1e-4 + writes * 2.0 ** -24 * np.linalg.norm(V0) / np.linalg.norm(dV)
    assert rel_l2(V.cpu().numpy() - V0, dV) <= tol


def test_all_tiles_in_one_launch(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import AllTilesWalk, ResidentTileWalk, TileWalk
    spec = ps.with_overrides(tiled_spec(), tiles=(3, 3))
    say("all tiles' gradients in one launch vs the tile-by-tile walk and the oracle")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    g_all = torch.empty_like(t["obj"])
    g_lanes = torch.empty_like(t["obj"])
    walk = AllTilesWalk(ctx, plan)
    for _ in range(2):
        l_all = float(walk.step(t["obj"], t["probe"], meas_sorted, g_all).item())
    assert walk.check() == 0
    l_lanes = float(ResidentTileWalk(ctx, plan).step(t["obj"], t["probe"], meas_sorted, g_lanes).sum())
    torch.cuda.synchronize()
    assert rel_l2(g_all.cpu().numpy(), g_lanes.cpu().numpy()) <= 1e-6
    assert abs(l_all - l_lanes) <= 1e-9 * l_lanes
    G_ref = oracle.loss_and_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"])[2]
    assert rel_l2(g_all.cpu().numpy(), G_ref) <= 1e-4
    for k, p in enumerate(plan.plans):  # each tile buffer against the oracle's tile gradient
        ty, tx = divmod(k, spec.tiles[1])
        ref = oracle.tile_gradient(d["obj_eval"], d["probe"], d["pos"], d["meas"], d["H"], spec.tiles, spec.halo,
                                   ty, tx)
        assert rel_l2(walk.bufs[k].cpu().numpy(), ref["grad"]) <= 1e-4, k
    # a position given to the wrong tile is skipped and reported on the device
    bad = walk.tile_of_pos.clone()
    bad[0] = (int(bad[0]) + 4) % 9
    pt.ptycho_tiles_grad(ctx, t["obj"], walk.tiles, spec.halo, bad, t["probe"], walk.pos, meas_sorted)
    with pytest.raises(pt.PtychoError) as e:
        ctx.check()
    assert e.value.name == "PTYCHO_E_ASSIGN"
    assert ctx.check() == 0  # reading the status clears it


def test_tiles_grad_host_validation(torch_cuda):
    import torch
    import paper_2205_06327_amd as pt
    from paper_2205_06327_amd.tilewalk import AllTilesWalk, TileWalk
    spec = ps.with_overrides(tiled_spec(), tiles=(2, 2))
    say("ptycho_tiles_grad rejects bad tile tables on the host")
    d = problem(spec)
    t = to_dev(d)
    plan = TileWalk(d["pos"], spec.W, spec.W, spec.M, spec.tiles, spec.halo)
    ctx = context(spec, spec.n)
    walk = AllTilesWalk(ctx, plan)
    meas_sorted = t["meas"][torch.tensor(plan.order, device="cuda:0")].contiguous()
    (tile, box, g) = walk.tiles[0]
    bad_box = [((tile), (box[0], box[1], box[2] - 1, box[3]), g[:, :-1, :].contiguous())] + walk.tiles[1:]
    with pytest.raises(pt.PtychoError) as e:
        pt.ptycho_tiles_grad(ctx, t["obj"], bad_box, spec.halo, walk.tile_of_pos, t["probe"], walk.pos, meas_sorted)
    assert e.value.name == "PTYCHO_E_SHAPE"
    with pytest.raises(pt.PtychoError) as e:
        pt.ptycho_tiles_grad(ctx, t["obj"], [], spec.halo, walk.tile_of_pos, t["probe"], walk.pos, meas_sorted)
    assert e.value.name == "PTYCHO_E_ARG"
    outside = [((0, spec.W + 1, 0, 10), box, g)] + walk.tiles[1:]
    with pytest.raises(pt.PtychoError) as e:
        pt.ptycho_tiles_grad(ctx, t["obj"], outside, spec.halo, walk.tile_of_pos, t["probe"], walk.pos, meas_sorted)
    assert e.value.name == "PTYCHO_E_SHAPE"
    assert ctx.check() == 0  # nothing was enqueued
